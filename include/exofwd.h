/*
 * exofwd -- batched atmospheric forward model and its adjoint on MI355X (gfx950).
 *
 * C ABI of the library.  One call evaluates, for B parameter samples at once,
 * the retrieval forward model of Lee (2026, "Exo Skryer"):
 *   - the temperature-pressure profile (isothermal, Eq. 7; reduced modified
 *     Guillot, Eq. 16; or PCHIP knots) on log-uniform pressure levels,
 *   - free chemistry with H2/He filling (Eq. 35-36),
 *   - the hydrostatic altitude grid about the reference radius and pressure
 *     (inverse-square gravity, layer-isothermal),
 *   - per-layer opacity from (T, log p)-interpolated log cross-section tables
 *     weighted by mixing ratio, plus CIA, Rayleigh and a grey cloud deck
 *     (Section "Gas phase opacities"; Eq. 18 and 23 with Q_ext = 2),
 *   - transmission: the slant optical depth through the path matrix
 *     tau = P_1D . dtau_vert (Eq. 43-44) and the transit depth;
 *     emission: linear-in-tau upward intensity over Gauss-Legendre angles and
 *     the planet/star flux ratio (Eq. 45),
 *   - box-car binning and the Gaussian log-likelihood (Eq. 1-3), with
 *     lnL = -1e300 for invalid samples (Section "Likelihood").
 *
 * Conventions
 *   - Units are cgs (pressures given in bar where a name says so).
 *   - Every pointer marked "dev" is device memory on the context's device,
 *     row-major and contiguous, owned by the caller.  "host" pointers are only
 *     read during the call that receives them and may be freed afterwards.
 *   - exofwd_forward / exofwd_grad only enqueue work on the given HIP stream
 *     (hipStream_t passed as void*, NULL = the null stream) and never
 *     synchronise; results are valid once the stream reaches that point.
 *   - Misuse visible on the host (bad sizes, NULL required pointers, a mode the
 *     context was not built for) returns an error status and enqueues nothing.
 *     Per-sample numerical invalidity is reported in status[b] bits; such a
 *     sample gets lnL = -1e300, a NaN spectrum and a zero gradient.
 *   - One context serves one stream at a time (calls on a context must not
 *     overlap); several contexts may share a device.
 */
#ifndef EXOFWD_H
#define EXOFWD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct exofwd_ctx exofwd_ctx;

typedef enum {
  EXOFWD_OK = 0,
  EXOFWD_ERR_ARG = 1,         /* NULL or out-of-range argument */
  EXOFWD_ERR_SHAPE = 2,       /* sizes inconsistent with the context */
  EXOFWD_ERR_CONFIG = 3,      /* invalid configuration at create time */
  EXOFWD_ERR_NOMEM = 4,       /* device allocation failed */
  EXOFWD_ERR_DEVICE = 5,      /* a HIP runtime call failed */
  EXOFWD_ERR_UNSUPPORTED = 6  /* valid request this build does not provide */
} exofwd_status;

enum { EXOFWD_TRANSMISSION = 0, EXOFWD_EMISSION = 1 };

/* FP64: FP64 tables and arithmetic throughout ("plain FP64").
 * MIXED: log-sigma tables stored relative to per-(species, nu) FP32 offsets,
 *        as FP16 entries in transmission and FP32 entries in emission; FP32
 *        opacity; transmission chords as bf16x3 split-precision MFMA products
 *        with FP32 accumulation, the emission sweep in FP32; profile,
 *        hydrostatics and likelihood sums stay FP64.                   */
enum { EXOFWD_PREC_FP64 = 0, EXOFWD_PREC_MIXED = 1 };

/* T-p profiles (Section "T-p profile parameterisation"): isothermal (Eq. 7), the
 * modified Guillot profile (Eq. 16) in three- and seven-parameter forms, PCHIP
 * knots, Barstow 2020 (Eq. 8) and the modified Milne profile (Eqs. 9-14). */
enum { EXOFWD_TP_ISOTHERMAL = 0, EXOFWD_TP_GUILLOT3 = 1, EXOFWD_TP_PCHIP = 2, EXOFWD_TP_BARSTOW = 3,
       EXOFWD_TP_MILNE = 4, EXOFWD_TP_GUILLOT7 = 5 };

/* Cloud models (transmission).  GREY_DECK: a slab from P_cloud down with a
 * fixed grey opacity kappa_cloud.  NONGREY: a condensate profile q_c(p)
 * (Eqs. 18-20) and the extinction efficiency Q_ext of an effective particle
 * size (Eqs. 23-25, 27-29): dtau_cloud = q_c rho dr 3 Q_ext / (4 r_eff). */
enum { EXOFWD_CLOUD_GREY_DECK = 0, EXOFWD_CLOUD_NONGREY = 1 };
enum { EXOFWD_QPROF_UNIFORM = 0, EXOFWD_QPROF_SLAB = 1, EXOFWD_QPROF_POWER = 2 };
enum { EXOFWD_QEXT_FIT = 0, EXOFWD_QEXT_FIT_FEATURE = 1, EXOFWD_QEXT_GREY = 2 };

/* per-sample status bits */
enum {
  EXOFWD_S_BAD_VMR = 1,      /* sum of absorber mixing ratios >= 1 */
  EXOFWD_S_UNBOUND = 2,      /* 1/r <= 0 somewhere: atmosphere not bound */
  EXOFWD_S_NONFINITE = 4,    /* a parameter or an output is not finite */
  EXOFWD_S_BAD_T = 8,        /* a temperature is <= 0 or not finite */
  EXOFWD_S_BAD_LAYERS = 16   /* n_layers[b] outside [1, n_layers_max] */
};

/*
 * Static description of one workload; read only by exofwd_create.
 *
 * Parameter vector layout, per sample (P = exofwd_num_params):
 *   T-p:  isothermal  -> [T_iso]
 *         guillot3    -> [T_int, T_eq, log10 gamma_v]          (Eq. 16, q = 2/3)
 *         pchip       -> [T_0 .. T_{n_knots-1}], knot k at log10 p equally
 *                        spaced from p_top (k = 0) to p_bot
 *         barstow     -> [T_strat]   (Eq. 8: isotherm to 0.1 bar, adiabat with kappa = 2/7
 *                        to 1 bar, isotherm below)
 *         milne       -> [T_int, log10 kappa_ir, T_ratio, log10 p_t/bar, beta]
 *                        (Eqs. 9-14: T^4 = 3/4 T_int^4 (tau + q), tau = kappa_ir p / g_ref,
 *                        q stretched from q0 = 4/3 T_ratio^4 to q_inf = 0.710446)
 *         guillot7    -> [T_int, T_eq, log10 kappa_ir, log10 gamma_v, q_irr0, log10 p_t/bar, beta]
 *                        (Eq. 16, q_int = 2/3, q_irr stretched from q_irr0 to 2/3;
 *                        kappa_ir here replaces the config's kappa_ir)
 *   then  log10 X_s for s = 0..n_species-1                       (Eq. 35)
 *   then  cloud parameters      if has_cloud:
 *           GREY_DECK: [log10 P_cloud/bar]
 *           NONGREY:   [log10 r_eff/um]
 *                      + [a, log10 Q0]                 unless QEXT_GREY (Eq. 24)
 *                      + [log10 q]                       (QPROF_UNIFORM, Eq. 18)
 *                        [log10 q, log10 p_top/bar, log10 dp/bar]   (SLAB, Eq. 19)
 *                        [log10 q_base, log10 p_base/bar, alpha]    (POWER, Eq. 20)
 *                      + [A, lambda0/um, log10 omega/um, xi]   if QEXT_FIT_FEATURE
 *                        (Eqs. 27-29; the window's x0 is 0.5 and Q_max is 2)
 *   then  f_cld                 if has_fcld: cloudy fraction of the limb in [0, 1] (Eq. 26);
 *                               the spectrum is f_cld x (cloudy) + (1 - f_cld) x (cloud-free)
 *   then  [log10 g/cgs, M/M_Jup] if has_bd (emission, isolated object, Eqs. 46-47): the gravity
 *                               replaces g_ref (hydrostatics, T-p optical depth), the radius at
 *                               p_ref is sqrt(G M / g), and the spectrum is the flux at the
 *                               observer s F_toa (R/bd_distance)^2 [erg s^-1 cm^-2 (cm^-1)^-1]
 *   then  R_p scale factor      if has_scale  (R_ref = scale * r_p)
 *   then  offset [ppm]          if has_offset (added to bins with offset_mask)
 */
typedef struct exofwd_config {
  int32_t mode;              /* EXOFWD_TRANSMISSION / EXOFWD_EMISSION */
  int32_t precision;         /* EXOFWD_PREC_FP64 / EXOFWD_PREC_MIXED */
  int32_t tp_kind;           /* EXOFWD_TP_* */
  int32_t n_knots;           /* PCHIP knots (2..8), else ignored */
  int32_t n_species;         /* absorbers S, 1..8 */
  int32_t n_layers_max;      /* L_max, 1..160; layers per sample default to it */
  int32_t batch_max;         /* B_max: largest B any call may pass */
  int32_t has_cia, has_rayleigh, has_cloud, has_scale, has_offset;
  int32_t n_mu;              /* emission Gauss-Legendre angles, 1..8 */
  int32_t cloud_model;       /* EXOFWD_CLOUD_* (has_cloud; NONGREY for transmission only) */
  int32_t cloud_profile;     /* EXOFWD_QPROF_* (NONGREY) */
  int32_t cloud_qext;        /* EXOFWD_QEXT_* (NONGREY) */
  int32_t has_fcld;          /* cloudy/clear mixing, Eq. 26 (transmission with has_cloud); each sample
                                costs two spectra */
  double mu_fixed;           /* > 0: fixed mean molecular weight [amu]; else from composition */
  double p_bot_bar, p_top_bar, p_ref_bar;   /* grid bottom/top, reference pressure [bar] */
  double r_p, r_s, g_ref;    /* reference radius [cm], stellar radius [cm], gravity at r_p [cm s^-2] */
  double kappa_ir, f_hem;    /* guillot3 infrared opacity [cm^2 g^-1]; redistribution factor (guillot3/7) */
  double kappa_cloud;        /* grey deck mass opacity [cm^2 g^-1] */
  double t_star, dilution;   /* emission: stellar blackbody T [K], dilution s */
  double err_c;              /* error inflation exponent c (Eq. 3); -99 = off */
  double ray_h2, ray_he;     /* Rayleigh cross sections at 1e4 cm^-1 [cm^2], scaled by (nu/1e4)^4 */
  int32_t n_nu;              /* wavenumbers */
  const double* nu;          /* host [n_nu], ascending [cm^-1] */
  int32_t n_t, n_p;          /* cross-section table axes (2..255 each) */
  const double* t_grid;      /* host [n_t] ascending [K] */
  const double* logp_grid;   /* host [n_p] ascending log10(p / 1 bar) */
  const double* log10_xsec;  /* host [n_species][n_t][n_p][n_nu] log10 sigma [cm^2] */
  const double* species_mass;/* host [n_species] [amu] */
  int32_t n_tc;              /* CIA temperature axis (2..255) if has_cia */
  const double* tc_grid;     /* host [n_tc] ascending [K] */
  const double* log10_cia;   /* host [2][n_tc][n_nu] log10 k [cm^5]: H2-H2, H2-He */
  int32_t n_bins;            /* K >= 1 */
  const int32_t* bin_lo;     /* host [K]: bin k averages native points [lo_k, hi_k) */
  const int32_t* bin_hi;     /* host [K] */
  const double* y_obs;       /* host [K] observed binned spectrum */
  const double* y_err;       /* host [K] 1-sigma errors */
  const uint8_t* offset_mask;/* host [K] or NULL: bins that receive the offset */
  int32_t device;            /* HIP device ordinal */
  int32_t has_bd;            /* emission of an isolated object (Eqs. 46-47); excludes has_scale */
  double bd_distance;        /* its distance [cm] (has_bd) */
  /* Correlated-k tables (Section "Gas phase opacities"): with ck_g > 0, nu holds the
   * n_nu spectral bin centres (ascending) and log10_xsec is [n_species][n_t][n_p][n_nu][ck_g]:
   * log10 k at ck_g g-points of each bin's cross-section distribution (non-decreasing in g,
 * else EXOFWD_ERR_CONFIG),
   * with weights ck_weights[ck_g] (each > 0, summing to 1).  log10_cia is given at the
   * bin centres.  The spectrum has one value per bin and the bins (bin_lo/bin_hi) group
   * spectral bins.  ck_g must be 8; MIXED precision only (FP32 table entries); no
   * gradient (exofwd_grad_supported gives 0), no cloudy/clear mixing, isolated object or
   * non-grey cloud; the absorbers are mixed by ck_mix. */
  int32_t ck_g;              /* g-points per bin, 8; 0 = cross-section (opacity-sampling) tables */
  int32_t ck_mix;            /* EXOFWD_CK_RORR or EXOFWD_CK_PRODUCT */
  const double* ck_weights;  /* host [ck_g] */
} exofwd_config;

/* Mixing of the absorbers' k-distributions in a layer: random overlap with resorting
 * and rebinning (Amundsen et al. 2017; the rebinned k is the mean of the sorted pair
 * distribution over each g-interval, the absorbers mixed in table order, the grey
 * continuum added to every g-point).  EXOFWD_CK_PRODUCT (transmission only): random
 * overlap along each chord, the product of the absorbers' transmission functions, each
 * absorber keeping its own g-points (the grey continuum a further factor). */
enum { EXOFWD_CK_RORR = 0, EXOFWD_CK_PRODUCT = 1 };

/* Validate the configuration, upload and encode the tables, allocate the
 * workspace for batch_max samples of n_layers_max layers.  Synchronous.
 * On success *out owns all device memory of the context.  Every check below runs
 * on the host before any device call:
 *   EXOFWD_ERR_CONFIG       an invalid description, including a non-finite entry in
 *                           log10_xsec or log10_cia (give a zero cross-section as a
 *                           finite floor);
 *   EXOFWD_ERR_UNSUPPORTED  in MIXED precision, a line or CIA table of 2^31 bytes or more once
 *                           encoded (2 bytes per entry in transmission, 4 in emission,
 *                           n_nu padded to a multiple of 128), or padded layers x padded
 *                           n_nu x 4 bytes of 2^31 or more (the reduced-precision
 *                           kernels address these buffers with 32-bit offsets).
 * EXOFWD_ERR_DEVICE / EXOFWD_ERR_NOMEM for device failures.  On failure
 * exofwd_last_error(NULL) gives the reason (per thread). */
exofwd_status exofwd_create(const exofwd_config* cfg, exofwd_ctx** out);

/* Free everything the context owns (synchronises its device). NULL is a no-op. */
exofwd_status exofwd_destroy(exofwd_ctx* ctx);

int32_t exofwd_num_params(const exofwd_ctx* ctx);   /* P, or -1 for NULL */
int32_t exofwd_num_nu(const exofwd_ctx* ctx);       /* n_nu, or -1 */
int32_t exofwd_num_bins(const exofwd_ctx* ctx);     /* K, or -1 */
int32_t exofwd_precision(const exofwd_ctx* ctx);    /* EXOFWD_PREC_*, or -1 */
/* 1 if exofwd_grad supports this context's workload, 0 if not, -1 for a NULL
 * context.  Supported: transmission and emission with cross-section tables
 * (n_layers_max <= 160, both precisions), every T-p profile and cloud model; not
 * the correlated-k tables, whose path is a forward model only. */
int32_t exofwd_grad_supported(const exofwd_ctx* ctx);

/*
 * Forward model for B samples (1 <= B <= batch_max).
 *   params   dev [B][P] double
 *   n_layers dev [B] int32 or NULL (NULL: every sample uses n_layers_max)
 *   spectra  dev [B][n_nu], double in FP64 precision, float in MIXED; or NULL
 *            (transit depth, or F_p/F_* for emission)
 *   lnL      dev [B] double or NULL
 *   status   dev [B] int32 or NULL
 */
exofwd_status exofwd_forward(exofwd_ctx* ctx, int32_t B, const double* params,
                             const int32_t* n_layers, void* spectra, double* lnL,
                             int32_t* status, void* hip_stream);

/* Size in bytes of the static device array that exofwd_forward_noalloc takes its
 * scratch from; every device the library runs on holds one until the process ends. */
#define EXOFWD_NOALLOC_SCRATCH_BYTES (64u << 20)

/*
 * exofwd_forward for callers that cannot allocate device memory: code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same arguments,
 * kernels and results (bit for bit) as exofwd_forward, but the per-call workspace
 * (profile records, path-matrix fragments, likelihood partials, and the spectra
 * when spectra is NULL or with the cloudy/clear mixing) lives in a static device
 * array of EXOFWD_NOALLOC_SCRATCH_BYTES on the context's device, not in the
 * context's own workspace.  The call allocates and frees nothing, creates no
 * events (per-kernel timing is skipped) and never captures or replays graphs (a
 * caller that is capturing its stream gets the kernels in its own graph).
 *   EXOFWD_ERR_SHAPE   the batch's workspace exceeds the array (last_error gives
 *                      the bytes needed); about 80 KB per sample of a 128-layer
 *                      reduced-precision transmission model, plus the spectra
 *   EXOFWD_ERR_DEVICE  the array's device address could not be looked up (done
 *                      once per device when the first context is created there)
 * Every call on a device shares that device's array and overwrites it: calls that
 * overlap in time on one device, from any context or stream, race and give wrong
 * results.  Nothing in the array needs to start at zero.
 */
exofwd_status exofwd_forward_noalloc(exofwd_ctx* ctx, int32_t B, const double* params,
                                     const int32_t* n_layers, void* spectra, double* lnL,
                                     int32_t* status, void* hip_stream);

/*
 * lnL and its gradient with respect to every parameter for B samples, by the
 * hand-written adjoint.  Workloads outside exofwd_grad_supported return
 * EXOFWD_ERR_UNSUPPORTED.
 *   lnL      dev [B] double (required)
 *   grad     dev [B][P] double (required): d lnL / d params
 *   spectra  dev [B][n_nu] (type as in exofwd_forward) or NULL
 *   status   dev [B] int32 or NULL
 */
exofwd_status exofwd_grad(exofwd_ctx* ctx, int32_t B, const double* params,
                          const int32_t* n_layers, void* spectra, double* lnL,
                          double* grad, int32_t* status, void* hip_stream);

/*
 * Launch choices of a reduced-precision transmission context, four int32:
 *   [0] forward grid order: 0 samples fastest, 1 wavenumber tiles fastest
 *   [1] reverse-kernel shape: 0 = 128-wavenumber tiles x 4 row blocks, 1 = 64 x 4,
 *       2 = 64 x 5 (padded layers <= 160; 0 and 1 alone serve <= 128).  With more than
 *       128 padded layers, 0 and 1 run the samples of at most 128 layers with their
 *       shape and the rest with 64 x 5 (and the forward kernel always runs those two
 *       classes, the longer one in two 128-layer chunks); 2 runs every sample with
 *       64 x 5
 *   [2] reverse work items per call, one of 512, 1024, 2048, 4096, 8192 (each sample's
 *       wavenumbers are split into ceil(items / B) chunks, which run on neighbouring
 *       workgroups)
 *   [3] 128-wavenumber tiles per wave of the layer-sum kernel: 4, 8, 16, 32 or 64
 * Every choice gives the same results up to FP32 summation order.
 * exofwd_set_tuning returns EXOFWD_ERR_ARG, changing nothing, for a choice that
 * does not serve the context (entries [1..3] are ignored when the context has no
 * reduced-precision gradient); it synchronises the device and drops captured
 * graphs.  exofwd_get_tuning writes the current choices.
 */
exofwd_status exofwd_set_tuning(exofwd_ctx* ctx, const int32_t* tuning);
exofwd_status exofwd_get_tuning(const exofwd_ctx* ctx, int32_t* tuning);

/*
 * Time the launch choices at batch B and keep the fastest (synchronous; it
 * allocates its own timing buffers and stream).  params dev [B][P] double, or
 * NULL for a built-in valid mid-range parameter vector; n_layers dev [B] int32
 * or NULL, as in exofwd_forward.  The step timed is exofwd_grad where supported,
 * else exofwd_forward.  cache_path (may be NULL) is a text file of earlier results,
 * one line per key (device architecture, CU count, workload shape, B); a matching
 * line is applied without timing, and a new result is written back to the file.
 * FP64 and emission contexts have no tunable choices: the call returns EXOFWD_OK.
 */
exofwd_status exofwd_autotune(exofwd_ctx* ctx, int32_t B, const double* params, const int32_t* n_layers,
                              const char* cache_path);

/*
 * Graph replay (off by default).  When enabled, the first exofwd_forward or
 * exofwd_grad call with a given (call kind, B, pointer arguments, stream) is
 * captured into a hipGraph on its stream and launched; later calls with the same
 * arguments launch that graph (up to 16 are kept, least recently used dropped).
 * Buffers are read at replay, so new parameter values in the same buffer are
 * evaluated.  The stream must not be the null stream (EXOFWD_ERR_ARG).  A call
 * made while the caller is itself capturing the stream is enqueued into the
 * caller's graph.  Changing the setting synchronises the device and drops the
 * captured graphs.  Per-kernel timing then reports one "graph" entry per call.
 */
exofwd_status exofwd_set_graphs(exofwd_ctx* ctx, int32_t enable);

/* Per-kernel timing of the calls that follow: when enabled, each kernel launch
 * is bracketed by HIP events on the call's stream.  exofwd_kernel_time then
 * reports the summed milliseconds and launch count for the kernel named
 * (e.g. "trans_fwd"), synchronising the stream of the last call.  Resetting
 * clears the tallies. */
exofwd_status exofwd_set_profiling(exofwd_ctx* ctx, int32_t enable);
exofwd_status exofwd_kernel_time(exofwd_ctx* ctx, const char* name, double* total_ms,
                                 int32_t* launches);

/* Bytes of device memory the context holds. */
int64_t exofwd_device_bytes(const exofwd_ctx* ctx);

const char* exofwd_strerror(exofwd_status s);
/* Text of the last error raised on this context (empty if none); with a NULL
 * context, the text of this thread's last failed exofwd_create. */
const char* exofwd_last_error(const exofwd_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* EXOFWD_H */
