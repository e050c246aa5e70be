// Internal definitions shared by the host library and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace exofwd {

// CODATA 2018 constants, cgs
constexpr double kB = 1.380649e-16;        // erg K^-1
constexpr double kHpl = 6.62607015e-27;    // erg s
constexpr double kC = 2.99792458e10;       // cm s^-1
constexpr double kMu = 1.66053906660e-24;  // g
constexpr double kBar = 1.0e6;             // dyn cm^-2
constexpr double kGrav = 6.67430e-8;       // cm^3 g^-1 s^-2
constexpr double kMJup = 1.89813e30;       // g (nominal G M_J / G)
constexpr double kHeH2 = 0.164;            // He/H2 filling ratio (Eq. 36)
constexpr double kMH2 = 2.01588, kMHe = 4.002602;
constexpr double kLog2_10 = 3.321928094887362347870319429489;
constexpr double kInvalidLnL = -1.0e300;

constexpr int kMaxSpecies = 8;
constexpr int kMaxLayers = 160;   // L_max; padded layer count is a multiple of 32
constexpr int kLsGroup = 3;       // most layers in one reduced-precision layer-sum group
constexpr int kMaxKnots = 8;
constexpr int kMaxMu = 8;
constexpr int kTileNu = 128;      // wavenumbers per tile of the reduced-precision transmission kernels
constexpr int kTile64 = 64;       // wavenumbers per tile of the FP64 and emission kernels
// cache policy of a buffer access that streams data read or written once (the
// non-temporal bit of gfx950's buffer instructions): it keeps the table lines and
// path-matrix fragments that other accesses reuse in L2
constexpr int kCpolStream = 2;
constexpr int kBlock = 256;       // threads per workgroup (4 wave64)
constexpr int kBlockT = 512;      // threads per workgroup of the reduced-precision transmission kernels
constexpr int kShortLayers = 128;  // layer capacity of the short class of a ragged reduced-precision batch
constexpr int kCkG = 8;           // g-points per bin of a correlated-k table
constexpr int kCkBinsPerWave = 16;  // bins one wave of the k-distribution mixing kernel walks through
// a chord optical depth beyond which e^-tau is zero in FP32 with a wide margin
// (e^-103.3 is already below the smallest denormal): its adjoint seed is exactly 0
constexpr float kOpaqueTau = 110.0f;

// per-layer record of the opacity kernels (one per sample and layer)
//   [0] wT, [1] wP, [2] wTc, [3] Rayleigh coefficient R_l (x (nu/1e4)^4),
//   [4] cloud term D_l, [5] lam_c1, [6] lam_c2, [7..7+S) lam_s
// with lam = log2 of the per-layer prefactor (n X dr, n^2 X X dr).  D_l is the
// grey deck's optical depth, or for the non-grey cloud the layer's column
// q_l rho_l dr_l 3 / (4 r_eff) that multiplies Q_ext(nu).
constexpr int kRecFixed = 7;
__host__ __device__ constexpr int rec_len(int s) { return kRecFixed + s; }

// packed interpolation cells of one layer: iT | iP << 8 | iTc << 16
__host__ __device__ inline int pack_cells(int it, int ip, int itc) { return it | (ip << 8) | (itc << 16); }

enum : int { kTransmission = 0, kEmission = 1 };
enum : int { kCkRorr = 0, kCkProduct = 1 };
enum : int { kFP64 = 0, kMixed = 1 };
enum : int { kTpIso = 0, kTpGuillot3 = 1, kTpPchip = 2, kTpBarstow = 3, kTpMilne = 4, kTpGuillot7 = 5 };
constexpr double kKappaAd = 2.0 / 7.0;    // adiabatic exponent of the Barstow profile (Eq. 8)
constexpr double kQHopfInf = 0.710446;    // large-depth Hopf value, q_inf of the modified Milne profile
enum : int { kQprofUniform = 0, kQprofSlab = 1, kQprofPower = 2 };
enum : int { kQextFit = 0, kQextFeature = 1, kQextGrey = 2 };
constexpr int kCloudSpec = 7;   // spectral cloud parameters: log10 r, a, log10 Q0, A, lambda0, log10 omega, xi
enum : int { kBadVmr = 1, kUnbound = 2, kNonfinite = 4, kBadT = 8, kBadLayers = 16 };

// Everything a kernel needs to know about the workload (by value).
struct Model {
  int mode, tp_kind, n_knots, S, L_max, L_pad, P;
  int has_cia, has_ray, has_cloud, has_scale, has_offset, n_mu;
  int n_nu, n_nu_pad, n_tiles, n_tiles64, n_t, n_p, n_tc, K;
  int ll_lanes;         // lanes that sum one bin in the likelihood kernel (8, 16, 32 or 64)
  int idx_cloud, idx_scale, idx_offset, n_tp;
  int fwd_tile_major;       // reduced-precision forward grid order: 0 samples fastest, 1 tiles fastest
  int cloud_ng;             // 1: non-grey cloud (q_c profile x Q_ext(nu)); 0: grey deck or none
  int cloud_profile, cloud_qext, n_cloud;   // kQprof*, kQext*, cloud parameters in theta
  int has_fcld, idx_fcld;   // cloudy/clear mixing: sample b runs as virtual samples 2b (cloudy) and 2b+1 (clear)
  int has_bd, idx_bd;       // isolated object: theta[idx_bd] = log10 g, theta[idx_bd + 1] = M / M_Jup
  double bd_dist;           // its distance [cm]
  int ck;                   // correlated-k tables: n_nu spectral bins of kCkG g-points (reduced precision)
  int ck_mix;               // their mixing (kCkRorr)
  double mu_fixed, log10_pbot, log10_ptop, p_ref, r_p, r_s, g_ref;
  double kappa_ir, f_hem, kappa_cloud, t_star, dilution, err_c, ray_h2, ray_he;
  double mass[kMaxSpecies];
  double mu_nodes[kMaxMu], mu_weights[kMaxMu];
  const double* t_grid;     // [n_t]
  const double* logp_grid;  // [n_p]
  const double* tc_grid;    // [n_tc]
  const double* nu;         // [n_nu_pad] (padded with the last value)
};

// The reduced-precision transmission records (not correlated-k) also carry, after
// the logs, the S line prefactors col_s = n X_s dr themselves (they fit FP32; the CIA
// prefactor, quadratic in n, need not): [7+S..7+2S) col_s
__host__ __device__ constexpr int rec_len_wide(int s) { return kRecFixed + 2 * s; }
__host__ __device__ inline bool rec_wide(const Model& m, bool fp64) { return m.mode == kTransmission && !fp64 && !m.ck; }
__host__ __device__ inline int rec_stride(const Model& m, bool fp64) {
  return rec_wide(m, fp64) ? rec_len_wide(m.S) : rec_len(m.S);
}

// real sample and cloud-free flag of a virtual sample
__host__ __device__ inline int real_sample(const Model& m, int b) { return m.has_fcld ? b >> 1 : b; }
__host__ __device__ inline bool clear_sample(const Model& m, int b) { return m.has_fcld && (b & 1); }

// Workspace of one context, sized for batch_max x L_pad (2 batch_max virtual
// samples with the cloudy/clear mixing).
struct Work {
  int32_t* status;      // [B]
  int32_t* nlay;        // [B] layers used per sample
  int32_t* cls;         // layer-count classes (L_pad > kShortLayers, reduced-precision transmission): [2 + 2B]
  double* t_lay;        // [B][L_pad]
  double* t_lev;        // [B][L_pad+1]
  double* inv_tlev;     // reduced-precision emission: [B][L_pad+1] 1 / T at the levels (the Planck exponents)
  double* r_lev;        // [B][L_pad+1]
  double* core;         // [B] r_0^2 / R_s^2
  double* cloud;        // [B][kCloudSpec] non-grey cloud: r_eff [cm], a, Q0, A, lambda0 [um], omega [um], xi
  float* cloud_q;       // reduced precision, non-grey: [B][1 + kCloudSpec][n_nu_pad] Q_ext(nu), dQ_ext/dp_k
  int32_t* cells;       // [B][L_pad] packed cells
  int32_t* lsg;         // reduced precision: [B][L_pad + 1] layer-sum groups, their number
                        //   and then (first layer | layers << 16) of each: runs of at most
                        //   kLsGroup consecutive layers in one table cell, in layer order
  int32_t* front;       // reduced precision: [B][n_tiles] opaque 32-row chord blocks at the bottom of
                        //   each 128-wavenumber tile (every tau > kOpaqueTau), set by a forward pass
                        //   that stores the layer optical depths
  void* rec;            // [B][L_pad][rec_stride] float (mixed) or double (fp64)
  void* area;           // [B][L_pad] (r_{i+1}^2 - r_i^2)/R_s^2, float or double
  double* pm64;         // fp64: [B][L_pad][L_pad] path matrix
  uint16_t* pfrag;      // mixed: [B][MB][KB][64][8] bf16, hi then lo planes
  uint16_t* ptfrag;     // mixed: transposed path matrix fragments (adjoint)
  void* spec;           // [B][n_nu] internal spectrum when the caller passes none
  double* dm;           // [B][K] d lnL / d m_k
  double* lnl_tmp;      // [B]
  double* gv;           // cloudy/clear mixing: [2B][P] gradients of the virtual samples
  double* fbar;         // cloudy/clear mixing: [B] d lnL / d f_cld
  double* mdot;         // [B] sum_k d lnL/dm_k (m_k - offset_k): d lnL / d ln(spectrum scale)
  float* ckmix;         // correlated-k: [B][L_pad][n_nu_pad * kCkG] mixed layer optical depths per (bin, g-point)
  const int32_t* bin_of;  // [n_nu_pad] bin holding each wavenumber, -1 if none
  const double* inv_cnt;  // [K] 1 / (hi_k - lo_k)
};

// Tables on the device.
struct Tables {
  const uint16_t* h;     // mixed: [S][n_t][n_p][n_nu_pad] fp16 (log2 sigma - c); emission: fp32 entries (two halves each)
  const float* c;        // mixed: [S][n_nu_pad] per-(species, nu) offsets, log2 units
  const uint16_t* hc;    // mixed: [2][n_tc][n_nu_pad] (fp32 entries for emission)
  const float* cc;       // mixed: [2][n_nu_pad]
  const float* nu4f;     // mixed: [n_nu_pad] (nu/1e4)^4
  const double* t64;     // fp64: [S][n_t][n_p][n_nu_pad] log10 sigma
  const double* tc64;    // fp64: [2][n_tc][n_nu_pad] log10 k
  const double* nu4d;    // fp64: [n_nu_pad]
  const float* ckw;      // correlated-k: [kCkG] g-point weights
  const double* ckwd;    // correlated-k: [kCkG] g-point weights in FP64 (the mixing's bookkeeping)
  const double* cke;     // correlated-k: [kCkG] upper edges of the g-intervals (running sums of the weights)
};

}  // namespace exofwd
