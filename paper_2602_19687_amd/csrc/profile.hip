// Per-sample atmospheric profile in FP64: T-p profile, free chemistry,
// hydrostatic altitudes, per-layer opacity records, path matrix and annulus
// areas.  One workgroup of 256 threads per sample.
#include "cloud.h"
#include "kernels.h"
#include "tp.h"

namespace exofwd {

// Largest i with grid[i] <= x, capped at n-2, and the linear weight; x is
// clamped to the grid first (a clamped x gets w = 0 or 1).  NaN maps to cell 0.
__device__ inline void cell_index(const double* grid, int n, double x, int& i, double& w) {
  if (!(x > grid[0])) { i = 0; w = 0.0; return; }
  if (x >= grid[n - 1]) { i = n - 2; w = 1.0; return; }
  int lo = 0, hi = n - 1;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (grid[mid] <= x) lo = mid; else hi = mid;
  }
  i = lo;
  w = (x - grid[lo]) / (grid[lo + 1] - grid[lo]);
}

// Monotone cubic Hermite slopes (Fritsch-Carlson with the Fritsch-Butland
// weighted harmonic mean inside, three-point shape-preserving ends).
__device__ void pchip_slopes(const double* xk, const double* yk, int n, double* d) {
  double h[kMaxKnots], del[kMaxKnots];
  for (int k = 0; k < n - 1; ++k) { h[k] = xk[k + 1] - xk[k]; del[k] = (yk[k + 1] - yk[k]) / h[k]; }
  if (n == 2) { d[0] = d[1] = del[0]; return; }
  for (int k = 1; k < n - 1; ++k) {
    double a = del[k - 1], b = del[k];
    if (a == 0.0 || b == 0.0 || (a > 0.0) != (b > 0.0)) {
      d[k] = 0.0;
    } else {
      double w1 = 2.0 * h[k] + h[k - 1], w2 = h[k] + 2.0 * h[k - 1];
      d[k] = (w1 + w2) / (w1 / a + w2 / b);
    }
  }
  auto end = [](double h0, double h1, double m0, double m1) {
    double dd = ((2.0 * h0 + h1) * m0 - h0 * m1) / (h0 + h1);
    auto sgn = [](double v) { return (v > 0.0) - (v < 0.0); };
    if (sgn(dd) != sgn(m0)) return 0.0;
    if (sgn(m0) != sgn(m1) && fabs(dd) > fabs(3.0 * m0)) return 3.0 * m0;
    return dd;
  };
  d[0] = end(h[0], h[1], del[0], del[1]);
  d[n - 1] = end(h[n - 2], h[n - 3], del[n - 2], del[n - 3]);
}

__device__ double pchip_eval(const double* xk, const double* yk, const double* d, int n, double x) {
  int k = 0;
  while (k < n - 2 && xk[k + 1] <= x) ++k;
  double hk = xk[k + 1] - xk[k];
  double t = (x - xk[k]) / hk;
  double omt = 1.0 - t;
  return (1.0 + 2.0 * t) * omt * omt * yk[k] + t * omt * omt * hk * d[k] + t * t * (3.0 - 2.0 * t) * yk[k + 1] +
         t * t * (t - 1.0) * hk * d[k + 1];
}

// Reduced modified Guillot profile (Eq. 16 with q_int = q_irr = 2/3, mu_* = 1/sqrt 3).
__device__ inline double guillot3(double t_int, double t_eq, double gam, double tau, double f_hem) {
  const double s3 = 1.7320508075688772935274463415059;
  const double q = 2.0 / 3.0;
  double ti2 = t_int * t_int, te2 = t_eq * t_eq;
  double t4 = 0.75 * ti2 * ti2 * (q + tau) +
              0.75 * te2 * te2 * 4.0 * f_hem * (q + 1.0 / (gam * s3) + (gam / s3 - 1.0 / (gam * s3)) * exp(-gam * tau * s3));
  return sqrt(sqrt(t4));
}

// Round to nearest even bf16 (finite inputs).
__device__ inline uint16_t bf16_rn(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf16_to_f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Path matrix entry P_1D[i][l] (Eq. 43) with b_i the mid radius of layer i.
// The l > i case uses sqrt(r_up^2-b^2) - sqrt(r_lo^2-b^2) = dr (r_up+r_lo)/(s_up+s_lo),
// which has no cancellation; square roots are taken of (r-b)(r+b).
__device__ inline double path_entry(const double* r, const double* dr, int i, int l) {
  if (l < i) return 0.0;
  double b = 0.5 * (r[i] + r[i + 1]);
  if (l == i) {
    double sup = sqrt(0.5 * dr[i] * (r[i + 1] + b));
    return 2.0 * sup / dr[i];
  }
  double rup = r[l + 1], rlo = r[l];
  double sup = sqrt((rup - b) * (rup + b));
  double slo = sqrt((rlo - b) * (rlo + b));
  return 2.0 * (rup + rlo) / (sup + slo);
}

template <typename Real>
__global__ __launch_bounds__(kBlock) void k_profile(Model m, Work w, const double* __restrict__ params,
                                                    const int32_t* __restrict__ n_layers) {
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  const int Lp = m.L_pad;
  __shared__ double s_t[kMaxLayers + 1];      // layer T
  __shared__ double s_tl[kMaxLayers + 1];     // level T (emission)
  __shared__ double s_u[kMaxLayers + 1];      // 1/r at levels
  __shared__ double s_r[kMaxLayers + 1];
  __shared__ double s_dr[kMaxLayers];
  __shared__ double s_inc[kMaxLayers];
  __shared__ double s_knot_x[kMaxKnots], s_knot_y[kMaxKnots], s_knot_d[kMaxKnots];
  __shared__ int s_status;
  __shared__ int s_badt;
  __shared__ int s_cell[kMaxLayers];

  // virtual sample b of real sample bs; a clear one (cloudy/clear mixing) has no cloud
  const int bs = real_sample(m, b);
  const bool cloudy = m.has_cloud && !clear_sample(m, b);
  const double* th = params + (size_t)bs * m.P;
  int L = n_layers ? n_layers[bs] : m.L_max;
  int status = 0;
  if (L < 1 || L > m.L_max) {
    status = kBadLayers;
    L = m.L_max;
  }
  bool finite = true;
  for (int k = 0; k < m.P; ++k) finite = finite && isfinite(th[k]);
  if (!status && !finite) status = kNonfinite;

  // chemistry (Eq. 35-36), every thread keeps its own copy
  double x[kMaxSpecies];
  double sx = 0.0;
  for (int s = 0; s < m.S; ++s) { x[s] = exp10(th[m.n_tp + s]); sx += x[s]; }
  const double xh2 = (1.0 - sx) / (1.0 + kHeH2);
  const double xhe = kHeH2 * xh2;
  double mu = m.mu_fixed;
  if (!(mu > 0.0)) {
    mu = xh2 * kMH2 + xhe * kMHe;
    for (int s = 0; s < m.S; ++s) mu += x[s] * m.mass[s];
  }
  const double scale = m.has_scale ? th[m.idx_scale] : 1.0;
  // an isolated object retrieves its gravity; its radius at p_ref is sqrt(G M / g) (Eq. 47)
  const double g_ref = m.has_bd ? exp10(th[m.idx_bd]) : m.g_ref;
  const double r_ref = m.has_bd ? sqrt(kGrav * th[m.idx_bd + 1] * kMJup / g_ref) : m.r_p * scale;

  const double step = (m.log10_ptop - m.log10_pbot) / L;   // log10 p per layer (negative)
  const double dlnp = -step * 2.302585092994045684017991454684;  // ln(p_l / p_{l+1})
  auto logp_lev = [&](int j) { return j == L ? m.log10_ptop : m.log10_pbot + j * step; };

  if (tid == 0) {
    s_badt = 0;
    if (m.tp_kind == kTpPchip) {
      for (int k = 0; k < m.n_knots; ++k) {
        s_knot_x[k] = m.n_knots == 1 ? m.log10_ptop
                                     : m.log10_ptop + k * ((m.log10_pbot - m.log10_ptop) / (m.n_knots - 1));
        s_knot_y[k] = th[k];
      }
      s_knot_x[m.n_knots - 1] = m.log10_pbot;
      pchip_slopes(s_knot_x, s_knot_y, m.n_knots, s_knot_d);
    }
  }
  __syncthreads();

  auto temperature = [&](double log10p_bar) {
    if (m.tp_kind == kTpIso) return th[0];
    if (m.tp_kind == kTpGuillot3) {
      double tau = m.kappa_ir * exp10(log10p_bar) * kBar / g_ref;
      return guillot3(th[0], th[1], exp10(th[2]), tau, m.f_hem);
    }
    if (m.tp_kind == kTpBarstow) return th[0] * barstow_factor(log10p_bar);
    if (m.tp_kind == kTpMilne) return sqrt(sqrt(milne_t4(th, log10p_bar, g_ref)));
    if (m.tp_kind == kTpGuillot7) return sqrt(sqrt(guillot7_t4(th, log10p_bar, g_ref, m.f_hem)));
    return pchip_eval(s_knot_x, s_knot_y, s_knot_d, m.n_knots, log10p_bar);
  };

  int badt = 0;
  for (int l = tid; l < L; l += kBlock) {
    double t = temperature(0.5 * (logp_lev(l) + logp_lev(l + 1)));
    s_t[l] = t;
    badt |= !(t > 0.0) || !isfinite(t);
  }
  if (m.mode == kEmission) {
    for (int j = tid; j <= L; j += kBlock) {
      double t = temperature(logp_lev(j));
      s_tl[j] = t;
      badt |= !(t > 0.0) || !isfinite(t);
    }
  }
  if (badt) atomicOr(&s_badt, 1);
  __syncthreads();
  if (!status) {
    if (s_badt) status |= kBadT;
    if (!(sx < 1.0)) status |= kBadVmr;
  }

  // hydrostatics (1/r linear in ln p inside each isothermal layer)
  const double kk = kB / (mu * kMu * g_ref * r_ref * r_ref);
  for (int l = tid; l < L; l += kBlock) s_inc[l] = kk * s_t[l] * dlnp;
  __syncthreads();
  if (tid == 0 && !status) {
    const double lpref = log10(m.p_ref / kBar);
    int cnt = 0;
    for (int j = 0; j <= L; ++j) cnt += logp_lev(j) > lpref;
    int lref = min(max(cnt - 1, 0), L - 1);
    const double ln10 = 2.302585092994045684017991454684;
    const double u_ref = 1.0 / r_ref;
    s_u[lref] = u_ref + kk * s_t[lref] * (logp_lev(lref) - lpref) * ln10;
    s_u[lref + 1] = u_ref - kk * s_t[lref] * (lpref - logp_lev(lref + 1)) * ln10;
    for (int j = lref - 1; j >= 0; --j) s_u[j] = s_u[j + 1] + s_inc[j];
    for (int j = lref + 1; j < L; ++j) s_u[j + 1] = s_u[j] - s_inc[j];
    int unbound = 0;
    for (int j = 0; j <= L; ++j) unbound |= !(s_u[j] > 0.0);
    s_status = unbound ? kUnbound : 0;
  }
  __syncthreads();
  if (!status) status = s_status;

  if (tid == 0) {
    w.status[b] = status;
    w.nlay[b] = L;
  }
  if (status) return;   // uniform across the workgroup

  for (int j = tid; j <= L; j += kBlock) s_r[j] = 1.0 / s_u[j];
  __syncthreads();
  // dr_l = r_{l+1} - r_l = (u_l - u_{l+1}) r_l r_{l+1}, and u_l - u_{l+1} = inc_l
  for (int l = tid; l < L; l += kBlock) s_dr[l] = s_inc[l] * s_r[l] * s_r[l + 1];
  __syncthreads();

  double* t_lay = w.t_lay + (size_t)b * Lp;
  double* t_lev = w.t_lev + (size_t)b * (Lp + 1);
  double* r_lev = w.r_lev + (size_t)b * (Lp + 1);
  for (int l = tid; l < Lp; l += kBlock) t_lay[l] = l < L ? s_t[l] : 0.0;
  for (int j = tid; j <= Lp; j += kBlock) {
    r_lev[j] = j <= L ? s_r[j] : 0.0;
    t_lev[j] = (m.mode == kEmission && j <= L) ? s_tl[j] : 0.0;
    if (w.inv_tlev) w.inv_tlev[(size_t)b * (Lp + 1) + j] = j <= L ? 1.0 / s_tl[j] : 0.0;
  }
  // transmission: opaque-core depth (r_0/R_s)^2; emission: (R_ref/R_s)^2 of Eq. 45
  if (tid == 0)
    w.core[b] = m.mode == kTransmission ? s_r[0] * s_r[0] / (m.r_s * m.r_s)
                                        : r_ref * r_ref / (m.has_bd ? m.bd_dist * m.bd_dist : m.r_s * m.r_s);

  // per-layer opacity records
  const bool wide = rec_wide(m, sizeof(Real) == 8);
  const int RL = rec_stride(m, sizeof(Real) == 8);
  Real* rec = reinterpret_cast<Real*>(w.rec) + (size_t)b * Lp * RL;
  Real* area = reinterpret_cast<Real*>(w.area) + (size_t)b * Lp;
  const double log10_pc = m.has_cloud ? th[m.idx_cloud] : 0.0;
  // non-grey cloud: per-sample constants of Q_ext and where the profile's parameters start
  const int q_first = m.idx_cloud + (m.cloud_qext == kQextGrey ? 1 : 3);
  const double r_eff = m.cloud_ng ? 1.0e-4 * exp10(th[m.idx_cloud]) : 1.0;
  if (m.cloud_ng && tid == 0) {
    double* cl = w.cloud + (size_t)b * kCloudSpec;
    const bool fit = m.cloud_qext != kQextGrey, feat = m.cloud_qext == kQextFeature;
    const int f0 = q_first + (m.cloud_profile == kQprofUniform ? 1 : 3);
    cl[0] = r_eff;
    cl[1] = fit ? th[m.idx_cloud + 1] : 0.0;
    cl[2] = fit ? exp10(th[m.idx_cloud + 2]) : 0.0;
    cl[3] = feat ? th[f0] : 0.0;
    cl[4] = feat ? th[f0 + 1] : 1.0;
    cl[5] = feat ? exp10(th[f0 + 2]) : 1.0;
    cl[6] = feat ? th[f0 + 3] : 0.0;
  }
  for (int l = tid; l < Lp; l += kBlock) {
    Real* rl = rec + (size_t)l * RL;
    if (l >= L) {
      w.cells[(size_t)b * Lp + l] = 0;
      for (int k = 0; k < RL; ++k) rl[k] = Real(0);
      rl[5] = rl[6] = Real(-1000);
      for (int s = 0; s < m.S; ++s) rl[kRecFixed + s] = Real(-1000);   // the prefactors stay 0
      area[l] = Real(0);
      continue;
    }
    const double t = s_t[l];
    const double lp_bar = 0.5 * (logp_lev(l) + logp_lev(l + 1));
    const double n = exp10(lp_bar) * kBar / (kB * t);
    const double dr = s_dr[l];
    int it, ip, itc = 0;
    double wt, wp, wtc = 0.0;
    cell_index(m.t_grid, m.n_t, t, it, wt);
    cell_index(m.logp_grid, m.n_p, lp_bar, ip, wp);
    if (m.has_cia) cell_index(m.tc_grid, m.n_tc, t, itc, wtc);
    w.cells[(size_t)b * Lp + l] = pack_cells(it, ip, itc);
    s_cell[l] = pack_cells(it, ip, itc);
    rl[0] = Real(wt);
    rl[1] = Real(wp);
    rl[2] = Real(wtc);
    const bool trans = m.mode == kTransmission;
    rl[3] = Real((trans && m.has_ray) ? n * (xh2 * m.ray_h2 + xhe * m.ray_he) * dr : 0.0);
    double dcl = 0.0;
    if (m.cloud_ng && cloudy) {
      // column q_l rho_l dr_l 3 / (4 r_eff); the kernels multiply it by Q_ext(nu) (Eq. 23)
      dcl = condensate_q(m.cloud_profile, th + q_first, logp_lev(l), logp_lev(l + 1), lp_bar, nullptr) * mu * kMu *
            n * dr * 0.75 / r_eff;
    } else if (trans && cloudy && !m.cloud_ng) {
      double f = (logp_lev(l) - log10_pc) * 2.302585092994045684017991454684 / dlnp;
      f = f < 0.0 ? 0.0 : (f > 1.0 ? 1.0 : f);
      dcl = m.kappa_cloud * mu * kMu * n * f * dr;
    }
    rl[4] = Real(dcl);
    rl[5] = Real(m.has_cia ? log2(n * n * xh2 * xh2 * dr) : -1000.0);
    rl[6] = Real(m.has_cia ? log2(n * n * xh2 * xhe * dr) : -1000.0);
    for (int s = 0; s < m.S; ++s) rl[kRecFixed + s] = Real(log2(n * x[s] * dr));
    if (wide)
      for (int s = 0; s < m.S; ++s) rl[kRecFixed + m.S + s] = Real(n * x[s] * dr);
    area[l] = Real(dr * (s_r[l] + s_r[l + 1]) / (m.r_s * m.r_s));
  }
  if (w.lsg) {
    // layer-sum groups: a run of layers in one table cell reads one set of table
    // rows, so the layer sums fetch them once per tile for the whole group
    __syncthreads();
    if (tid == 0) {
      int32_t* grp = w.lsg + (size_t)b * (Lp + 1);
      int n = 0;
      for (int l = 0; l < L;) {
        int e = l + 1;
        while (e < L && e - l < kLsGroup && s_cell[e] == s_cell[l]) ++e;
        grp[1 + n++] = l | ((e - l) << 16);
        l = e;
      }
      grp[0] = n;
    }
  }

  if (m.mode != kTransmission) return;
  if constexpr (sizeof(Real) == 8) {
    double* pm = w.pm64 + (size_t)b * Lp * Lp;
    for (int e = tid; e < Lp * Lp; e += kBlock) {
      int i = e / Lp, l = e % Lp;
      pm[e] = (i < L && l < L) ? path_entry(s_r, s_dr, i, l) : 0.0;
    }
  } else {
    // bf16 hi/lo A-operand fragments of v_mfma_f32_32x32x16_bf16:
    // lane holds row 32*mi + lane%32, columns 16*kb + 8*(lane/32) + j, j = 0..7
    const int MB = Lp / 32, KB = Lp / 16;
    const size_t plane = (size_t)MB * KB * 512;
    uint16_t* fh = w.pfrag + (size_t)b * 2 * plane;
    uint16_t* fl = fh + plane;
    // the transposed fragments serve only the adjoint; a forward-only workspace has none
    uint16_t* th_ = w.ptfrag ? w.ptfrag + (size_t)b * 2 * plane : nullptr;
    uint16_t* tl_ = th_ ? th_ + plane : nullptr;
    for (int e = tid; e < MB * KB * 64; e += kBlock) {
      const int lane = e & 63, kb = (e >> 6) % KB, mi = (e >> 6) / KB;
      const int row = 32 * mi + (lane & 31);
      const int col0 = 16 * kb + 8 * (lane >> 5);
      uint16_t hv[8], lv[8], thv[8], tlv[8];
      for (int j = 0; j < 8; ++j) {
        const int col = col0 + j;
        // P[row][col] for the forward product, P[col][row] (transpose) for the adjoint
        double v = (row < L && col < L) ? path_entry(s_r, s_dr, row, col) : 0.0;
        double vt = (row < L && col < L) ? path_entry(s_r, s_dr, col, row) : 0.0;
        hv[j] = bf16_rn((float)v);
        lv[j] = bf16_rn((float)(v - (double)bf16_to_f(hv[j])));
        thv[j] = bf16_rn((float)vt);
        tlv[j] = bf16_rn((float)(vt - (double)bf16_to_f(thv[j])));
      }
      const size_t off = (size_t)e * 8;
      for (int j = 0; j < 8; ++j) {
        fh[off + j] = hv[j];
        fl[off + j] = lv[j];
      }
      if (th_)
        for (int j = 0; j < 8; ++j) {
          th_[off + j] = thv[j];
          tl_[off + j] = tlv[j];
        }
    }
  }
}

// Non-grey cloud, reduced precision: Q_ext and its derivatives once per (sample,
// wavenumber), read by the forward kernel (Q_ext) and the layer sums (both).
// One thread per wavenumber; grid (n_nu_pad / kBlock, B).
__global__ __launch_bounds__(kBlock) void k_cloud_q(Model m, Work w) {
  const int b = blockIdx.y;
  const int nu = blockIdx.x * kBlock + threadIdx.x;
  if (nu >= m.n_nu_pad || w.status[b]) return;
  float dq[kCloudSpec];
  const float q = cloud_q<float>(m.cloud_qext, load_cloud<float>(w.cloud + (size_t)b * kCloudSpec), (float)m.nu[nu], dq);
  float* out = w.cloud_q + (size_t)b * (1 + kCloudSpec) * m.n_nu_pad + nu;
  out[0] = q;
#pragma unroll
  for (int k = 0; k < kCloudSpec; ++k) out[(size_t)(1 + k) * m.n_nu_pad] = dq[k];
}

// Layer-count classes of the call: class 0 holds the samples of at most kShortLayers
// layers (and invalid samples, which the kernels skip), class 1 the rest; each list is
// ordered longest first (ties by sample index), so the most expensive work items start
// first.  One workgroup; a sample's rank counts the samples ahead of it in its class.
__global__ __launch_bounds__(kBlock) void k_layer_classes(Work w, int B) {
  for (int b = threadIdx.x; b < B; b += kBlock) {
    const int lb = w.status[b] ? 0 : w.nlay[b];
    const int cb = lb > kShortLayers ? 1 : 0;
    int rank = 0;
    for (int q = 0; q < B; ++q) {
      const int lq = w.status[q] ? 0 : w.nlay[q];
      if ((lq > kShortLayers ? 1 : 0) == cb && (lq > lb || (lq == lb && q < b))) ++rank;
    }
    w.cls[2 + cb * B + rank] = b;
  }
  if (threadIdx.x < 2) {
    int n = 0;
    for (int q = 0; q < B; ++q) {
      const int lq = w.status[q] ? 0 : w.nlay[q];
      n += (lq > kShortLayers ? 1 : 0) == (int)threadIdx.x;
    }
    w.cls[threadIdx.x] = n;
  }
}

void launch_layer_classes(const Model& m, const Work& w, int B, hipStream_t st) {
  (void)m;
  hipLaunchKernelGGL(k_layer_classes, dim3(1), dim3(kBlock), 0, st, w, B);
}

void launch_profile(const Model& m, const Work& w, int B, const double* params, const int32_t* n_layers,
                    bool fp64, hipStream_t st) {
  if (fp64) {
    hipLaunchKernelGGL(k_profile<double>, dim3(B), dim3(kBlock), 0, st, m, w, params, n_layers);
  } else {
    hipLaunchKernelGGL(k_profile<float>, dim3(B), dim3(kBlock), 0, st, m, w, params, n_layers);
    if (m.cloud_ng)
      hipLaunchKernelGGL(k_cloud_q, dim3((unsigned)((m.n_nu_pad + kBlock - 1) / kBlock), (unsigned)B), dim3(kBlock), 0,
                         st, m, w);
  }
}

}  // namespace exofwd
