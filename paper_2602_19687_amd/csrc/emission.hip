// Emission forward kernel: per (sample, 64-wavenumber tile) the vertical
// optical depth of every layer (pure absorption: line tables and CIA), the
// Planck intensity at every level, the upward linear-in-tau intensity sweep
// for each Gauss-Legendre angle and the planet/star flux ratio (Eq. 45).
// One thread owns one (wavenumber, angle) pair during the sweep.
#include "emission.h"
#include "kernels.h"

namespace exofwd {

__device__ inline float opacity_mixed_e(const Model& m, const Tables& tb, int cells, const float* __restrict__ rl,
                                        int nu, const float* cs, const float* ccs) {
  const int it = cells & 255, ip = (cells >> 8) & 255, itc = cells >> 16;
  const float wt = rl[0], wp = rl[1];
  const float w11 = wt * wp, w10 = wt - w11, w01 = wp - w11, w00 = 1.0f - wt - wp + w11;
  const size_t npad = (size_t)m.n_nu_pad;
  float acc = 0.0f;
  const _Float16* __restrict__ h = reinterpret_cast<const _Float16*>(tb.h);
  for (int s = 0; s < m.S; ++s) {
    const _Float16* p = h + (((size_t)s * m.n_t + it) * m.n_p + ip) * npad + nu;
    float v = cs[s] + rl[kRecFixed + s];
    v = fmaf(w00, (float)p[0], v);
    v = fmaf(w10, (float)p[(size_t)m.n_p * npad], v);
    v = fmaf(w01, (float)p[npad], v);
    v = fmaf(w11, (float)p[(size_t)(m.n_p + 1) * npad], v);
    acc += exp2f(v);
  }
  if (m.has_cia) {
    const float wtc = rl[2];
    const _Float16* __restrict__ hc = reinterpret_cast<const _Float16*>(tb.hc);
    for (int c = 0; c < 2; ++c) {
      const _Float16* p = hc + ((size_t)c * m.n_tc + itc) * npad + nu;
      float v = ccs[c] + rl[5 + c];
      v = fmaf(1.0f - wtc, (float)p[0], v);
      v = fmaf(wtc, (float)p[npad], v);
      acc += exp2f(v);
    }
  }
  return acc;
}

__device__ inline double opacity_fp64_e(const Model& m, const Tables& tb, int cells, const double* __restrict__ rl,
                                        int nu) {
  const int it = cells & 255, ip = (cells >> 8) & 255, itc = cells >> 16;
  const double wt = rl[0], wp = rl[1];
  const size_t npad = (size_t)m.n_nu_pad;
  double acc = 0.0;
  for (int s = 0; s < m.S; ++s) {
    const double* p = tb.t64 + (((size_t)s * m.n_t + it) * m.n_p + ip) * npad + nu;
    const double v = (1.0 - wt) * (1.0 - wp) * p[0] + wt * (1.0 - wp) * p[(size_t)m.n_p * npad] +
                     (1.0 - wt) * wp * p[npad] + wt * wp * p[(size_t)(m.n_p + 1) * npad];
    acc += exp2(v * kLog2_10 + rl[kRecFixed + s]);
  }
  if (m.has_cia) {
    const double wtc = rl[2];
    for (int c = 0; c < 2; ++c) {
      const double* p = tb.tc64 + ((size_t)c * m.n_tc + itc) * npad + nu;
      acc += exp2(((1.0 - wtc) * p[0] + wtc * p[npad]) * kLog2_10 + rl[5 + c]);
    }
  }
  return acc;
}

// Planck intensity per unit wavenumber: 2 h c^2 nu^3 / (exp(h c nu / k T) - 1)
template <typename Real>
__device__ inline Real planck(Real t, Real nu) {
  const Real c1 = Real(2.0 * kHpl * kC * kC);
  const Real c2 = Real(kHpl * kC / kB);
  if constexpr (sizeof(Real) == 8) return c1 * nu * nu * nu / expm1(c2 * nu / t);
  else return c1 * nu * nu * nu / expm1f(c2 * nu / t);
}

// (1 - e^-x)/x - e^-x: Taylor series where cancellation would cost digits
template <typename Real>
__device__ inline Real lin_source(Real x, Real e) {
  if constexpr (sizeof(Real) == 8) {
    if (x < 1.0e-4) return x * (0.5 + x * (-1.0 / 3.0 + x * (0.125 + x * (-1.0 / 30.0))));
    return -expm1(-x) / x - e;
  } else {
    if (x < 0.1f)
      return x * (0.5f + x * (-1.0f / 3.0f + x * (0.125f + x * (-1.0f / 30.0f + x * (1.0f / 144.0f + x * (-1.0f / 840.0f))))));
    return (1.0f - e) / x - e;
  }
}

template <typename Real>
__global__ __launch_bounds__(kBlock) void k_emission(Model m, Work w, Tables tb, int B, Real* __restrict__ spec) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int logical = xcd_logical_block(blockIdx.x, gridDim.x);
  const int b = logical % B, tile = logical / B;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int Lp = m.L_pad;
  const int nu0 = tile * kTile64;
  Real* out = spec + (size_t)b * m.n_nu;
  if (w.status[b]) {
    if (tid < kTile64 && nu0 + tid < m.n_nu) out[nu0 + tid] = Real(NAN);
    return;
  }
  const int L = w.nlay[b];
  Real* s_dt = reinterpret_cast<Real*>(lds);          // [Lp][64]
  Real* s_b = s_dt + (size_t)Lp * kTile64;            // [Lp+1][64] Planck at levels
  Real* s_f = s_b + (size_t)(Lp + 1) * kTile64;       // [4][64] flux partials
  const int RL = rec_len(m.S);
  const Real* rec = reinterpret_cast<const Real*>(w.rec) + (size_t)b * Lp * RL;
  const int32_t* cells = w.cells + (size_t)b * Lp;
  const int nu = nu0 + lane;
  const double* t_lev = w.t_lev + (size_t)b * (Lp + 1);
  const Real nuv = Real(m.nu[nu]);
  if constexpr (sizeof(Real) == 4) {
    float cs[kMaxSpecies], ccs[2] = {0.0f, 0.0f};
    for (int s = 0; s < m.S; ++s) cs[s] = tb.c[(size_t)s * m.n_nu_pad + nu];
    if (m.has_cia) {
      ccs[0] = tb.cc[nu];
      ccs[1] = tb.cc[(size_t)m.n_nu_pad + nu];
    }
    for (int l = wv; l < L; l += 4) s_dt[l * kTile64 + lane] = opacity_mixed_e(m, tb, cells[l], rec + (size_t)l * RL, nu, cs, ccs);
  } else {
    for (int l = wv; l < L; l += 4) s_dt[l * kTile64 + lane] = opacity_fp64_e(m, tb, cells[l], rec + (size_t)l * RL, nu);
  }
  for (int j = wv; j <= L; j += 4) s_b[j * kTile64 + lane] = planck<Real>(Real(t_lev[j]), nuv);
  __syncthreads();

  // upward sweep, one (wavenumber, angle) per thread
  Real flux = Real(0);
  for (int k = wv; k < m.n_mu; k += 4) {
    const Real mu = Real(m.mu_nodes[k]);
    const Real inv_mu = Real(1) / mu;
    Real inten = s_b[lane];
    for (int l = 0; l < L; ++l) {
      const Real x = s_dt[l * kTile64 + lane] * inv_mu;
      Real e;
      if constexpr (sizeof(Real) == 8) e = exp(-x); else e = __expf(-x);
      const Real bb = s_b[l * kTile64 + lane], bt = s_b[(l + 1) * kTile64 + lane];
      inten = inten * e + bt * (Real(1) - e) + (bb - bt) * lin_source<Real>(x, e);
    }
    flux += Real(2.0 * M_PI * m.mu_weights[k]) * mu * inten;
  }
  s_f[wv * kTile64 + lane] = flux;
  __syncthreads();
  if (tid < kTile64 && nu0 + tid < m.n_nu) {
    const Real f = (s_f[tid] + s_f[kTile64 + tid]) + (s_f[2 * kTile64 + tid] + s_f[3 * kTile64 + tid]);
    const Real fstar = Real(M_PI) * planck<Real>(Real(m.t_star), Real(m.nu[nu0 + tid]));
    out[nu0 + tid] = Real(m.dilution) * f / fstar * Real(w.core[b]);
  }
}

size_t emission_lds_bytes(const Model& m, bool fp64) {
  const size_t rs = fp64 ? 8 : 4;
  return rs * ((size_t)m.L_pad * kTile64 + (size_t)(m.L_pad + 1) * kTile64 + 4 * kTile64);
}

hipError_t emission_configure(const Model& m, bool fp64) {
  const size_t bytes = emission_lds_bytes(m, fp64);
  if (bytes > 160 * 1024) return hipErrorInvalidValue;
  if (fp64) return hipFuncSetAttribute((const void*)k_emission<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  return hipFuncSetAttribute((const void*)k_emission<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

void launch_emission(const Model& m, const Work& w, const Tables& tb, int B, void* spec, bool fp64, hipStream_t st) {
  const dim3 grid((unsigned)(m.n_tiles64 * B));
  const size_t lds = emission_lds_bytes(m, fp64);
  if (fp64)
    hipLaunchKernelGGL(k_emission<double>, grid, dim3(kBlock), lds, st, m, w, tb, B, (double*)spec);
  else
    hipLaunchKernelGGL(k_emission<float>, grid, dim3(kBlock), lds, st, m, w, tb, B, (float*)spec);
}

}  // namespace exofwd
