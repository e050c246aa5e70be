// Emission forward kernels: per (sample, 64-wavenumber tile) the vertical
// optical depth of every layer (pure absorption: line tables and CIA), the
// Planck intensity at every level, the upward linear-in-tau intensity sweep
// for each Gauss-Legendre angle and the planet/star flux ratio (Eq. 45).
// One thread owns one (wavenumber, angle) pair during the sweep.
//
// Reduced precision: the tables store log2 sigma - c as FP32, one 4-byte word
// per entry (24 significant bits, against 11 for the FP16 transmission tables):
// emitted flux is far more sensitive to opacity errors than the transit depth.
#include "emission.h"
#include "kernels.h"
#include "opacity.h"

namespace exofwd {

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

// plain FP64 path.  STAGED: the Planck intensities at the levels are staged in LDS
// with the layer optical depths (up to 128 padded layers); beyond, the LDS holds the
// optical depths alone and each angle's sweep forms the level intensities itself
// (the same values)
template <typename Real, bool STAGED>
__global__ __launch_bounds__(kBlock) void k_emission(Model m, Work w, Tables tb, int B, Real* __restrict__ spec,
                                                     Real* __restrict__ dtau_out) {
  static_assert(sizeof(Real) == 8, "the reduced-precision path is k_emission_mixed");
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
  Real* s_dt = reinterpret_cast<Real*>(lds);                        // [Lp][64]
  Real* s_b = s_dt + (size_t)Lp * kTile64;                          // [Lp+1][64] Planck at levels (STAGED)
  Real* s_f = s_b + (STAGED ? (size_t)(Lp + 1) * kTile64 : 0);      // [4][64] flux partials
  const int RL = rec_len(m.S);
  const Real* rec = reinterpret_cast<const Real*>(w.rec) + (size_t)b * Lp * RL;
  const int32_t* cells = w.cells + (size_t)b * Lp;
  const int nu = nu0 + lane;
  const double* t_lev = w.t_lev + (size_t)b * (Lp + 1);
  const Real nuv = Real(m.nu[nu]);
  for (int l = wv; l < L; l += 4) {
    s_dt[l * kTile64 + lane] = opacity_fp64_e(m, tb, cells[l], rec + (size_t)l * RL, nu);
    // the reverse pass reads the layer optical depths back
    if (dtau_out) dtau_out[((size_t)b * Lp + l) * m.n_nu_pad + nu] = s_dt[l * kTile64 + lane];
  }
  if constexpr (STAGED)
    for (int j = wv; j <= L; j += 4) s_b[j * kTile64 + lane] = planck<Real>(Real(t_lev[j]), nuv);
  __syncthreads();
  auto level_b = [&](int j) {
    if constexpr (STAGED) return s_b[j * kTile64 + lane];
    else return planck<Real>(Real(t_lev[j]), nuv);
  };

  // upward sweep, one (wavenumber, angle) per thread
  Real flux = Real(0);
  for (int k = wv; k < m.n_mu; k += 4) {
    const Real mu = Real(m.mu_nodes[k]);
    const Real inv_mu = Real(1) / mu;
    Real inten = level_b(0), bb = inten;
    for (int l = 0; l < L; ++l) {
      const Real x = s_dt[l * kTile64 + lane] * inv_mu;
      Real e;
      if constexpr (sizeof(Real) == 8) e = exp(-x); else e = __expf(-x);
      const Real bt = level_b(l + 1);
      // I e^-x + B_top (1 - e^-x) + (B_bot - B_top) src, as an increment of I
      inten += -expm1(-x) * (bt - inten) + (bb - bt) * lin_source<Real>(x, e);
      bb = bt;
    }
    flux += Real(2.0 * M_PI * m.mu_weights[k]) * mu * inten;
  }
  s_f[wv * kTile64 + lane] = flux;
  __syncthreads();
  if (tid < kTile64 && nu0 + tid < m.n_nu) {
    const Real f = (s_f[tid] + s_f[kTile64 + tid]) + (s_f[2 * kTile64 + tid] + s_f[3 * kTile64 + tid]);
    const Real fstar = m.has_bd ? Real(1) : Real(M_PI) * planck<Real>(Real(m.t_star), Real(m.nu[nu0 + tid]));
    out[nu0 + tid] = Real(m.dilution) * f / fstar * Real(w.core[b]);
  }
}


// reduced precision: one wave per (sample, 64-wavenumber tile), one wavenumber per
// lane, streaming up the layers: each layer's optical depth and its upper level's
// Planck intensity are formed where the angle sweeps need them, so nothing is
// staged in LDS and waves never wait for each other.  A workgroup holds four
// neighbouring tiles of one sample.
template <int S, bool CIA>
__global__ __launch_bounds__(kBlock) void k_emission_mixed(Model m, Work w, Tables tb, int B, float* __restrict__ spec,
                                                           float* __restrict__ dtau_out) {
  const int logical = xcd_logical_block(blockIdx.x, gridDim.x);
  const int b = logical % B;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tile = (logical / B) * 4 + wv;
  if (tile >= m.n_tiles64) return;
  const int nu0 = tile * kTile64, nu = nu0 + lane;
  float* out = spec + (size_t)b * m.n_nu;
  if (w.status[b]) {
    if (nu < m.n_nu) out[nu] = __builtin_nanf("");
    return;
  }
  const int L = w.nlay[b], Lp = m.L_pad;
  constexpr int RL = rec_len(S);
  const float* rec = reinterpret_cast<const float*>(w.rec) + (size_t)b * Lp * RL;
  const int32_t* cells = w.cells + (size_t)b * Lp;
  const double* t_lev = w.t_lev + (size_t)b * (Lp + 1);
  const double* inv_t = w.inv_tlev + (size_t)b * (Lp + 1);
  const size_t npad = (size_t)m.n_nu_pad;
  // FP32 tables: 4 bytes per (row, wavenumber)
  const uint32_t row_bytes = (uint32_t)npad * 4u, tstep = (uint32_t)m.n_p * row_bytes;
  const __amdgpu_buffer_rsrc_t rh = make_rsrc(tb.h, (size_t)S * m.n_t * m.n_p * npad * 4);
  const __amdgpu_buffer_rsrc_t rhc = make_rsrc(CIA ? (const void*)tb.hc : (const void*)tb.h,
                                               CIA ? (size_t)2 * m.n_tc * npad * 4 : 0);
  const uint32_t voff = (uint32_t)lane * 4u, nu0_bytes = (uint32_t)nu0 * 4u;
  float cs[S], ccs[2];
#pragma unroll
  for (int s2 = 0; s2 < S; ++s2) cs[s2] = tb.c[(size_t)s2 * npad + nu];
#pragma unroll
  for (int p = 0; p < 2; ++p) ccs[p] = CIA ? tb.cc[(size_t)p * npad + nu] : 0.0f;

  const double nud = m.nu[nu];
  const float c1n3 = (float)(2.0 * kHpl * kC * kC * nud * nud * nud);
  const double c2n_log2e = kHpl * kC / kB * 1.4426950408889634074 * nud;
  auto planck_at = [&](int j) {
    float y, em1;
    return planck_split(c1n3, c2n_log2e, inv_t[j], y, em1);
  };
  const int n_mu = m.n_mu;
  // the intensities accumulate in FP64: a hundred FP32 updates would leave ~1e-6 of
  // rounding in the flux, which the likelihood residuals near the best fit amplify
  float inv_mu[kMaxMu];
  double inten[kMaxMu];
  float b_bot = planck_at(0);
#pragma unroll
  for (int k = 0; k < kMaxMu; ++k) {
    inv_mu[k] = k < n_mu ? (float)(1.0 / m.mu_nodes[k]) : 0.0f;
    inten[k] = b_bot;
  }

  // table entries of the current cell: a layer in the same cell as the one below reuses them
  float tp[4 * S + 4];
  int cell_prev = -1;
  for (int l = 0; l < L; ++l) {
    // ---- optical depth of layer l
    const int cl = cells[l];
    const float* rl = rec + (size_t)l * RL;
    if (cl != cell_prev) {
      const int it = cl & 255, ip = (cl >> 8) & 255, itc = cl >> 16;
#pragma unroll
      for (int s2 = 0; s2 < S; ++s2) {
        const uint32_t row = (uint32_t)((s2 * m.n_t + it) * m.n_p + ip) * row_bytes + nu0_bytes;
        tp[4 * s2] = load_f32(rh, voff, row);
        tp[4 * s2 + 1] = load_f32(rh, voff, row + tstep);
        tp[4 * s2 + 2] = load_f32(rh, voff, row + row_bytes);
        tp[4 * s2 + 3] = load_f32(rh, voff, row + tstep + row_bytes);
      }
      if (CIA) {
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          const uint32_t row = (uint32_t)(p * m.n_tc + itc) * row_bytes + nu0_bytes;
          tp[4 * S + 2 * p] = load_f32(rhc, voff, row);
          tp[4 * S + 2 * p + 1] = load_f32(rhc, voff, row + row_bytes);
        }
      }
      cell_prev = cl;
    }
    const float wt = rl[0], wp = rl[1];
    const float w11 = wt * wp, w10 = wt - w11, w01 = wp - w11, w00 = 1.0f - wt - wp + w11;
    float d = 0.0f;
#pragma unroll
    for (int s2 = 0; s2 < S; ++s2) {
      const float p00 = tp[4 * s2], p10 = tp[4 * s2 + 1], p01 = tp[4 * s2 + 2], p11 = tp[4 * s2 + 3];
      float v = cs[s2] + rl[kRecFixed + s2];
      v = fmaf(w00, p00, v);
      v = fmaf(w10, p10, v);
      v = fmaf(w01, p01, v);
      v = fmaf(w11, p11, v);
      d += exp2_fast(v);
    }
    if (CIA) {
      const float wtc = rl[2];
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const float a = tp[4 * S + 2 * p], c2 = tp[4 * S + 2 * p + 1];
        float v = ccs[p] + rl[5 + p];
        v = fmaf(1.0f - wtc, a, v);
        v = fmaf(wtc, c2, v);
        d += exp2_fast(v);
      }
    }
    // the reverse pass reads the layer optical depths back
    if (dtau_out) __builtin_nontemporal_store(d, &dtau_out[((size_t)b * Lp + l) * npad + nu]);
    // ---- the sweep through layer l for every angle
    const float b_top = planck_at(l + 1);
    const float db = b_bot - b_top;
#pragma unroll
    for (int k = 0; k < kMaxMu; ++k) {
      if (k >= n_mu) break;
      const float x = d * inv_mu[k];
      const float e = exp2_fast(-1.4426950408889634f * x);
      float om, src;
      slab_terms(x, e, om, src);
      // I e^-x + B_top (1 - e^-x) + (B_bot - B_top) src, as an increment of I
      inten[k] = fma((double)om, (double)b_top - inten[k], fma((double)db, (double)src, inten[k]));
    }
    b_bot = b_top;
  }
  double flux = 0.0;
#pragma unroll
  for (int k = 0; k < kMaxMu; ++k)
    if (k < n_mu) flux = fma(2.0 * M_PI * m.mu_weights[k] * m.mu_nodes[k], inten[k], flux);
  if (nu < m.n_nu) {
    const double fstar =
        m.has_bd ? 1.0 : M_PI * 2.0 * kHpl * kC * kC * nud * nud * nud / expm1(kHpl * kC * nud / (kB * m.t_star));
    out[nu] = (float)(m.dilution * flux / fstar * w.core[b]);
  }
}

template <int S, bool CIA>
const void* emis_kernel() { return (const void*)k_emission_mixed<S, CIA>; }

const void* emis_kernel_for(int S, bool cia) {
#define EXOFWD_CASE(n) \
  case n: return cia ? emis_kernel<n, true>() : emis_kernel<n, false>();
  switch (S) {
    EXOFWD_CASE(1) EXOFWD_CASE(2) EXOFWD_CASE(3) EXOFWD_CASE(4)
    EXOFWD_CASE(5) EXOFWD_CASE(6) EXOFWD_CASE(7) EXOFWD_CASE(8)
  }
#undef EXOFWD_CASE
  return nullptr;
}

// FP64: level intensities staged with the optical depths up to 128 padded layers
static bool emis_staged(const Model& m) { return m.L_pad <= 128; }

static const void* emis_fp64_kernel(const Model& m) {
  return emis_staged(m) ? (const void*)k_emission<double, true> : (const void*)k_emission<double, false>;
}

size_t emission_lds_bytes(const Model& m, bool fp64) {
  if (!fp64) return 0;   // the reduced-precision kernel streams without LDS
  const size_t rs = 8;
  return rs * ((size_t)m.L_pad * kTile64 + (emis_staged(m) ? (size_t)(m.L_pad + 1) * kTile64 : 0) + 4 * kTile64);
}

hipError_t emission_configure(const Model& m, bool fp64) {
  const size_t bytes = emission_lds_bytes(m, fp64);
  if (bytes > 160 * 1024) return hipErrorInvalidValue;
  if (fp64) return hipFuncSetAttribute(emis_fp64_kernel(m), hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  const void* k = emis_kernel_for(m.S, m.has_cia);
  if (!k) return hipErrorInvalidValue;
  return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

void launch_emission(const Model& m, const Work& w, const Tables& tb, int B, void* spec, bool fp64, hipStream_t st,
                     void* dtau_out) {
  const size_t lds = emission_lds_bytes(m, fp64);
  if (fp64) {
    double* spec_d = (double*)spec;
    double* dtau_d = (double*)dtau_out;
    void* args[] = {(void*)&m, (void*)&w, (void*)&tb, (void*)&B, (void*)&spec_d, (void*)&dtau_d};
    hipLaunchKernel(emis_fp64_kernel(m), dim3((unsigned)(m.n_tiles64 * B)), dim3(kBlock), args, lds, st);
  } else {
    // four 64-wavenumber tiles (one per wave) of one sample per workgroup
    const dim3 grid((unsigned)((m.n_tiles64 + 3) / 4 * B));
    float* dtau_f = (float*)dtau_out;
    void* args[] = {(void*)&m, (void*)&w, (void*)&tb, (void*)&B, (void*)&spec, (void*)&dtau_f};
    hipLaunchKernel(emis_kernel_for(m.S, m.has_cia), grid, dim3(kBlock), args, lds, st);
  }
}

}  // namespace exofwd
