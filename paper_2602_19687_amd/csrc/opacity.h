// Per-layer opacity evaluation shared by the transmission forward and adjoint
// kernels.  A wave evaluates one layer at a time (all per-layer data are
// wave-uniform and live in SGPRs); lanes run along wavenumber.
//
// Reduced-precision form, two adjacent wavenumbers per lane:
//   dtau = D + R nu4 + sum_s 2^(c_s + bilinear(h_s) + lam_s) + sum_pairs 2^(c_p + lerp_T(h_p) + lam_p)
// with FP16 table entries h = log2 sigma - c (c per source and wavenumber),
// bilinear weights in (T, log p), lam = log2 of the layer prefactor
// (n X dr for lines, n^2 X X dr for CIA), R the Rayleigh and D the cloud term
// (the non-grey cloud's D is a column that multiplies Q_ext(nu)).
#pragma once
#include "common.h"

namespace exofwd {

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

__device__ inline float exp2_fast(float x) { return __builtin_amdgcn_exp2f(x); }

// 1 - e^-tau given e = e^-tau: below tau = 1/64, where 1 - e keeps too few digits
// of a thin chord's absorption in FP32, the series tau (1 - tau/2 + tau^2/6)
// (truncation tau^3/24 relative, under 2e-7)
__device__ inline float one_minus_exp(float tau, float e) {
  return tau < 0.015625f ? tau * (1.0f - tau * (0.5f - tau * (1.0f / 6.0f))) : 1.0f - e;
}

// Wave-uniform data of one (sample, layer).
template <int S>
struct LayerCoef {
  uint32_t row[S];      // byte offset of the (s, iT, iP) table row at the tile start
  uint32_t rowc[2];     // byte offset of the (pair, iTc) CIA row at the tile start
  float w00, w10, w01, w11, wtc, R, D;
  float lam[S], lamc[2];
  float col[S];        // line prefactors n X_s dr (2^lam)
  float wt, wp, omp;   // T and log p weights, 1 - wP (derivative form of the bilinear)
  int cell;            // packed (iT, iP, iTc): equal cells read equal table pairs
};

struct TableGeom {
  uint32_t row_bytes;   // n_nu_pad * 2
  uint32_t tstep;       // bytes from iT to iT+1
  uint32_t pstep;       // bytes from iP to iP+1
};

template <int S>
__device__ inline LayerCoef<S> load_layer(const Model& m, const int32_t* __restrict__ cells,
                                          const float* __restrict__ rec, int l, uint32_t nu0_bytes,
                                          const TableGeom& g) {
  LayerCoef<S> c;
  const int cl = cells[l];
  const int it = cl & 255, ip = (cl >> 8) & 255, itc = cl >> 16;
  c.cell = cl;
  const float* rl = rec + (size_t)l * rec_len_wide(S);
  const float wt = rl[0], wp = rl[1];
  c.wt = wt;
  c.wp = wp;
  c.omp = 1.0f - wp;
  c.w11 = wt * wp;
  c.w10 = wt - c.w11;
  c.w01 = wp - c.w11;
  c.w00 = 1.0f - wt - wp + c.w11;
  c.wtc = rl[2];
  c.R = rl[3];
  c.D = rl[4];
  c.lamc[0] = rl[5];
  c.lamc[1] = rl[6];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    c.lam[s] = rl[kRecFixed + s];
    c.col[s] = rl[kRecFixed + S + s];
    c.row[s] = (uint32_t)(((s * m.n_t + it) * m.n_p + ip)) * g.row_bytes + nu0_bytes;
  }
#pragma unroll
  for (int p = 0; p < 2; ++p) c.rowc[p] = (uint32_t)(p * m.n_tc + itc) * g.row_bytes + nu0_bytes;
  return c;
}

// Per-lane constants for two adjacent wavenumbers.
template <int S>
struct LaneConst {
  float c0[S], c1[S], cc0[2], cc1[2], nu4_0, nu4_1;
};

template <int S, bool CIA>
__device__ inline LaneConst<S> load_lane(const Model& m, const Tables& tb, int nu) {
  LaneConst<S> k;
  const size_t np = (size_t)m.n_nu_pad;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const float2 c = *reinterpret_cast<const float2*>(tb.c + s * np + nu);
    k.c0[s] = c.x;
    k.c1[s] = c.y;
  }
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    if (CIA) {
      const float2 c = *reinterpret_cast<const float2*>(tb.cc + p * np + nu);
      k.cc0[p] = c.x;
      k.cc1[p] = c.y;
    } else {
      k.cc0[p] = k.cc1[p] = 0.0f;
    }
  }
  const float2 n4 = *reinterpret_cast<const float2*>(tb.nu4f + nu);
  k.nu4_0 = n4.x;
  k.nu4_1 = n4.y;
  return k;
}

__device__ inline float load_f32(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ inline half2_t load_h2(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(half2_t, (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

// Raw FP16 table pairs of one layer: four bilinear corners per line source,
// two T rows per CIA pair.
template <int S, bool CIA>
struct LayerRaw {
  half2_t h[4 * S + (CIA ? 4 : 0)];
};

template <int S, bool CIA>
__device__ inline void fetch_terms(const LayerCoef<S>& c, const TableGeom& g, __amdgpu_buffer_rsrc_t rh,
                                   __amdgpu_buffer_rsrc_t rhc, uint32_t voff, LayerRaw<S, CIA>& r) {
#pragma unroll
  for (int s = 0; s < S; ++s) {
    r.h[4 * s + 0] = load_h2(rh, voff, c.row[s]);
    r.h[4 * s + 1] = load_h2(rh, voff, c.row[s] + g.tstep);
    r.h[4 * s + 2] = load_h2(rh, voff, c.row[s] + g.pstep);
    r.h[4 * s + 3] = load_h2(rh, voff, c.row[s] + g.tstep + g.pstep);
  }
  if constexpr (CIA) {
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      r.h[4 * S + 2 * p] = load_h2(rhc, voff, c.rowc[p]);
      r.h[4 * S + 2 * p + 1] = load_h2(rhc, voff, c.rowc[p] + g.row_bytes);
    }
  }
}

// Optical depth of one layer at two wavenumbers from its fetched table pairs:
// Rayleigh + cloud, the VMR-weighted line terms (bilinear in T and log p of the
// log2 tables) and the CIA pair terms (linear in T).
// With the non-grey cloud (NGC) D is the layer's cloud column and q0, q1 the
// extinction efficiency Q_ext at the two wavenumbers.
template <int S, bool CIA, bool NGC = false>
__device__ inline void eval_terms(const LayerCoef<S>& c, const LaneConst<S>& k, const LayerRaw<S, CIA>& r, float& d0,
                                  float& d1, float q0 = 1.0f, float q1 = 1.0f) {
  if constexpr (NGC) {
    d0 = fmaf(c.D, q0, c.R * k.nu4_0);
    d1 = fmaf(c.D, q1, c.R * k.nu4_1);
  } else {
    d0 = fmaf(c.R, k.nu4_0, c.D);
    d1 = fmaf(c.R, k.nu4_1, c.D);
  }
  // line terms: the cross-section (log2 sigma = c + the interpolated entry) times the
  // layer's prefactor, which then costs no add to the exponent
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const half2_t h00 = r.h[4 * s], h10 = r.h[4 * s + 1], h01 = r.h[4 * s + 2], h11 = r.h[4 * s + 3];
    float v0 = fmaf(c.w00, (float)h00.x, k.c0[s]);
    float v1 = fmaf(c.w00, (float)h00.y, k.c1[s]);
    v0 = fmaf(c.w10, (float)h10.x, v0);
    v1 = fmaf(c.w10, (float)h10.y, v1);
    v0 = fmaf(c.w01, (float)h01.x, v0);
    v1 = fmaf(c.w01, (float)h01.y, v1);
    v0 = fmaf(c.w11, (float)h11.x, v0);
    v1 = fmaf(c.w11, (float)h11.y, v1);
    d0 = fmaf(c.col[s], exp2_fast(v0), d0);
    d1 = fmaf(c.col[s], exp2_fast(v1), d1);
  }
  if constexpr (CIA) {
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const half2_t a = r.h[4 * S + 2 * p], b = r.h[4 * S + 2 * p + 1];
      float v0 = k.cc0[p] + c.lamc[p];
      float v1 = k.cc1[p] + c.lamc[p];
      v0 = fmaf(1.0f - c.wtc, (float)a.x, v0);
      v1 = fmaf(1.0f - c.wtc, (float)a.y, v1);
      v0 = fmaf(c.wtc, (float)b.x, v0);
      v1 = fmaf(c.wtc, (float)b.y, v1);
      d0 += exp2_fast(v0);
      d1 += exp2_fast(v1);
    }
  }
}

// Fetch and evaluate in one step.
template <int S, bool CIA, bool NGC = false>
__device__ inline void layer_terms(const LayerCoef<S>& c, const LaneConst<S>& k, const TableGeom& g,
                                   __amdgpu_buffer_rsrc_t rh, __amdgpu_buffer_rsrc_t rhc, uint32_t voff,
                                   float& d0, float& d1, float q0 = 1.0f, float q1 = 1.0f) {
  LayerRaw<S, CIA> r;
  fetch_terms<S, CIA>(c, g, rh, rhc, voff, r);
  eval_terms<S, CIA, NGC>(c, k, r, d0, d1, q0, q1);
}

// Line and CIA terms of one layer for two wavenumbers together with the
// derivative of each exponent with respect to the T weight, from the two
// log p-interpolated rows u0 (at iT) and u1 (at iT+1), both offset by c + lam:
//   exponent = u0 + wT (u1 - u0),  d exponent / d wT = u1 - u0.
template <int S, bool CIA>
__device__ inline void eval_terms_deriv(const LayerCoef<S>& c, const LaneConst<S>& k, const LayerRaw<S, CIA>& r,
                                        float* t0, float* t1, float* dw0, float* dw1) {
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const half2_t h00 = r.h[4 * s], h10 = r.h[4 * s + 1], h01 = r.h[4 * s + 2], h11 = r.h[4 * s + 3];
    const float cl0 = k.c0[s] + c.lam[s], cl1 = k.c1[s] + c.lam[s];
    const float u00 = fmaf(c.omp, (float)h00.x, fmaf(c.wp, (float)h01.x, cl0));
    const float u10 = fmaf(c.omp, (float)h10.x, fmaf(c.wp, (float)h11.x, cl0));
    const float u01 = fmaf(c.omp, (float)h00.y, fmaf(c.wp, (float)h01.y, cl1));
    const float u11 = fmaf(c.omp, (float)h10.y, fmaf(c.wp, (float)h11.y, cl1));
    dw0[s] = u10 - u00;
    dw1[s] = u11 - u01;
    t0[s] = exp2_fast(fmaf(c.wt, dw0[s], u00));
    t1[s] = exp2_fast(fmaf(c.wt, dw1[s], u01));
  }
  if constexpr (CIA) {
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const half2_t a = r.h[4 * S + 2 * p], b = r.h[4 * S + 2 * p + 1];
      const float u0 = (float)a.x + (k.cc0[p] + c.lamc[p]);
      const float u1 = (float)a.y + (k.cc1[p] + c.lamc[p]);
      dw0[S + p] = (float)b.x - (float)a.x;
      dw1[S + p] = (float)b.y - (float)a.y;
      t0[S + p] = exp2_fast(fmaf(c.wtc, dw0[S + p], u0));
      t1[S + p] = exp2_fast(fmaf(c.wtc, dw1[S + p], u1));
    }
  }
}

template <int S, bool CIA>
__device__ inline void layer_terms_deriv(const LayerCoef<S>& c, const LaneConst<S>& k, const TableGeom& g,
                                         __amdgpu_buffer_rsrc_t rh, __amdgpu_buffer_rsrc_t rhc, uint32_t voff,
                                         float* t0, float* t1, float* dw0, float* dw1) {
  LayerRaw<S, CIA> r;
  fetch_terms<S, CIA>(c, g, rh, rhc, voff, r);
  eval_terms_deriv<S, CIA>(c, k, r, t0, t1, dw0, dw1);
}

__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void* p, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)(bytes > 0x7fffffffu ? 0x7fffffff : bytes),
                                           0x00020000);
}

typedef __attribute__((ext_vector_type(2))) float float2v;
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;

// A float as a packed (bf16 hi | bf16 lo << 16) pair, hi + lo ~ 16 significant
// bits; both roundings are the hardware's round-to-nearest-even conversion.
__device__ inline uint32_t pack_hl(float v) {
  const float hf = (float)(__bf16)v;
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((float2v){v, v - hf}, bf16x2));
}

// bf16 hi pair (a, b) and lo pair of two floats, each as one dword (a in the low half).
__device__ inline void split_pair(float a, float b, uint32_t& hp, uint32_t& lp) {
  hp = __builtin_bit_cast(uint32_t, __builtin_convertvector((float2v){a, b}, bf16x2));
  const float ha = __uint_as_float(hp << 16), hb = __uint_as_float(hp & 0xffff0000u);
  lp = __builtin_bit_cast(uint32_t, __builtin_convertvector((float2v){a - ha, b - hb}, bf16x2));
}

// hi and lo bf16x8 fragments from eight packed pairs
__device__ inline void frag_hl(const uint32_t* x, bf16x8& hi, bf16x8& lo) {
  uint32_t h[4], l[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    h[i] = __builtin_amdgcn_perm(x[2 * i + 1], x[2 * i], 0x05040100u);
    l[i] = __builtin_amdgcn_perm(x[2 * i + 1], x[2 * i], 0x07060302u);
  }
  hi = __builtin_bit_cast(bf16x8, make_uint4(h[0], h[1], h[2], h[3]));
  lo = __builtin_bit_cast(bf16x8, make_uint4(l[0], l[1], l[2], l[3]));
}

}  // namespace exofwd
