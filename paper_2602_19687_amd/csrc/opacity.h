// Per-layer opacity evaluation shared by the transmission forward and adjoint
// kernels.  A wave evaluates one layer at a time (all per-layer data are
// wave-uniform and live in SGPRs); lanes run along wavenumber.
//
// Reduced-precision form, two adjacent wavenumbers per lane:
//   dtau = D + R nu4 + sum_s 2^(c_s + bilinear(h_s) + lam_s) + sum_pairs 2^(c_p + lerp_T(h_p) + lam_p)
// with FP16 table entries h = log2 sigma - c (c per source and wavenumber),
// bilinear weights in (T, log p), lam = log2 of the layer prefactor
// (n X dr for lines, n^2 X X dr for CIA), R the Rayleigh and D the cloud term.
#pragma once
#include "common.h"

namespace exofwd {

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

__device__ inline float exp2_fast(float x) { return __builtin_amdgcn_exp2f(x); }

// Wave-uniform data of one (sample, layer).
template <int S>
struct LayerCoef {
  uint32_t row[S];      // byte offset of the (s, iT, iP) table row at the tile start
  uint32_t rowc[2];     // byte offset of the (pair, iTc) CIA row at the tile start
  float w00, w10, w01, w11, wtc, R, D;
  float lam[S], lamc[2];
  float wt, inv_dt, inv_dtc;   // used by the adjoint (T derivative of the weights)
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
  const float* rl = rec + (size_t)l * rec_len(S);
  const float wt = rl[0], wp = rl[1];
  c.wt = wt;
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

__device__ inline half2_t load_h2(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(half2_t, (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

// Line and CIA terms of one layer for two wavenumbers.  Terms and the
// T-weight derivatives of their exponents are returned per source when
// requested (the adjoint); the forward only needs the sums.
template <int S, bool CIA, bool DERIV>
__device__ inline void layer_terms(const LayerCoef<S>& c, const LaneConst<S>& k, const TableGeom& g,
                                   __amdgpu_buffer_rsrc_t rh, __amdgpu_buffer_rsrc_t rhc, uint32_t voff,
                                   float& d0, float& d1, float* t0 = nullptr, float* t1 = nullptr,
                                   float* dw0 = nullptr, float* dw1 = nullptr) {
  d0 = fmaf(c.R, k.nu4_0, c.D);
  d1 = fmaf(c.R, k.nu4_1, c.D);
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const half2_t h00 = load_h2(rh, voff, c.row[s]);
    const half2_t h10 = load_h2(rh, voff, c.row[s] + g.tstep);
    const half2_t h01 = load_h2(rh, voff, c.row[s] + g.pstep);
    const half2_t h11 = load_h2(rh, voff, c.row[s] + g.tstep + g.pstep);
    float v0 = k.c0[s] + c.lam[s];
    float v1 = k.c1[s] + c.lam[s];
    v0 = fmaf(c.w00, (float)h00.x, v0);
    v1 = fmaf(c.w00, (float)h00.y, v1);
    v0 = fmaf(c.w10, (float)h10.x, v0);
    v1 = fmaf(c.w10, (float)h10.y, v1);
    v0 = fmaf(c.w01, (float)h01.x, v0);
    v1 = fmaf(c.w01, (float)h01.y, v1);
    v0 = fmaf(c.w11, (float)h11.x, v0);
    v1 = fmaf(c.w11, (float)h11.y, v1);
    const float e0 = exp2_fast(v0), e1 = exp2_fast(v1);
    d0 += e0;
    d1 += e1;
    if (DERIV) {
      t0[s] = e0;
      t1[s] = e1;
      // d(exponent)/d wT = (1 - wP)(h10 - h00) + wP (h11 - h01) = (w00 + w10)... expressed with the weights:
      // wP = w01 + w11, 1 - wP = w00 + w10
      const float omp = c.w00 + c.w10, wp = c.w01 + c.w11;
      dw0[s] = omp * ((float)h10.x - (float)h00.x) + wp * ((float)h11.x - (float)h01.x);
      dw1[s] = omp * ((float)h10.y - (float)h00.y) + wp * ((float)h11.y - (float)h01.y);
    }
  }
  if (CIA) {
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const half2_t a = load_h2(rhc, voff, c.rowc[p]);
      const half2_t b = load_h2(rhc, voff, c.rowc[p] + g.row_bytes);
      float v0 = k.cc0[p] + c.lamc[p];
      float v1 = k.cc1[p] + c.lamc[p];
      v0 = fmaf(1.0f - c.wtc, (float)a.x, v0);
      v1 = fmaf(1.0f - c.wtc, (float)a.y, v1);
      v0 = fmaf(c.wtc, (float)b.x, v0);
      v1 = fmaf(c.wtc, (float)b.y, v1);
      const float e0 = exp2_fast(v0), e1 = exp2_fast(v1);
      d0 += e0;
      d1 += e1;
      if (DERIV) {
        t0[S + p] = e0;
        t1[S + p] = e1;
        dw0[S + p] = (float)b.x - (float)a.x;
        dw1[S + p] = (float)b.y - (float)a.y;
      }
    }
  }
}

__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void* p, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)(bytes > 0x7fffffffu ? 0x7fffffff : bytes),
                                           0x00020000);
}

// Round to nearest even bf16 and back (finite inputs).
__device__ inline uint16_t bf16_bits_rn(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf16_bits_to_f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

}  // namespace exofwd

namespace exofwd {

// ---- one wavenumber per lane (reverse kernel tiles of 64)
template <int S>
struct LaneConst1 {
  float c[S], cc[2], nu4;
};

template <int S, bool CIA>
__device__ inline LaneConst1<S> load_lane1(const Model& m, const Tables& tb, int nu) {
  LaneConst1<S> k;
  const size_t np = (size_t)m.n_nu_pad;
#pragma unroll
  for (int s = 0; s < S; ++s) k.c[s] = tb.c[s * np + nu];
#pragma unroll
  for (int p = 0; p < 2; ++p) k.cc[p] = CIA ? tb.cc[p * np + nu] : 0.0f;
  k.nu4 = tb.nu4f[nu];
  return k;
}

__device__ inline float load_h1(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return (float)__builtin_bit_cast(_Float16, (unsigned short)__builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
}

// Vertical optical depth of one layer at one wavenumber per lane.
template <int S, bool CIA>
__device__ inline float layer_dtau1(const LayerCoef<S>& c, const LaneConst1<S>& k, const TableGeom& g,
                                    __amdgpu_buffer_rsrc_t rh, __amdgpu_buffer_rsrc_t rhc, uint32_t voff) {
  float d = fmaf(c.R, k.nu4, c.D);
#pragma unroll
  for (int s = 0; s < S; ++s) {
    float v = k.c[s] + c.lam[s];
    v = fmaf(c.w00, load_h1(rh, voff, c.row[s]), v);
    v = fmaf(c.w10, load_h1(rh, voff, c.row[s] + g.tstep), v);
    v = fmaf(c.w01, load_h1(rh, voff, c.row[s] + g.pstep), v);
    v = fmaf(c.w11, load_h1(rh, voff, c.row[s] + g.tstep + g.pstep), v);
    d += exp2_fast(v);
  }
  if (CIA) {
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      float v = k.cc[p] + c.lamc[p];
      v = fmaf(1.0f - c.wtc, load_h1(rhc, voff, c.rowc[p]), v);
      v = fmaf(c.wtc, load_h1(rhc, voff, c.rowc[p] + g.row_bytes), v);
      d += exp2_fast(v);
    }
  }
  return d;
}

// bf16x8 hi/lo split of eight consecutive floats
__device__ inline void split8(const float* p, bf16x8& hi, bf16x8& lo) {
  const float4 a = *reinterpret_cast<const float4*>(p);
  const float4 b = *reinterpret_cast<const float4*>(p + 4);
  const float v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
  uint32_t h[4], l[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint16_t h0 = bf16_bits_rn(v[2 * i]), h1 = bf16_bits_rn(v[2 * i + 1]);
    const uint16_t l0 = bf16_bits_rn(v[2 * i] - bf16_bits_to_f(h0));
    const uint16_t l1 = bf16_bits_rn(v[2 * i + 1] - bf16_bits_to_f(h1));
    h[i] = (uint32_t)h0 | ((uint32_t)h1 << 16);
    l[i] = (uint32_t)l0 | ((uint32_t)l1 << 16);
  }
  hi = __builtin_bit_cast(bf16x8, make_uint4(h[0], h[1], h[2], h[3]));
  lo = __builtin_bit_cast(bf16x8, make_uint4(l[0], l[1], l[2], l[3]));
}

}  // namespace exofwd
