// Fused transmission forward kernel: per (sample, 64-wavenumber tile) it
// builds every layer's vertical optical depth from the interpolated
// cross-section tables, forms the slant optical depth through the path matrix
// (Eq. 44) and reduces it to the transit depth of each wavenumber.
//
// MIXED instance: FP16 log2-sigma tables with FP32 per-(species, nu) offsets,
// FP32 opacity (one exp2 per layer, species and wavenumber), chord product on
// v_mfma_f32_32x32x16_bf16 with a bf16 hi/lo split of both operands
// (hi*hi + hi*lo + lo*hi, FP32 accumulation).
// FP64 instance: FP64 tables and arithmetic, chord product on the FP64 VALU.
#include "kernels.h"

namespace exofwd {

__device__ inline uint16_t bf16_bits_rn(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf16_bits_to_f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Opacity of one (layer, wavenumber) element, reduced-precision form:
//   dtau = D + R nu4 + sum_s 2^(c_s + bilinear(h_s) + lam_s) + sum_pairs 2^(c_c + lerp_T(h_c) + lam_c)
__device__ inline float opacity_mixed(const Model& m, const Tables& tb, int cells, const float* __restrict__ rl,
                                      int nu, float nu4, const float* cs, const float* ccs) {
  const int it = cells & 255, ip = (cells >> 8) & 255, itc = cells >> 16;
  const float wt = rl[0], wp = rl[1];
  const float w11 = wt * wp, w10 = wt - w11, w01 = wp - w11, w00 = 1.0f - wt - wp + w11;
  const size_t npad = (size_t)m.n_nu_pad;
  float acc = fmaf(rl[3], nu4, rl[4]);
  const _Float16* __restrict__ h = reinterpret_cast<const _Float16*>(tb.h);
  for (int s = 0; s < m.S; ++s) {
    const _Float16* p = h + (((size_t)s * m.n_t + it) * m.n_p + ip) * npad + nu;
    const float h00 = (float)p[0];
    const float h01 = (float)p[npad];
    const float h10 = (float)p[(size_t)m.n_p * npad];
    const float h11 = (float)p[(size_t)(m.n_p + 1) * npad];
    float v = cs[s] + rl[kRecFixed + s];
    v = fmaf(w00, h00, v);
    v = fmaf(w10, h10, v);
    v = fmaf(w01, h01, v);
    v = fmaf(w11, h11, v);
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
  return fminf(acc, 16384.0f);
}

// The same element in FP64 from log10-sigma tables.
__device__ inline double opacity_fp64(const Model& m, const Tables& tb, int cells, const double* __restrict__ rl,
                                      int nu, double nu4) {
  const int it = cells & 255, ip = (cells >> 8) & 255, itc = cells >> 16;
  const double wt = rl[0], wp = rl[1];
  const size_t npad = (size_t)m.n_nu_pad;
  double acc = rl[3] * nu4 + rl[4];
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
      const double v = (1.0 - wtc) * p[0] + wtc * p[npad];
      acc += exp2(v * kLog2_10 + rl[5 + c]);
    }
  }
  return acc;
}

__global__ __launch_bounds__(kBlock) void k_trans_fwd_mixed(Model m, Work w, Tables tb, int B, float* __restrict__ spec) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int logical = xcd_logical_block(blockIdx.x, gridDim.x);
  const int b = logical % B, tile = logical / B;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int Lp = m.L_pad;
  const int nu0 = tile * kTileNu;
  float* out = spec + (size_t)b * m.n_nu;
  if (w.status[b]) {
    if (tid < kTileNu && nu0 + tid < m.n_nu) out[nu0 + tid] = __builtin_nanf("");
    return;
  }
  const int L = w.nlay[b];
  const int stride = Lp + 8;   // bf16 per wavenumber row of the B operand
  uint16_t* s_bhi = reinterpret_cast<uint16_t*>(lds);
  uint16_t* s_blo = s_bhi + kTileNu * stride;
  float* s_area = reinterpret_cast<float*>(s_blo + kTileNu * stride);
  float* s_red = s_area + Lp;   // [4][32]

  const float* area = reinterpret_cast<const float*>(w.area) + (size_t)b * Lp;
  for (int i = tid; i < Lp; i += kBlock) s_area[i] = area[i];

  // phase A: vertical optical depth of every layer, bf16 hi/lo into LDS
  const int RL = rec_len(m.S);
  const float* rec = reinterpret_cast<const float*>(w.rec) + (size_t)b * Lp * RL;
  const int32_t* cells = w.cells + (size_t)b * Lp;
  const int nu = nu0 + lane;
  const float nu4 = tb.nu4f[nu];
  float cs[kMaxSpecies], ccs[2];
  for (int s = 0; s < m.S; ++s) cs[s] = tb.c[(size_t)s * m.n_nu_pad + nu];
  ccs[0] = ccs[1] = 0.0f;
  if (m.has_cia) {
    ccs[0] = tb.cc[nu];
    ccs[1] = tb.cc[(size_t)m.n_nu_pad + nu];
  }
  const int KBe = (L + 15) >> 4;   // K blocks of 16 layers that hold real layers
  for (int o = wv; o < 2 * KBe; o += 4) {
    uint16_t hv[8], lv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int l = 8 * o + j;
      float dt = 0.0f;
      if (l < L) dt = opacity_mixed(m, tb, cells[l], rec + (size_t)l * RL, nu, nu4, cs, ccs);
      hv[j] = bf16_bits_rn(dt);
      lv[j] = bf16_bits_rn(dt - bf16_bits_to_f(hv[j]));
    }
    uint4 ph, pl;
    ph.x = hv[0] | ((uint32_t)hv[1] << 16); ph.y = hv[2] | ((uint32_t)hv[3] << 16);
    ph.z = hv[4] | ((uint32_t)hv[5] << 16); ph.w = hv[6] | ((uint32_t)hv[7] << 16);
    pl.x = lv[0] | ((uint32_t)lv[1] << 16); pl.y = lv[2] | ((uint32_t)lv[3] << 16);
    pl.z = lv[4] | ((uint32_t)lv[5] << 16); pl.w = lv[6] | ((uint32_t)lv[7] << 16);
    *reinterpret_cast<uint4*>(s_bhi + lane * stride + 8 * o) = ph;
    *reinterpret_cast<uint4*>(s_blo + lane * stride + 8 * o) = pl;
  }
  __syncthreads();

  // phase B: tau = P dtau on MFMA; wave pair (wv >> 1) takes a cost-balanced set of
  // 32-row blocks, wave parity (wv & 1) picks the 32-column half of the tile
  const int MBe = (L + 31) >> 5;
  const int KB = Lp >> 4;
  const int ni = wv & 1, pair = wv >> 1;
  unsigned mine = 0;
  {
    int c0 = 0, c1 = 0;
    for (int mi = 0; mi < MBe; ++mi) {
      const int cost = KBe - 2 * mi;
      if (c0 <= c1) { if (pair == 0) mine |= 1u << mi; c0 += cost; }
      else { if (pair == 1) mine |= 1u << mi; c1 += cost; }
    }
  }
  const size_t plane = (size_t)(Lp >> 5) * KB * 512;
  const uint16_t* fh = w.pfrag + (size_t)b * 2 * plane;
  const uint16_t* fl = fh + plane;
  const int col = 32 * ni + (lane & 31);
  const int khalf = 8 * (lane >> 5);
  float dsum = 0.0f;
  for (int mi = 0; mi < MBe; ++mi) {
    if (!(mine & (1u << mi))) continue;
    f32x16 acc = {};
    for (int kb = 2 * mi; kb < KBe; ++kb) {
      const size_t fo = ((size_t)(mi * KB + kb) * 64 + lane) * 8;
      const bf16x8 ah = *reinterpret_cast<const bf16x8*>(fh + fo);
      const bf16x8 al = *reinterpret_cast<const bf16x8*>(fl + fo);
      const bf16x8 bh = *reinterpret_cast<const bf16x8*>(s_bhi + col * stride + 16 * kb + khalf);
      const bf16x8 bl = *reinterpret_cast<const bf16x8*>(s_blo + col * stride + 16 * kb + khalf);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc, 0, 0, 0);
    }
    // phase C: annulus-weighted absorption 1 - e^-tau, summed over rows
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int row = 32 * mi + 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
      dsum = fmaf(s_area[row], 1.0f - __expf(-acc[j]), dsum);
    }
  }
  dsum += __shfl_xor(dsum, 32);
  if (lane < 32) s_red[wv * 32 + lane] = dsum;
  __syncthreads();
  if (tid < kTileNu) {
    const int h = tid >> 5, c = tid & 31;
    const float tot = s_red[h * 32 + c] + s_red[(h + 2) * 32 + c];
    if (nu0 + tid < m.n_nu) out[nu0 + tid] = (float)w.core[b] + tot;
  }
}

__global__ __launch_bounds__(kBlock) void k_trans_fwd_fp64(Model m, Work w, Tables tb, int B, double* __restrict__ spec) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int logical = xcd_logical_block(blockIdx.x, gridDim.x);
  const int b = logical % B, tile = logical / B;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int Lp = m.L_pad;
  const int nu0 = tile * kTileNu;
  double* out = spec + (size_t)b * m.n_nu;
  if (w.status[b]) {
    if (tid < kTileNu && nu0 + tid < m.n_nu) out[nu0 + tid] = __builtin_nan("");
    return;
  }
  const int L = w.nlay[b];
  double* s_dt = reinterpret_cast<double*>(lds);   // [Lp][64]
  double* s_red = s_dt + (size_t)Lp * kTileNu;     // [4][64]
  const int RL = rec_len(m.S);
  const double* rec = reinterpret_cast<const double*>(w.rec) + (size_t)b * Lp * RL;
  const int32_t* cells = w.cells + (size_t)b * Lp;
  const int nu = nu0 + lane;
  const double nu4 = tb.nu4d[nu];
  for (int l = wv; l < L; l += 4) s_dt[l * kTileNu + lane] = opacity_fp64(m, tb, cells[l], rec + (size_t)l * RL, nu, nu4);
  __syncthreads();
  const double* pm = w.pm64 + (size_t)b * Lp * Lp;
  const double* area = reinterpret_cast<const double*>(w.area) + (size_t)b * Lp;
  double dsum = 0.0;
  for (int i = wv; i < L; i += 4) {
    const double* prow = pm + (size_t)i * Lp;
    double tau = 0.0;
    for (int l = i; l < L; ++l) tau = fma(prow[l], s_dt[l * kTileNu + lane], tau);
    dsum += area[i] * -expm1(-tau);
  }
  s_red[wv * kTileNu + lane] = dsum;
  __syncthreads();
  if (tid < kTileNu) {
    const double tot = (s_red[tid] + s_red[kTileNu + tid]) + (s_red[2 * kTileNu + tid] + s_red[3 * kTileNu + tid]);
    if (nu0 + tid < m.n_nu) out[nu0 + tid] = w.core[b] + tot;
  }
}

size_t trans_fwd_lds_bytes(const Model& m, bool fp64) {
  if (fp64) return (size_t)m.L_pad * kTileNu * 8 + 4 * kTileNu * 8;
  return (size_t)2 * kTileNu * (m.L_pad + 8) * 2 + (size_t)m.L_pad * 4 + 4 * 32 * 4;
}

hipError_t trans_fwd_configure(const Model& m, bool fp64) {
  const int bytes = (int)trans_fwd_lds_bytes(m, fp64);
  if (fp64) return hipFuncSetAttribute((const void*)k_trans_fwd_fp64, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  return hipFuncSetAttribute((const void*)k_trans_fwd_mixed, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

void launch_trans_fwd(const Model& m, const Work& w, const Tables& tb, int B, void* spec, bool fp64, hipStream_t st) {
  const dim3 grid((unsigned)(m.n_tiles * B));
  const size_t lds = trans_fwd_lds_bytes(m, fp64);
  if (fp64)
    hipLaunchKernelGGL(k_trans_fwd_fp64, grid, dim3(kBlock), lds, st, m, w, tb, B, (double*)spec);
  else
    hipLaunchKernelGGL(k_trans_fwd_mixed, grid, dim3(kBlock), lds, st, m, w, tb, B, (float*)spec);
}

}  // namespace exofwd
