// Correlated-k path (Section "Gas phase opacities"): per spectral bin, each
// absorber's k-table holds the cross section at kCkG g-points of the bin's
// cumulative distribution with quadrature weights w_g (sum 1).  The species are
// mixed layer by layer by random overlap with resorting and rebinning (RORR,
// Amundsen et al. 2017): two k-distributions, as layer optical depths, combine on
// all g-point pairs (sum of the depths, product of the weights); the pairs are
// sorted and the sorted distribution is averaged over each original g-interval
// [E_{n-1}, E_n], E_n = w_1 + ... + w_n.  The next absorber is then mixed into the
// result, in table order.  The grey continuum (CIA, Rayleigh, grey deck at the bin
// centre) is added to every g-point.  Each g-point's column then goes through the
// transmission chord (Eq. 44) or the emission sweep (Eq. 45), and the bin's
// spectrum is the g-weighted sum.
//
// k_ck_mix: one wave per (sample, layer) and a run of 16 bins, eight bins at a time,
//   one per group of eight lanes.  Lane p of a group interpolates every absorber at
//   g-point p (FP32 table entries relative to per-(absorber, column) offsets,
//   bilinear in (T, log p), exp2 with the layer prefactor).  A merge gives lane p row
//   p of the 8 x 8 pair matrix, mixture point p with each absorber point, which
//   ascends because both distributions do; the 64 pair sums are sorted by the three
//   merge levels of a bitonic network (DPP lane moves inside the group and
//   compare-exchanges inside a lane; keys = the value's bits above the low six, the
//   pair index in the low six), the exact sums and weights are looked up by index, and
//   the integral of the sorted distribution over each g-interval comes from each
//   element's overlap with it, in FP64, reduce-scattered over the group so that lane p
//   receives its own interval.  Output: the mixed layer optical depths
//   [B][L_pad][n_bins_pad x 8] (FP32), read by k_ck_trans (bf16x3 MFMA chord, as the
//   cross-section path) or k_ck_emis (one lane per (bin, g-point) column sweeping up
//   the layers).
#include "ck.h"
#include "emission.h"
#include "kernels.h"
#include "opacity.h"

namespace exofwd {

// DPP lane moves inside 8-lane groups (gfx9 encodings): quad_perm patterns and the
// half-row (8-lane) mirror
constexpr int kDppXor1 = 0xB1;     // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;     // quad_perm [2,3,0,1]
constexpr int kDppQuadMirror = 0x1B;   // quad_perm [3,2,1,0]
constexpr int kDppHalfMirror = 0x141;  // row_half_mirror: lane p <-> 7 - p of each 8
constexpr int kDppShr1 = 0x111, kDppShr2 = 0x112, kDppShr4 = 0x114;   // row_shr:1, 2, 4

template <int CTRL>
__device__ inline uint32_t dpp_u(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, true);
}

// One cross-lane step of the sorting network: register r meets the partner lane's
// register r (or 7 - r with `rev`); the lower lane of the pair keeps the smaller key.
template <int CTRL, bool REV>
__device__ inline void net_cross(uint32_t (&k)[8], bool lower) {
  uint32_t o[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) o[r] = dpp_u<CTRL>(k[REV ? 7 - r : r]);
#pragma unroll
  for (int r = 0; r < 8; ++r) k[r] = lower ? min(k[r], o[r]) : max(k[r], o[r]);
}
// half-cleaner inside a lane: registers r and r + J (r & J == 0) ordered ascending
template <int J>
__device__ inline void net_local(uint32_t (&k)[8]) {
#pragma unroll
  for (int r = 0; r < 8; ++r)
    if (!(r & J)) {
      const uint32_t lo = min(k[r], k[r + J]), hi = max(k[r], k[r + J]);
      k[r] = lo;
      k[r + J] = hi;
    }
}

// Sort the 64 keys of an 8-lane group, element 8p + r on lane p, register r, when each
// lane's eight registers already ascend: the three merge levels of a bitonic network
// whose first step in each level pairs mirror images (so every run is merged ascending).
__device__ inline void sort_group64(uint32_t (&k)[8], int p) {
  // runs of 16: lanes p, p ^ 1
  net_cross<kDppXor1, true>(k, (p & 1) == 0);
  net_local<4>(k); net_local<2>(k); net_local<1>(k);
  // runs of 32: lanes of a quad, mirrored, then p ^ 1
  net_cross<kDppQuadMirror, true>(k, (p & 2) == 0);
  net_cross<kDppXor1, false>(k, (p & 1) == 0);
  net_local<4>(k); net_local<2>(k); net_local<1>(k);
  // runs of 64: the 8 lanes mirrored, then p ^ 2, p ^ 1
  net_cross<kDppHalfMirror, true>(k, (p & 4) == 0);
  net_cross<kDppXor2, false>(k, (p & 2) == 0);
  net_cross<kDppXor1, false>(k, (p & 1) == 0);
  net_local<4>(k); net_local<2>(k); net_local<1>(k);
}

template <int CTRL>
__device__ inline double dpp_d(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint64_t lo = dpp_u<CTRL>((uint32_t)u), hi = dpp_u<CTRL>((uint32_t)(u >> 32));
  return __longlong_as_double((long long)(lo | (hi << 32)));
}

// exclusive prefix over the 8 lanes of a group (lane p gets the sum of lanes < p)
__device__ inline double group_excl8(double x, int p) {
  double s = x, t;
  t = dpp_d<kDppShr1>(s);
  s += p >= 1 ? t : 0.0;
  t = dpp_d<kDppShr2>(s);
  s += p >= 2 ? t : 0.0;
  t = dpp_d<kDppShr4>(s);
  s += p >= 4 ? t : 0.0;
  return s - x;
}

// reduce-scatter over the 8 lanes of a group: lane p gets the sum over the lanes of
// their d[p].  Three halving steps, each with a partner whose lane differs in the bit
// that decides which half of the remaining entries a lane keeps.
__device__ inline double group_reduce_scatter8(const double (&d)[8], int p) {
  double h[4], q[2];
  const bool k4 = p & 4, k2 = p & 2, k1 = p & 1;
#pragma unroll
  for (int i = 0; i < 4; ++i) {   // partner 7 - p: the other bit 2
    const double keep = k4 ? d[i + 4] : d[i], send = k4 ? d[i] : d[i + 4];
    h[i] = keep + dpp_d<kDppHalfMirror>(send);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {   // partner p ^ 3: the same bit 2, the other bit 1
    const double keep = k2 ? h[i + 2] : h[i], send = k2 ? h[i] : h[i + 2];
    q[i] = keep + dpp_d<kDppQuadMirror>(send);
  }
  const double keep = k1 ? q[1] : q[0], send = k1 ? q[0] : q[1];
  return keep + dpp_d<kDppXor1>(send);
}

// lane r of this lane's group of eight (ds_swizzle bit mode: and 0x18, or r)
template <int R>
__device__ inline float group_bcast(float v) {
  return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x18 | (R << 5)));
}

template <int S, bool CIA>
__global__ __launch_bounds__(kBlock) void k_ck_mix(Model m, Work w, Tables tb, int B) {
  // per wave: the 64 pair sums of each of its 8 bins, looked up after the sort; per
  // block: the 64 pair weights w_a w_b (FP64)
  __shared__ float s_val[kBlock / 64][512];
  __shared__ double s_wpair[64];
  if (threadIdx.x < 64) s_wpair[threadIdx.x] = tb.ckwd[threadIdx.x >> 3] * tb.ckwd[threadIdx.x & 7];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int b = blockIdx.z, l = blockIdx.y;
  const int j0 = (blockIdx.x * (kBlock / 64) + wv) * kCkBinsPerWave;
  if (j0 >= m.n_nu || w.status[b] || l >= w.nlay[b]) return;
  const int Lp = m.L_pad;
  constexpr int RL = rec_len(S);
  const float* rl = reinterpret_cast<const float*>(w.rec) + ((size_t)b * Lp + l) * RL;
  const int cl = w.cells[(size_t)b * Lp + l];
  const int it = cl & 255, ip = (cl >> 8) & 255, itc = cl >> 16;
  const float wt = rl[0], wp = rl[1], wtc = rl[2], ray = rl[3], deck = rl[4];
  const float w11 = wt * wp, w10 = wt - w11, w01 = wp - w11, w00 = 1.0f - wt - wp + w11;
  const size_t npad = (size_t)m.n_nu_pad, ncol = npad * kCkG;
  const uint32_t row_bytes = (uint32_t)ncol * 4u, tstep = (uint32_t)m.n_p * row_bytes;
  const __amdgpu_buffer_rsrc_t rh = make_rsrc(tb.h, (size_t)S * m.n_t * m.n_p * ncol * 4);
  const __amdgpu_buffer_rsrc_t rhc = make_rsrc(CIA ? (const void*)tb.hc : (const void*)tb.h,
                                               CIA ? (size_t)2 * m.n_tc * npad * 4 : 0);
  // eight bins per pass, one per group of eight lanes; lane p of a group is g-point p
  // of its bin and row p of each merge's pair matrix
  const int grp = lane >> 3, p = lane & 7;
  const double inv_wg = 1.0 / tb.ckwd[p];
  float* vals = s_val[wv] + grp * 64;
  float* out = w.ckmix + ((size_t)b * Lp + l) * ncol;

  for (int t = 0; t < kCkBinsPerWave; t += 8) {
    const int jr = j0 + t + grp;
    const bool real = jr < m.n_nu;
    const int j = real ? jr : m.n_nu - 1;   // a group past the last bin repeats it and stores nothing
    const uint32_t col = (uint32_t)(j * kCkG + p);
    // this lane's g-point of every absorber
    float sp[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const uint32_t row = (uint32_t)((s * m.n_t + it) * m.n_p + ip) * row_bytes, voff = col * 4u;
      float v = tb.c[(size_t)s * ncol + col] + rl[kRecFixed + s];
      v = fmaf(w00, load_f32(rh, voff, row), v);
      v = fmaf(w10, load_f32(rh, voff, row + tstep), v);
      v = fmaf(w01, load_f32(rh, voff, row + row_bytes), v);
      v = fmaf(w11, load_f32(rh, voff, row + tstep + row_bytes), v);
      sp[s] = exp2_fast(v);
    }
    float mix = sp[0];   // the running mixture at g-point p: absorber 0 to start
#pragma unroll
    for (int s = 1; s < S; ++s) {
      // row p of the pair matrix: mixture point p with each point r of absorber s, which
      // ascends in r (a k-table row ascends in g)
      float v[8];
      v[0] = mix + group_bcast<0>(sp[s]);
      v[1] = mix + group_bcast<1>(sp[s]);
      v[2] = mix + group_bcast<2>(sp[s]);
      v[3] = mix + group_bcast<3>(sp[s]);
      v[4] = mix + group_bcast<4>(sp[s]);
      v[5] = mix + group_bcast<5>(sp[s]);
      v[6] = mix + group_bcast<6>(sp[s]);
      v[7] = mix + group_bcast<7>(sp[s]);
      // the previous merge's lookups are done before the table is rewritten
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      uint32_t key[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        vals[8 * p + r] = v[r];
        // optical depths are >= 0, so the bit patterns order like the values; the low
        // six bits carry the pair index (pairs within 64 ulp may swap: < 4e-6 relative)
        key[r] = (__float_as_uint(v[r]) & ~63u) | (uint32_t)(8 * p + r);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      sort_group64(key, p);
      // The group's 64 pairs in sorted order, element 8p + r on lane p, and where each
      // ends on the g axis, U_r.  The g bookkeeping runs in FP64: an interval edge often
      // falls exactly on an element boundary (a negligible absorber leaves the pairs in
      // blocks of one mixture point, whose weights sum to the edge), and there an FP32
      // rounding of the running weight would move a sliver of the next, possibly far
      // larger, value into the interval.
      double vd[8], U[8];
      double cs = 0.0;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const uint32_t idx = key[r] & 63u;
        vd[r] = (double)vals[idx];
        U[r] = s_wpair[idx];
        cs += U[r];
      }
      const double c_lane = group_excl8(cs, p);
      double run = c_lane;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        run += U[r];
        U[r] = run;
      }
      // D[n]: this lane's share of the integral of the sorted distribution over the
      // g-interval [E_{n-1}, E_n], from the overlap of each element [U_{r-1}, U_r) with it
      double D[8], prev = 0.0;
#pragma unroll
      for (int n = 0; n < kCkG; ++n) {
        double part = 0.0;
        if (n < kCkG - 1) {
          const double E = tb.cke[n];
          double lo = fmin(E, c_lane);
#pragma unroll
          for (int r = 0; r < 8; ++r) {
            const double hi = fmin(E, U[r]);
            part = fma(vd[r], hi - lo, part);
            lo = hi;
          }
        } else {
          double lo = c_lane;
#pragma unroll
          for (int r = 0; r < 8; ++r) {
            part = fma(vd[r], U[r] - lo, part);
            lo = U[r];
          }
        }
        D[n] = part - prev;
        prev = part;
      }
      // lane p: the integral over its own interval, summed over the group, / w_p
      mix = (float)(group_reduce_scatter8(D, p) * inv_wg);
    }
    // grey continuum at the bin centre: deck, Rayleigh and the two CIA pairs
    float dc = fmaf(ray, tb.nu4f[j], deck);
    if (CIA) {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const uint32_t rowc = (uint32_t)(q * m.n_tc + itc) * (uint32_t)npad * 4u;
        const uint32_t vo = (uint32_t)j * 4u;
        float v = tb.cc[(size_t)q * npad + j] + rl[5 + q];
        v = fmaf(1.0f - wtc, load_f32(rhc, vo, rowc), v);
        v = fmaf(wtc, load_f32(rhc, vo, rowc + (uint32_t)npad * 4u), v);
        dc += exp2_fast(v);
      }
    }
    if (real) __builtin_nontemporal_store(mix + dc, &out[col]);   // read once, by the spectrum kernel
  }
}

// Transmission: per (sample, 128-column tile) the chord tau = P dtau on MFMA
// (bf16 hi/lo split of both operands, as the cross-section kernel), the transit
// depth of every (bin, g-point) column and the g-weighted sum per bin.
__global__ __launch_bounds__(kBlockT) void k_ck_trans(Model m, Work w, Tables tb, int B, float* __restrict__ spec) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int n_ct = m.n_tiles * kCkG;   // 128-column tiles per sample
  const int logical = xcd_logical_block(blockIdx.x, gridDim.x);
  const int b = logical / n_ct, tile = logical % n_ct;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int Lp = m.L_pad;
  const int c0 = tile * kTileNu;          // first column; bins c0/8 .. c0/8 + 15
  const int j0 = c0 / kCkG;
  float* out = spec + (size_t)b * m.n_nu;
  if (w.status[b]) {
    if (tid < kTileNu / kCkG && j0 + tid < m.n_nu) out[j0 + tid] = __builtin_nanf("");
    return;
  }
  const int L = w.nlay[b];
  const size_t ncol = (size_t)m.n_nu_pad * kCkG;
  const int stride = Lp + 8;
  uint16_t* s_bhi = reinterpret_cast<uint16_t*>(lds);
  uint16_t* s_blo = s_bhi + kTileNu * stride;
  float* s_area = reinterpret_cast<float*>(s_blo + kTileNu * stride);
  float* s_red = s_area + Lp;   // [8][32]
  const float* area = reinterpret_cast<const float*>(w.area) + (size_t)b * Lp;
  for (int i = tid; i < Lp; i += kBlockT) s_area[i] = area[i];

  // phase A: the mixed layer optical depths of the tile -> bf16 hi/lo B operand in LDS
  const float* src = w.ckmix + (size_t)b * Lp * ncol + c0 + 2 * lane;
  const bool real = (c0 + 2 * lane) / kCkG < m.n_nu;   // columns of padding bins hold nothing
  const int KBe = (L + 15) >> 4;
  for (int o = wv; o < 2 * KBe; o += kBlockT / 64) {
    float e0[8], e1[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int l = 8 * o + q;
      float2 d = make_float2(0.0f, 0.0f);
      if (l < L && real) {
        const float2v v = __builtin_nontemporal_load(reinterpret_cast<const float2v*>(src + (size_t)l * ncol));
        d = make_float2(v.x, v.y);
      }
      e0[q] = fminf(d.x, 16384.0f);
      e1[q] = fminf(d.y, 16384.0f);
    }
    uint32_t h0[4], l0[4], h1[4], l1[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      split_pair(e0[2 * q], e0[2 * q + 1], h0[q], l0[q]);
      split_pair(e1[2 * q], e1[2 * q + 1], h1[q], l1[q]);
    }
    const int r0 = (2 * lane) * stride + 8 * o, r1 = r0 + stride;
    *reinterpret_cast<uint4*>(s_bhi + r0) = make_uint4(h0[0], h0[1], h0[2], h0[3]);
    *reinterpret_cast<uint4*>(s_blo + r0) = make_uint4(l0[0], l0[1], l0[2], l0[3]);
    *reinterpret_cast<uint4*>(s_bhi + r1) = make_uint4(h1[0], h1[1], h1[2], h1[3]);
    *reinterpret_cast<uint4*>(s_blo + r1) = make_uint4(l1[0], l1[1], l1[2], l1[3]);
  }
  __syncthreads();

  // phase B: tau = P dtau; wave wv owns 32-column block (wv & 3) and half (wv >> 2) of the row blocks
  const int MBe = (L + 31) >> 5;
  const int KB = Lp >> 4;
  const int nb = wv & 3;
  const size_t plane = (size_t)(Lp >> 5) * KB * 512;
  const uint16_t* fh = w.pfrag + (size_t)b * 2 * plane;
  const uint16_t* fl = fh + plane;
  const int col = 32 * nb + (lane & 31);
  const int khalf = 8 * (lane >> 5);
  float dsum = 0.0f;
  for (int mi = (wv >> 2); mi < MBe; mi += 2) {
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
    // phase C: annulus-weighted absorption of each column's chords
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int r = 32 * mi + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
      dsum = fmaf(s_area[r], one_minus_exp(acc[q], exp2_fast(-1.4426950408889634f * acc[q])), dsum);
    }
  }
  dsum += __shfl_xor(dsum, 32);
  if (lane < 32) s_red[wv * 32 + lane] = dsum;
  __syncthreads();
  if (tid < kTileNu) {
    // column tid = bin tid/8, g-point tid%8: weighted, then summed over the bin's eight columns
    const int h = tid >> 5, c = tid & 31;
    float v = (float)w.core[b] + s_red[h * 32 + c] + s_red[(h + 4) * 32 + c];
    v *= tb.ckw[tid & (kCkG - 1)];
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    const int j = j0 + (tid >> 3);
    if ((tid & (kCkG - 1)) == 0 && j < m.n_nu) out[j] = v;
  }
}

// Transmission with random overlap along each chord (the product of the absorbers'
// transmission functions): a tile of 16 bins x 8 g-points (128 columns) runs one
// pass per absorber; absorber 0's columns also carry the grey continuum (exact: the
// chord is linear, so its factor e^-tau_c multiplies absorber 0's g-sum).  Per chord
// row the absorption of absorber s is A_s = sum_g w_g (1 - e^-tau_s,g), and the
// passes combine it as A (+) A_s = A + A_s - A A_s (= 1 - (1 - A)(1 - A_s), without
// the cancellation of a thin chord's 1 - product of transmissions), kept in LDS per
// (bin, row).  One absorber per pass keeps a wave's table loads on 16 contiguous
// bins of one table row.
constexpr int kProdBins = kTileNu / kCkG;   // bins per tile

// two adjacent FP32 table entries (8 bytes) through a buffer resource
__device__ inline float2 load_f32x2(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
  return make_float2(__uint_as_float(v[0]), __uint_as_float(v[1]));
}

template <int S, bool CIA>
__global__ __launch_bounds__(kBlockT) void k_ck_trans_prod(Model m, Work w, Tables tb, int B,
                                                           float* __restrict__ spec) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int n_bt = (m.n_nu + kProdBins - 1) / kProdBins;   // bin tiles per sample
  const int logical = xcd_logical_block(blockIdx.x, gridDim.x);
  const int b = logical / n_bt, tile = logical % n_bt;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int Lp = m.L_pad;
  const int j0 = kProdBins * tile;
  float* out = spec + (size_t)b * m.n_nu;
  if (w.status[b]) {
    if (tid < kProdBins && j0 + tid < m.n_nu) out[j0 + tid] = __builtin_nanf("");
    return;
  }
  const int L = w.nlay[b];
  const int stride = Lp + 8;
  uint16_t* s_bhi = reinterpret_cast<uint16_t*>(lds);
  uint16_t* s_blo = s_bhi + kTileNu * stride;
  float* s_area = reinterpret_cast<float*>(s_blo + kTileNu * stride);
  float* s_abs = s_area + Lp;   // [kProdBins][Lp]: combined absorption per bin and chord row
  const float* area = reinterpret_cast<const float*>(w.area) + (size_t)b * Lp;
  for (int i = tid; i < Lp; i += kBlockT) s_area[i] = area[i];

  // this lane's two columns: bin jj of the tile, g-points g and g + 1
  const int c2 = 2 * lane, jj = c2 >> 3, g = c2 & 7;
  const bool real = j0 + jj < m.n_nu;   // columns of bins past the last hold nothing
  const int j = real ? j0 + jj : m.n_nu - 1;
  const size_t npad = (size_t)m.n_nu_pad, ncol = npad * kCkG;
  const uint32_t row_bytes = (uint32_t)ncol * 4u, tstep = (uint32_t)m.n_p * row_bytes;
  const __amdgpu_buffer_rsrc_t rh = make_rsrc(tb.h, (size_t)S * m.n_t * m.n_p * ncol * 4);
  const __amdgpu_buffer_rsrc_t rhc = make_rsrc(CIA ? (const void*)tb.hc : (const void*)tb.h,
                                               CIA ? (size_t)2 * m.n_tc * npad * 4 : 0);
  const uint32_t col = (uint32_t)(j * kCkG + g), vo = col * 4u;
  const float nu4 = tb.nu4f[j];
  float cc[2] = {0.0f, 0.0f};
  if (CIA) {
    cc[0] = tb.cc[j];
    cc[1] = tb.cc[npad + j];
  }
  constexpr int RL = rec_len(S);
  const float* rec = reinterpret_cast<const float*>(w.rec) + (size_t)b * Lp * RL;
  const int32_t* cells = w.cells + (size_t)b * Lp;
  const int KBe = (L + 15) >> 4, MBe = (L + 31) >> 5, KB = Lp >> 4;
  const int nb = wv & 3;
  const size_t plane = (size_t)(Lp >> 5) * KB * 512;
  const uint16_t* fh = w.pfrag + (size_t)b * 2 * plane;
  const uint16_t* fl = fh + plane;
  const int ccol = 32 * nb + (lane & 31);
  const int khalf = 8 * (lane >> 5);
  const float wg = tb.ckw[lane & 7];
  const int bin_c = 4 * nb + ((lane & 31) >> 3);   // the tile bin of this lane's MFMA column

#pragma unroll 1
  for (int s = 0; s < S; ++s) {
    // phase A: absorber s's optical depth of every layer at the tile's columns -> bf16
    // hi/lo B operand in LDS
    const float2 cof = *reinterpret_cast<const float2*>(tb.c + (size_t)s * ncol + col);
    for (int o = wv; o < 2 * KBe; o += kBlockT / 64) {
      float e0[8], e1[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int l = 8 * o + q;
        float d0 = 0.0f, d1 = 0.0f;
        if (l < L) {
          const float* rl = rec + (size_t)l * RL;
          const int cl = cells[l];
          const int it = cl & 255, ip = (cl >> 8) & 255, itc = cl >> 16;
          const float wt = rl[0], wp = rl[1];
          const float w11 = wt * wp, w10 = wt - w11, w01 = wp - w11, w00 = 1.0f - wt - wp + w11;
          const uint32_t row = (uint32_t)((s * m.n_t + it) * m.n_p + ip) * row_bytes;
          const float lam = rl[kRecFixed + s];
          float v0 = cof.x + lam, v1 = cof.y + lam;
          const float2 t00 = load_f32x2(rh, vo, row), t10 = load_f32x2(rh, vo, row + tstep);
          const float2 t01 = load_f32x2(rh, vo, row + row_bytes), t11 = load_f32x2(rh, vo, row + tstep + row_bytes);
          v0 = fmaf(w00, t00.x, v0);
          v1 = fmaf(w00, t00.y, v1);
          v0 = fmaf(w10, t10.x, v0);
          v1 = fmaf(w10, t10.y, v1);
          v0 = fmaf(w01, t01.x, v0);
          v1 = fmaf(w01, t01.y, v1);
          v0 = fmaf(w11, t11.x, v0);
          v1 = fmaf(w11, t11.y, v1);
          d0 = exp2_fast(v0);
          d1 = exp2_fast(v1);
          if (s == 0) {
            // the grey continuum at the bin centre rides on absorber 0
            float dc = fmaf(rl[3], nu4, rl[4]);
            if (CIA) {
              const float wtc = rl[2];
#pragma unroll
              for (int p = 0; p < 2; ++p) {
                const uint32_t rowc = (uint32_t)(p * m.n_tc + itc) * (uint32_t)npad * 4u;
                const uint32_t vj = (uint32_t)j * 4u;
                float v = cc[p] + rl[5 + p];
                v = fmaf(1.0f - wtc, load_f32(rhc, vj, rowc), v);
                v = fmaf(wtc, load_f32(rhc, vj, rowc + (uint32_t)npad * 4u), v);
                dc += exp2_fast(v);
              }
            }
            d0 += dc;
            d1 += dc;
          }
          if (!real) d0 = d1 = 0.0f;
        }
        e0[q] = fminf(d0, 16384.0f);
        e1[q] = fminf(d1, 16384.0f);
      }
      uint32_t h0[4], l0[4], h1[4], l1[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        split_pair(e0[2 * q], e0[2 * q + 1], h0[q], l0[q]);
        split_pair(e1[2 * q], e1[2 * q + 1], h1[q], l1[q]);
      }
      const int r0 = c2 * stride + 8 * o, r1 = r0 + stride;
      *reinterpret_cast<uint4*>(s_bhi + r0) = make_uint4(h0[0], h0[1], h0[2], h0[3]);
      *reinterpret_cast<uint4*>(s_blo + r0) = make_uint4(l0[0], l0[1], l0[2], l0[3]);
      *reinterpret_cast<uint4*>(s_bhi + r1) = make_uint4(h1[0], h1[1], h1[2], h1[3]);
      *reinterpret_cast<uint4*>(s_blo + r1) = make_uint4(l1[0], l1[1], l1[2], l1[3]);
    }
    __syncthreads();

    // phase B: tau = P dtau; wave wv owns 32-column block nb and half (wv >> 2) of the row blocks
    for (int mi = (wv >> 2); mi < MBe; mi += 2) {
      f32x16 acc = {};
      for (int kb = 2 * mi; kb < KBe; ++kb) {
        const size_t fo = ((size_t)(mi * KB + kb) * 64 + lane) * 8;
        const bf16x8 ah = *reinterpret_cast<const bf16x8*>(fh + fo);
        const bf16x8 al = *reinterpret_cast<const bf16x8*>(fl + fo);
        const bf16x8 bh = *reinterpret_cast<const bf16x8*>(s_bhi + ccol * stride + 16 * kb + khalf);
        const bf16x8 bl = *reinterpret_cast<const bf16x8*>(s_blo + ccol * stride + 16 * kb + khalf);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc, 0, 0, 0);
      }
      // phase C: per row, absorber s's g-weighted absorption in its bin (8 lanes),
      // combined into the bin's running absorption
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        float a = wg * one_minus_exp(acc[q], exp2_fast(-1.4426950408889634f * acc[q]));
        a += __shfl_xor(a, 1);
        a += __shfl_xor(a, 2);
        a += __shfl_xor(a, 4);
        const int r = 32 * mi + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
        if ((lane & 7) == 0) {
          float* pa = s_abs + bin_c * Lp + r;
          const float prev = s == 0 ? 0.0f : *pa;
          *pa = prev + a - prev * a;
        }
      }
    }
    __syncthreads();   // the next pass overwrites the B operand
  }
  // the bins' combined absorption, annulus-weighted and summed over the rows: 32
  // threads per bin
  const int bj = tid >> 5;
  float v = 0.0f;
  for (int i = tid & 31; i < 32 * MBe; i += 32) v = fmaf(s_area[i], s_abs[bj * Lp + i], v);
#pragma unroll
  for (int off = 16; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if ((tid & 31) == 0 && j0 + bj < m.n_nu) out[j0 + bj] = (float)w.core[b] + v;
}

// Emission: one lane per (bin, g-point) column, sweeping up the layers with the
// linear-in-tau source at the bin centre's Planck intensity (FP64 intensities, as
// the cross-section kernel), then the g-weighted flux per bin and F_p / F_*.
__global__ __launch_bounds__(kBlock) void k_ck_emis(Model m, Work w, Tables tb, int B, float* __restrict__ spec) {
  const int n_ct = m.n_tiles64 * kCkG;   // 64-column tiles per sample
  const int logical = xcd_logical_block(blockIdx.x, gridDim.x);
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int gw = logical * (kBlock / 64) + wv;
  const int b = gw / n_ct, tile = gw % n_ct;
  if (b >= B) return;
  const int colx = tile * kTile64 + lane, j = colx / kCkG;
  float* out = spec + (size_t)b * m.n_nu;
  if (w.status[b]) {
    if ((lane & (kCkG - 1)) == 0 && j < m.n_nu) out[j] = __builtin_nanf("");
    return;
  }
  const int L = w.nlay[b], Lp = m.L_pad;
  const size_t ncol = (size_t)m.n_nu_pad * kCkG;
  const float* dt = w.ckmix + (size_t)b * Lp * ncol + colx;
  const double* t_lev = w.t_lev + (size_t)b * (Lp + 1);
  const double* inv_t = w.inv_tlev + (size_t)b * (Lp + 1);
  const double nud = m.nu[j];
  const float c1n3 = (float)(2.0 * kHpl * kC * kC * nud * nud * nud);
  const double c2n_log2e = kHpl * kC / kB * 1.4426950408889634074 * nud;
  auto planck_at = [&](int lv) {
    float y, em1;
    return planck_split(c1n3, c2n_log2e, inv_t[lv], y, em1);
  };
  const int n_mu = m.n_mu;
  float inv_mu[kMaxMu];
  double inten[kMaxMu];
  float b_bot = planck_at(0);
#pragma unroll
  for (int k = 0; k < kMaxMu; ++k) {
    inv_mu[k] = k < n_mu ? (float)(1.0 / m.mu_nodes[k]) : 0.0f;
    inten[k] = b_bot;
  }
  const bool real = j < m.n_nu;   // columns of padding bins hold nothing
  for (int l = 0; l < L; ++l) {
    const float d = real ? __builtin_nontemporal_load(&dt[(size_t)l * ncol]) : 0.0f;
    const float b_top = planck_at(l + 1);
    const float db = b_bot - b_top;
#pragma unroll
    for (int k = 0; k < kMaxMu; ++k) {
      if (k >= n_mu) break;
      const float x = d * inv_mu[k];
      const float e = exp2_fast(-1.4426950408889634f * x);
      float om, src;
      slab_terms(x, e, om, src);
      inten[k] = fma((double)om, (double)b_top - inten[k], fma((double)db, (double)src, inten[k]));
    }
    b_bot = b_top;
  }
  double flux = 0.0;
#pragma unroll
  for (int k = 0; k < kMaxMu; ++k)
    if (k < n_mu) flux = fma(2.0 * M_PI * m.mu_weights[k] * m.mu_nodes[k], inten[k], flux);
  flux *= (double)tb.ckw[lane & (kCkG - 1)];
  flux += __shfl_xor(flux, 1);
  flux += __shfl_xor(flux, 2);
  flux += __shfl_xor(flux, 4);
  if ((lane & (kCkG - 1)) == 0 && j < m.n_nu) {
    const double fstar = M_PI * 2.0 * kHpl * kC * kC * nud * nud * nud / expm1(kHpl * kC * nud / (kB * m.t_star));
    out[j] = (float)(m.dilution * flux / fstar * w.core[b]);
  }
}

// ---------------------------------------------------------------------------
template <int S, bool CIA>
const void* ck_mix_kernel() { return (const void*)k_ck_mix<S, CIA>; }

static const void* ck_mix_kernel_for(int S, bool cia) {
#define EXOFWD_CASE(n) \
  case n: return cia ? ck_mix_kernel<n, true>() : ck_mix_kernel<n, false>();
  switch (S) {
    EXOFWD_CASE(1) EXOFWD_CASE(2) EXOFWD_CASE(3) EXOFWD_CASE(4)
    EXOFWD_CASE(5) EXOFWD_CASE(6) EXOFWD_CASE(7) EXOFWD_CASE(8)
  }
#undef EXOFWD_CASE
  return nullptr;
}

template <int S, bool CIA>
const void* ck_prod_kernel() { return (const void*)k_ck_trans_prod<S, CIA>; }

static const void* ck_prod_kernel_for(int S, bool cia) {
#define EXOFWD_CASE(n) \
  case n: return cia ? ck_prod_kernel<n, true>() : ck_prod_kernel<n, false>();
  switch (S) {
    EXOFWD_CASE(1) EXOFWD_CASE(2) EXOFWD_CASE(3) EXOFWD_CASE(4)
    EXOFWD_CASE(5) EXOFWD_CASE(6) EXOFWD_CASE(7) EXOFWD_CASE(8)
  }
#undef EXOFWD_CASE
  return nullptr;
}

static size_t ck_trans_lds_bytes(const Model& m) {
  return (size_t)2 * kTileNu * (m.L_pad + 8) * 2 + (size_t)m.L_pad * 4 + 8 * 32 * 4;
}
static size_t ck_prod_lds_bytes(const Model& m) {
  return (size_t)2 * kTileNu * (m.L_pad + 8) * 2 + (size_t)m.L_pad * 4 * (1 + kProdBins);
}

hipError_t ck_configure(const Model& m) {
  if (m.mode != kTransmission) return ck_mix_kernel_for(m.S, m.has_cia) ? hipSuccess : hipErrorInvalidValue;
  if (m.ck_mix == kCkProduct) {
    const void* k = ck_prod_kernel_for(m.S, m.has_cia);
    if (!k) return hipErrorInvalidValue;
    return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)ck_prod_lds_bytes(m));
  }
  if (!ck_mix_kernel_for(m.S, m.has_cia)) return hipErrorInvalidValue;
  return hipFuncSetAttribute((const void*)k_ck_trans, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)ck_trans_lds_bytes(m));
}

void launch_ck_mix(const Model& m, const Work& w, const Tables& tb, int B, hipStream_t st) {
  if (m.ck_mix != kCkRorr) return;   // the product of transmissions mixes inside its chord kernel
  const unsigned gx = (unsigned)((m.n_nu + kCkBinsPerWave * (kBlock / 64) - 1) / (kCkBinsPerWave * (kBlock / 64)));
  void* args[] = {(void*)&m, (void*)&w, (void*)&tb, (void*)&B};
  hipLaunchKernel(ck_mix_kernel_for(m.S, m.has_cia), dim3(gx, (unsigned)m.L_max, (unsigned)B), dim3(kBlock), args, 0,
                  st);
}

void launch_ck_spectrum(const Model& m, const Work& w, const Tables& tb, int B, void* spec, hipStream_t st) {
  if (m.ck_mix == kCkProduct) {
    void* args[] = {(void*)&m, (void*)&w, (void*)&tb, (void*)&B, (void*)&spec};
    hipLaunchKernel(ck_prod_kernel_for(m.S, m.has_cia),
                    dim3((unsigned)(B * ((m.n_nu + kProdBins - 1) / kProdBins))), dim3(kBlockT), args,
                    ck_prod_lds_bytes(m), st);
    return;
  }
  if (m.mode == kTransmission) {
    hipLaunchKernelGGL(k_ck_trans, dim3((unsigned)(B * m.n_tiles * kCkG)), dim3(kBlockT), ck_trans_lds_bytes(m), st, m,
                       w, tb, B, (float*)spec);
  } else {
    const int waves = B * m.n_tiles64 * kCkG;
    hipLaunchKernelGGL(k_ck_emis, dim3((unsigned)((waves + kBlock / 64 - 1) / (kBlock / 64))), dim3(kBlock), 0, st, m,
                       w, tb, B, (float*)spec);
  }
}

}  // namespace exofwd
