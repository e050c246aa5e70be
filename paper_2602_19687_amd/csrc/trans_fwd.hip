// Fused transmission forward kernels: per (sample, wavenumber tile) they build
// every layer's vertical optical depth from the interpolated cross-section
// tables, form the slant optical depth through the path matrix (Eq. 44) and
// reduce it to the transit depth of each wavenumber.
//
// Reduced-precision instance (512 threads, 128 wavenumbers per tile, two per
// lane): FP16 log2-sigma tables read with scalar-offset buffer loads, FP32
// opacity with one exp2 per layer, source and wavenumber, chord product on
// v_mfma_f32_32x32x16_bf16 with a bf16 hi/lo split of both operands
// (hi*hi + hi*lo + lo*hi, FP32 accumulation).
// FP64 instance (256 threads, 64 wavenumbers per tile): FP64 tables and
// arithmetic, chord product on the FP64 VALU.
#include "cloud.h"
#include "kernels.h"
#include "opacity.h"

namespace exofwd {

// Path-matrix A fragments: cost-balanced split of the 32-row blocks between the
// two waves that share a 32-column block.
__device__ inline unsigned mblocks_for(int part, int MBe, int KBe) {
  unsigned mine = 0;
  int c0 = 0, c1 = 0;
  for (int mi = 0; mi < MBe; ++mi) {
    const int cost = KBe - 2 * mi;
    if (c0 <= c1) {
      if (part == 0) mine |= 1u << mi;
      c0 += cost;
    } else {
      if (part == 1) mine |= 1u << mi;
      c1 += cost;
    }
  }
  return mine;
}

// `cls` (may be null): the layer-count classes of the call (layer_classes), whose class
// `cl` this launch serves; `lt` is the LDS tile's layer capacity, a multiple of 32: at
// least every served sample's layers, or with KS (K split) fewer: the layers then pass
// through LDS in chunks of lt, each chunk's products accumulating into the chords, and
// the packed optical depths for the reverse pass are written as they are formed
template <int S, bool CIA, bool NGC, bool KS>
__global__ __launch_bounds__(kBlockT) void k_trans_fwd_mixed(Model m, Work w, Tables tb, int B, float* __restrict__ spec,
                                                              float* __restrict__ dtau_out, const int32_t* __restrict__ cls,
                                                              int cl, int lt) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int logical = xcd_logical_block(blockIdx.x, gridDim.x);
  // samples fastest: neighbouring workgroups (one XCD) share table columns;
  // tiles fastest: they share one sample's profile
  int b = m.fwd_tile_major ? logical / m.n_tiles : logical % B;
  const int tile = m.fwd_tile_major ? logical % m.n_tiles : logical / B;
  if (cls) {
    // the class's samples, longest first; the grid covers the whole batch (tiles
    // fastest: sample slots dealt round the XCDs)
    if (m.fwd_tile_major) b = class_position(b, B, m.n_tiles);
    if (b >= cls[cl]) return;
    b = cls[2 + cl * B + b];
  }
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int Lp = m.L_pad;
  const int nu0 = tile * kTileNu;
  float* out = spec + (size_t)b * m.n_nu;
  if (w.status[b]) {
    if (tid < kTileNu && nu0 + tid < m.n_nu) out[nu0 + tid] = __builtin_nanf("");
    return;
  }
  const int L = w.nlay[b];
  const int stride = lt + 8;   // bf16 per wavenumber row of the B operand (keeps b128 reads conflict-free)
  uint16_t* s_bhi = reinterpret_cast<uint16_t*>(lds);
  uint16_t* s_blo = s_bhi + kTileNu * stride;
  const int n_area = KS ? Lp : lt;   // chord rows
  float* s_area = reinterpret_cast<float*>(s_blo + kTileNu * stride);
  double* s_red = reinterpret_cast<double*>(s_area + n_area);   // [8][32]
  int* s_live = reinterpret_cast<int*>(s_red + 8 * 32);   // [0, MB): row block holds a chord below kOpaqueTau; [7]: frontier
  if (tid < 8) s_live[tid] = 0;

  const float* area = reinterpret_cast<const float*>(w.area) + (size_t)b * Lp;
  for (int i = tid; i < n_area; i += kBlockT) s_area[i] = area[i];

  // phase A: vertical optical depth of every layer -> bf16 hi/lo B operand in LDS
  const float* rec = reinterpret_cast<const float*>(w.rec) + (size_t)b * Lp * rec_len_wide(S);
  const int32_t* cells = w.cells + (size_t)b * Lp;
  TableGeom g;
  g.row_bytes = (uint32_t)m.n_nu_pad * 2u;
  g.tstep = (uint32_t)m.n_p * g.row_bytes;
  g.pstep = g.row_bytes;
  const size_t npad = (size_t)m.n_nu_pad;
  const __amdgpu_buffer_rsrc_t rh = make_rsrc(tb.h, (size_t)S * m.n_t * m.n_p * npad * 2);
  const __amdgpu_buffer_rsrc_t rhc = make_rsrc(CIA ? (const void*)tb.hc : (const void*)tb.h,
                                               CIA ? (size_t)2 * m.n_tc * npad * 2 : 0);
  const uint32_t voff = (uint32_t)lane * 4u;
  const LaneConst<S> kc = load_lane<S, CIA>(m, tb, nu0 + 2 * lane);
  float q0 = 1.0f, q1 = 1.0f;
  if constexpr (NGC) {
    const float2 q = *reinterpret_cast<const float2*>(w.cloud_q + (size_t)b * (1 + kCloudSpec) * npad + nu0 + 2 * lane);
    q0 = q.x;
    q1 = q.y;
  }
  const int KBe = (L + 15) >> 4;
  // a layer in the same table cell as the wave's previous one reuses its pairs
  LayerRaw<S, CIA> raw;
  int cell_prev = -1;
  // layer octets [o_lo, o_hi) -> LDS rows from 8 (o - o_lo)
  auto phase_a = [&](int o_lo, int o_hi) {
    for (int o = o_lo + wv; o < o_hi; o += kBlockT / 64) {
      float e0[8], e1[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int l = 8 * o + j;
        float d0 = 0.0f, d1 = 0.0f;
        if (l < L) {
          const LayerCoef<S> c = load_layer<S>(m, cells, rec, l, (uint32_t)nu0 * 2u, g);
          if (c.cell != cell_prev) {
            fetch_terms<S, CIA>(c, g, rh, rhc, voff, raw);
            cell_prev = c.cell;
          }
          eval_terms<S, CIA, NGC>(c, kc, raw, d0, d1, q0, q1);
          d0 = fminf(d0, 16384.0f);
          d1 = fminf(d1, 16384.0f);
        }
        e0[j] = d0;
        e1[j] = d1;
      }
      // bf16 hi/lo planes, pairs of consecutive layers per dword
      uint32_t h0[4], l0[4], h1[4], l1[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        split_pair(e0[2 * j], e0[2 * j + 1], h0[j], l0[j]);
        split_pair(e1[2 * j], e1[2 * j + 1], h1[j], l1[j]);
      }
      const int r0 = (2 * lane) * stride + 8 * (o - o_lo), r1 = r0 + stride;
      *reinterpret_cast<uint4*>(s_bhi + r0) = make_uint4(h0[0], h0[1], h0[2], h0[3]);
      *reinterpret_cast<uint4*>(s_blo + r0) = make_uint4(l0[0], l0[1], l0[2], l0[3]);
      *reinterpret_cast<uint4*>(s_bhi + r1) = make_uint4(h1[0], h1[1], h1[2], h1[3]);
      *reinterpret_cast<uint4*>(s_blo + r1) = make_uint4(l1[0], l1[1], l1[2], l1[3]);
      if (KS && dtau_out) {
        // the packed optical depths (bf16 hi | bf16 lo << 16) of the octet's layers
        // for the reverse pass: a later chunk overwrites these LDS rows
        uint32_t* dt = reinterpret_cast<uint32_t*>(dtau_out) + (size_t)b * Lp * npad + nu0 + 2 * lane;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int l = 8 * o + 2 * j;
          if (l < L) {
            __builtin_nontemporal_store(__builtin_amdgcn_perm(l0[j], h0[j], 0x05040100u), dt + (size_t)l * npad);
            __builtin_nontemporal_store(__builtin_amdgcn_perm(l1[j], h1[j], 0x05040100u), dt + (size_t)l * npad + 1);
          }
          if (l + 1 < L) {
            __builtin_nontemporal_store(__builtin_amdgcn_perm(l0[j], h0[j], 0x07060302u), dt + (size_t)(l + 1) * npad);
            __builtin_nontemporal_store(__builtin_amdgcn_perm(l1[j], h1[j], 0x07060302u), dt + (size_t)(l + 1) * npad + 1);
          }
        }
      }
    }
  };

  // phase B: tau = P dtau on MFMA; wave wv owns 32-column block (wv & 3) and a
  // cost-balanced half (wv >> 2) of the 32-row blocks
  const int MBe = (L + 31) >> 5;
  const int KB = Lp >> 4;
  const int nb = wv & 3;
  const unsigned mine = mblocks_for(wv >> 2, MBe, KBe);
  const size_t plane = (size_t)(Lp >> 5) * KB * 512;
  // this sample's P fragments (hi plane, then lo plane): lanes address their 16 bytes
  // with the vector offset, blocks with the scalar offset
  const __amdgpu_buffer_rsrc_t rs_f = make_rsrc(w.pfrag + (size_t)b * 2 * plane, 2 * plane * 2);
  const uint32_t lo_plane = (uint32_t)plane * 2u, voff_f = (uint32_t)lane * 16u;
  auto frag = [&](int blk, uint32_t pl) {
    return __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(rs_f, voff_f, (uint32_t)blk * 1024u + pl, 0));
  };
  const int col = 32 * nb + (lane & 31);
  const int khalf = 8 * (lane >> 5);
  // the annulus sum in FP64: near the best fit the likelihood seeds carry the spectrum's
  // rounding relative to the noise level, and a gradient that cancels to a fraction of
  // its terms carries it too
  double dsum = 0.0;
  // row block mi's products over the K blocks [k_lo, k_hi), B rows from LDS row 16 (kb - k_base).
  // The fragments go in two groups of two K blocks, one group's loads in flight while the
  // other's products run; every iteration issues the same loads (blocks past k_hi read
  // the next row block's fragments, or zeros past the buffer's range, and are never used)
  auto chord = [&](f32x16 acc, int mi, int k_lo, int k_hi, int k_base) {
    if (k_lo >= k_hi) return acc;
    bf16x8 ga[2][2], gb[2][2];   // [K block][hi, lo]
    auto load = [&](bf16x8 (&gr)[2][2], int k) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        gr[u][0] = frag(mi * KB + k + u, 0);
        gr[u][1] = frag(mi * KB + k + u, lo_plane);
      }
    };
    auto product = [&](const bf16x8 (&gr)[2][2], int k0) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int kb = k0 + u;
        if (kb >= k_hi) break;
        const int kr = 16 * (kb - k_base) + khalf;
        const bf16x8 bh = *reinterpret_cast<const bf16x8*>(s_bhi + col * stride + kr);
        const bf16x8 bl = *reinterpret_cast<const bf16x8*>(s_blo + col * stride + kr);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(gr[u][1], bh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(gr[u][0], bl, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(gr[u][0], bh, acc, 0, 0, 0);
      }
    };
    load(ga, k_lo);
#pragma unroll 1
    for (int kb = k_lo; kb < k_hi; kb += 4) {
      load(gb, kb + 2);
      product(ga, kb);
      if (kb + 2 >= k_hi) break;
      load(ga, kb + 4);
      product(gb, kb + 2);
    }
    return acc;
  };
  // phase C: annulus-weighted absorption 1 - e^-tau of row block mi, summed over rows
  auto absorb = [&](const f32x16& acc, int mi) {
    bool live = false;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int row = 32 * mi + 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
      dsum = fma((double)s_area[row], (double)one_minus_exp(acc[j], exp2_fast(-1.4426950408889634f * acc[j])), dsum);
      live |= !(acc[j] > kOpaqueTau);
    }
    // the reverse pass skips row blocks whose chords are all opaque across the tile
    if (dtau_out && __builtin_amdgcn_ballot_w64(live) != 0 && lane == 0) s_live[mi] = 1;
  };
  if constexpr (!KS) {
    phase_a(0, 2 * KBe);
    __syncthreads();
    for (int mi = 0; mi < MBe; ++mi) {
      if (!(mine & (1u << mi))) continue;
      absorb(chord(f32x16{}, mi, 2 * mi, KBe, 0), mi);
    }
  } else {
    // up to three row blocks per wave (five row blocks in two cost-balanced halves)
    int slot_mi[3];
    {
      int q = 0;
      for (int mi = 0; mi < MBe; ++mi)
        if ((mine & (1u << mi)) && q < 3) slot_mi[q++] = mi;
      for (; q < 3; ++q) slot_mi[q] = -1;
    }
    f32x16 acc[3] = {f32x16{}, f32x16{}, f32x16{}};
    const int kc = lt >> 4;   // K blocks per chunk
    for (int k0 = 0; k0 < KBe; k0 += kc) {
      const int k1 = k0 + kc < KBe ? k0 + kc : KBe;
      phase_a(2 * k0, 2 * k1);
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int mi = slot_mi[q];
        if (mi < 0) continue;
        acc[q] = chord(acc[q], mi, 2 * mi > k0 ? 2 * mi : k0, k1, k0);
      }
      __syncthreads();   // the next chunk overwrites the LDS rows
    }
#pragma unroll
    for (int q = 0; q < 3; ++q)
      if (slot_mi[q] >= 0) absorb(acc[q], slot_mi[q]);
  }
  dsum += __shfl_xor(dsum, 32);
  if (lane < 32) s_red[wv * 32 + lane] = dsum;
  __syncthreads();
  if (tid < kTileNu) {
    const int h = tid >> 5, c = tid & 31;
    const double tot = s_red[h * 32 + c] + s_red[(h + 4) * 32 + c];
    if (nu0 + tid < m.n_nu) out[nu0 + tid] = (float)(w.core[b] + tot);
  }
  if (dtau_out) {
    if (tid == 0) {
      int f = 0;
      while (f < MBe && !s_live[f]) ++f;
      w.front[(size_t)b * m.n_tiles + tile] = f;
      s_live[7] = f;
    }
    if constexpr (KS) return;   // the optical depths were written as they were formed
    __syncthreads();
    // the reverse pass reads the layer optical depths back instead of recomputing
    // them, already split: one dword (bf16 hi | bf16 lo << 16) per layer and
    // wavenumber, from the LDS planes, and only above the opaque frontier (the
    // layers below feed only chords whose seeds are zero)
    const int k0 = 16 * s_live[7], k1 = (L + 1) >> 1;   // layer pairs
    const uint32_t* ph = reinterpret_cast<const uint32_t*>(s_bhi);
    const uint32_t* pl = reinterpret_cast<const uint32_t*>(s_blo);
    uint32_t* dt = reinterpret_cast<uint32_t*>(dtau_out) + (size_t)b * Lp * npad + nu0;
    for (int e = tid; e < (k1 - k0) * kTileNu; e += kBlockT) {
      const int nu = e & (kTileNu - 1), k = k0 + e / kTileNu;
      const int a = nu * (stride >> 1) + k;
      const uint32_t hp = ph[a], lp = pl[a];
      __builtin_nontemporal_store(__builtin_amdgcn_perm(lp, hp, 0x05040100u), &dt[(size_t)(2 * k) * npad + nu]);
      if (2 * k + 1 < L)
        __builtin_nontemporal_store(__builtin_amdgcn_perm(lp, hp, 0x07060302u), &dt[(size_t)(2 * k + 1) * npad + nu]);
    }
  }
}

// FP64 element: bilinear log10 sigma, 2^(v log2 10 + lam)
template <int S, bool CIA>
__device__ inline double opacity_fp64(const Model& m, const Tables& tb, int cl, const double* __restrict__ rl, int nu,
                                      double nu4, double qext) {
  const int it = cl & 255, ip = (cl >> 8) & 255, itc = cl >> 16;
  const double wt = rl[0], wp = rl[1];
  const size_t npad = (size_t)m.n_nu_pad;
  double acc = rl[3] * nu4 + rl[4] * qext;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const double* p = tb.t64 + (((size_t)s * m.n_t + it) * m.n_p + ip) * npad + nu;
    const double v = (1.0 - wt) * (1.0 - wp) * p[0] + wt * (1.0 - wp) * p[(size_t)m.n_p * npad] +
                     (1.0 - wt) * wp * p[npad] + wt * wp * p[(size_t)(m.n_p + 1) * npad];
    acc += exp2(v * kLog2_10 + rl[kRecFixed + s]);
  }
  if (CIA) {
    const double wtc = rl[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const double* p = tb.tc64 + ((size_t)c * m.n_tc + itc) * npad + nu;
      acc += exp2(((1.0 - wtc) * p[0] + wtc * p[npad]) * kLog2_10 + rl[5 + c]);
    }
  }
  return acc;
}

template <int S, bool CIA>
__global__ __launch_bounds__(kBlock) void k_trans_fwd_fp64(Model m, Work w, Tables tb, int B, double* __restrict__ spec) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int logical = xcd_logical_block(blockIdx.x, gridDim.x);
  const int b = logical % B, tile = logical / B;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int Lp = m.L_pad;
  const int nu0 = tile * kTile64;
  double* out = spec + (size_t)b * m.n_nu;
  if (w.status[b]) {
    if (tid < kTile64 && nu0 + tid < m.n_nu) out[nu0 + tid] = __builtin_nan("");
    return;
  }
  const int L = w.nlay[b];
  double* s_dt = reinterpret_cast<double*>(lds);   // [Lp][64]
  double* s_red = s_dt + (size_t)Lp * kTile64;     // [4][64]
  const double* rec = reinterpret_cast<const double*>(w.rec) + (size_t)b * Lp * rec_len(S);
  const int32_t* cells = w.cells + (size_t)b * Lp;
  const int nu = nu0 + lane;
  const double nu4 = tb.nu4d[nu];
  // grey deck: the record holds the optical depth; non-grey: the column times Q_ext(nu)
  const double qext =
      m.cloud_ng ? cloud_q<double>(m.cloud_qext, load_cloud<double>(w.cloud + (size_t)b * kCloudSpec), m.nu[nu], nullptr)
                 : 1.0;
  for (int l = wv; l < L; l += 4)
    s_dt[l * kTile64 + lane] = opacity_fp64<S, CIA>(m, tb, cells[l], rec + (size_t)l * rec_len(S), nu, nu4, qext);
  __syncthreads();
  const double* pm = w.pm64 + (size_t)b * Lp * Lp;
  const double* area = reinterpret_cast<const double*>(w.area) + (size_t)b * Lp;
  double dsum = 0.0;
  for (int i = wv; i < L; i += 4) {
    const double* prow = pm + (size_t)i * Lp;
    double tau = 0.0;
    for (int l = i; l < L; ++l) tau = fma(prow[l], s_dt[l * kTile64 + lane], tau);
    dsum += area[i] * -expm1(-tau);
  }
  s_red[wv * kTile64 + lane] = dsum;
  __syncthreads();
  if (tid < kTile64) {
    const double tot = (s_red[tid] + s_red[kTile64 + tid]) + (s_red[2 * kTile64 + tid] + s_red[3 * kTile64 + tid]);
    if (nu0 + tid < m.n_nu) out[nu0 + tid] = w.core[b] + tot;
  }
}

// ---------------------------------------------------------------------------
// host side: one instance per (species count, CIA present)
template <bool F64, int S, bool CIA>
const void* fwd_kernel(bool ng, bool ks) {
  if constexpr (F64) return (const void*)k_trans_fwd_fp64<S, CIA>;
  else if (ks) return ng ? (const void*)k_trans_fwd_mixed<S, CIA, true, true> : (const void*)k_trans_fwd_mixed<S, CIA, false, true>;
  else return ng ? (const void*)k_trans_fwd_mixed<S, CIA, true, false> : (const void*)k_trans_fwd_mixed<S, CIA, false, false>;
}

template <bool F64>
const void* fwd_kernel_for(int S, bool cia, bool ng, bool ks = false) {
#define EXOFWD_CASE(n) \
  case n: return cia ? fwd_kernel<F64, n, true>(ng, ks) : fwd_kernel<F64, n, false>(ng, ks);
  switch (S) {
    EXOFWD_CASE(1) EXOFWD_CASE(2) EXOFWD_CASE(3) EXOFWD_CASE(4)
    EXOFWD_CASE(5) EXOFWD_CASE(6) EXOFWD_CASE(7) EXOFWD_CASE(8)
  }
#undef EXOFWD_CASE
  return nullptr;
}

static size_t fwd_lds_bytes(const Model& m, bool fp64, int lt, bool ks = false) {
  if (fp64) return (size_t)m.L_pad * kTile64 * 8 + 4 * kTile64 * 8;
  return (size_t)2 * kTileNu * (lt + 8) * 2 + (size_t)(ks ? m.L_pad : lt) * 4 + 8 * 32 * 8 + 8 * 4;
}

size_t trans_fwd_lds_bytes(const Model& m, bool fp64) { return fwd_lds_bytes(m, fp64, m.L_pad); }

hipError_t trans_fwd_configure(const Model& m, bool fp64) {
  const void* k = fp64 ? fwd_kernel_for<true>(m.S, m.has_cia, m.cloud_ng) : fwd_kernel_for<false>(m.S, m.has_cia, m.cloud_ng);
  if (!k) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)trans_fwd_lds_bytes(m, fp64));
  if (e != hipSuccess || fp64 || !layer_classes_used(m)) return e;
  const void* ks = fwd_kernel_for<false>(m.S, m.has_cia, m.cloud_ng, true);
  if (!ks) return hipErrorInvalidValue;
  return hipFuncSetAttribute(ks, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)fwd_lds_bytes(m, false, kShortLayers, true));
}

void launch_trans_fwd(const Model& m, const Work& w, const Tables& tb, int B, void* spec, bool fp64, hipStream_t st,
                      float* dtau_out) {
  const size_t lds = trans_fwd_lds_bytes(m, fp64);
  if (fp64) {
    void* args[] = {(void*)&m, (void*)&w, (void*)&tb, (void*)&B, (void*)&spec};
    hipLaunchKernel(fwd_kernel_for<true>(m.S, m.has_cia, m.cloud_ng), dim3((unsigned)(m.n_tiles64 * B)), dim3(kBlock), args, lds, st);
  } else {
    const void* k = fwd_kernel_for<false>(m.S, m.has_cia, m.cloud_ng);
    if (layer_classes_used(m)) {
      // samples of at most kShortLayers layers run with a kShortLayers-row LDS tile, the
      // rest with the same tile in two K chunks (two workgroups per CU either way); each
      // launch's grid covers the batch
      launch_layer_classes(m, w, B, st);
      const void* ks = fwd_kernel_for<false>(m.S, m.has_cia, m.cloud_ng, true);
      for (int cl = 0; cl < 2; ++cl) {
        const int32_t* cls = w.cls;
        int lt = kShortLayers;
        void* args[] = {(void*)&m, (void*)&w, (void*)&tb, (void*)&B, (void*)&spec, (void*)&dtau_out, (void*)&cls,
                        (void*)&cl, (void*)&lt};
        hipLaunchKernel(cl == 0 ? k : ks, dim3((unsigned)(m.n_tiles * B)), dim3(kBlockT), args,
                        fwd_lds_bytes(m, false, lt, cl == 1), st);
      }
      return;
    }
    const int32_t* cls = nullptr;
    int cl = 0, lt = m.L_pad;
    void* args[] = {(void*)&m, (void*)&w, (void*)&tb, (void*)&B, (void*)&spec, (void*)&dtau_out, (void*)&cls, (void*)&cl,
                    (void*)&lt};
    hipLaunchKernel(k, dim3((unsigned)(m.n_tiles * B)), dim3(kBlockT), args, lds, st);
  }
}

}  // namespace exofwd
