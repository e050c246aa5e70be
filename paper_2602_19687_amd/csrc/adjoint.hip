// Reverse pass of the transmission path.
//
// For every (sample, wavenumber chunk) a fused kernel takes the layer optical
// depths (stored by the forward kernel in the reduced-precision path,
// recomputed in FP64), forms the slant optical depth and the seeds
//   delta_bar(nu) = (d lnL / d m_k) / N_k          (nu in bin k)
//   tau_bar_i(nu) = delta_bar(nu) a_i e^{-tau_i(nu)}
// and accumulates, over its wavenumbers,
//   abar_i   = sum_nu delta_bar (1 - e^{-tau_i})                      (annulus areas)
//   Pbar_il  = sum_nu tau_bar_i dtau_l                                (path matrix)
//   dtau_bar = P^T tau_bar                                            (opacity)
// The per-layer sums of adjoint.h over dtau_bar are formed in the same kernel
// (FP64) or by a separate high-occupancy kernel from the stored dtau_bar
// (reduced precision). The FP64 chain kernel then walks back through the
// path-matrix geometry, the hydrostatic recursion, n = p/kT, chemistry, the
// cloud deck and the T-p profile to d lnL / d params.
#include "adjoint.h"
#include "kernels.h"
#include "cloud.h"
#include "opacity.h"
#include "tp.h"

namespace exofwd {

typedef __attribute__((ext_vector_type(4))) double f64x4;

// a float pair read once (stored dtau_bar): a non-temporal load
__device__ inline float2 ld_stream2(const float* p) {
  const float2v v = __builtin_nontemporal_load(reinterpret_cast<const float2v*>(p));
  return make_float2(v.x, v.y);
}

__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// cost-balanced split of 32-row blocks between `parts` (2 or 4) waves: each block in
// turn goes to the part with the least cost so far (the lowest such part on a tie);
// `rev` costs rows by their K extent in the transposed product (grows with the
// block index)
__host__ __device__ inline unsigned split_blocks(int part, int parts, int MBe, int KBe, bool rev) {
  unsigned mine = 0;
  int c[4] = {0, 0, 0, 0};
  for (int q = 0; q < MBe; ++q) {
    const int mi = rev ? MBe - 1 - q : q;
    const int cost = rev ? (2 * mi + 2 < KBe ? 2 * mi + 2 : KBe) : KBe - 2 * mi;
    int best = 0;
    for (int p = 1; p < parts; ++p)
      if (c[p] < c[best]) best = p;
    if (best == part) mine |= 1u << mi;
    c[best] += cost;
  }
  return mine;
}

// index of the q-th set bit of mask (or -1)
__device__ inline int nth_bit(unsigned mask, int q) {
  for (int i = 0; i < 32; ++i)
    if (mask & (1u << i)) {
      if (q == 0) return i;
      --q;
    }
  return -1;
}

// ============================================================================
// reduced-precision reverse kernel over TILE-wavenumber tiles for up to MB
// 32-row blocks (L_pad <= 32 MB); each wave owns one 32-wavenumber column block
// and one of PARTS cost-balanced parts of the row blocks, so every path-matrix
// fragment it loads feeds the products of its whole column block
template <int TILE, int MB, int PARTS>
struct AdjShape {
  static constexpr int kTile = TILE;
  static constexpr int kNb = TILE / 32;                           // column blocks per tile
  static constexpr int kWaves = PARTS * kNb;                      // PARTS row-block parts per column block
  static constexpr int kThreads = 64 * kWaves;
  static constexpr int kHalves = TILE / 64;                       // 64-wavenumber halves (phase A items)
  static constexpr int kSlots = PARTS == 2 ? (MB + 1) / 2 : (MB <= 4 ? 1 : 2);   // row blocks per wave (checked on the host)
  static constexpr int kPSlots = (MB * (MB + 1) / 2 + kWaves - 1) / kWaves;   // 32x32 Pbar tiles per wave
  static constexpr int kItems = (4 * kHalves * MB + kWaves - 1) / kWaves;     // (layer octet, half) items per wave
};

// `cls` (may be null): the layer-count classes of the call (layer_classes), whose class
// `cl` this launch serves (its samples have at most 32 MB layers)
template <int S, bool CIA, int TILE, int MB, int PARTS>
__global__ __launch_bounds__(2 * PARTS * TILE) void k_trans_adj_mixed(Model m, Work w, Tables tb, AdjWork aw, int B,
                                                                      int C, const int32_t* __restrict__ cls, int cl) {
  using Sh = AdjShape<TILE, MB, PARTS>;
  static_assert(Sh::kThreads == 2 * PARTS * TILE, "launch bound");
  static_assert(Sh::kItems * Sh::kWaves >= 4 * Sh::kHalves * MB, "phase A items cover 4 MB octets per half");
  constexpr int kTileA = Sh::kTile, kBlockA = Sh::kThreads, kNbA = Sh::kNb, kWavesA = Sh::kWaves;
  constexpr int kSlots = Sh::kSlots, kPSlotsA = Sh::kPSlots, kItemsA = Sh::kItems, kHalves = Sh::kHalves;
  extern __shared__ __align__(16) unsigned char lds[];
  const int logical = xcd_logical_block(blockIdx.x, gridDim.x);
  // a sample's chunks on neighbouring workgroups of one XCD: its path-matrix fragments,
  // re-read for every tile, stay in that XCD's L2 while its chunks run
  const int chunk = logical % C;
  int b = logical / C;
  if (cls) {
    // the class's samples, longest first, dealt round the XCDs; the grid covers the whole batch
    b = class_position(b, B, C);
    if (b >= cls[cl]) return;
    b = cls[2 + cl * B + b];
  }
  if (w.status[b]) return;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int Lp = m.L_pad, L = w.nlay[b];
  const int rows = Lp < 32 * MB ? Lp : 32 * MB;        // LDS rows: the layers this shape can hold
  // dwords per wavenumber row (b128-conflict-free), fixed by the shape rather than by
  // L_pad: the gathers of phase E then address eight rows from one register with
  // immediate offsets
  constexpr int ld = 32 * MB + 4;
  uint32_t* s_dt = reinterpret_cast<uint32_t*>(lds);   // dtau    [nu][ld] as packed bf16 hi/lo
  uint32_t* s_tt = s_dt + kTileA * ld;                 // tau_bar [nu][ld] as packed bf16 hi/lo
  float* s_area = reinterpret_cast<float*>(s_tt + kTileA * ld);   // [Lp]

  const float* area = reinterpret_cast<const float*>(w.area) + (size_t)b * Lp;
  for (int i = tid; i < rows; i += kBlockA) s_area[i] = area[i];

  const size_t npad = (size_t)m.n_nu_pad;
  const int KBe = (L + 15) >> 4, MBe = (L + 31) >> 5, KB = Lp >> 4;
  const int nb = wv % kNbA, part = wv / kNbA;
  // row blocks of this wave (slot q -> block index or -1), fixed for the whole call;
  // readfirstlane keeps them in scalar registers
  int t_mi[kSlots], d_ml[kSlots];
  {
    const unsigned mine_t = split_blocks(part, PARTS, MBe, KBe, false);   // rows i of tau
    const unsigned mine_d = split_blocks(part, PARTS, MBe, KBe, true);    // rows l of dtau_bar
#pragma unroll
    for (int q = 0; q < kSlots; ++q) {
      t_mi[q] = __builtin_amdgcn_readfirstlane(nth_bit(mine_t, q));
      d_ml[q] = __builtin_amdgcn_readfirstlane(nth_bit(mine_d, q));
    }
  }
  const size_t plane = (size_t)(Lp >> 5) * KB * 512;
  // this sample's P and P^T fragments (hi plane, then lo plane); lanes address
  // their 16 bytes with the vector offset, blocks with the scalar offset
  const __amdgpu_buffer_rsrc_t rs_p = make_rsrc(w.pfrag + (size_t)b * 2 * plane, 2 * plane * 2);
  const __amdgpu_buffer_rsrc_t rs_pt = make_rsrc(w.ptfrag + (size_t)b * 2 * plane, 2 * plane * 2);
  const uint32_t lo_plane = (uint32_t)plane * 2u, voff_f = (uint32_t)lane * 16u;
  auto frag = [&](__amdgpu_buffer_rsrc_t rs, int blk, uint32_t pl) {
    return __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(rs, voff_f, (uint32_t)blk * 1024u + pl, 0));
  };
  const int col = 32 * nb + (lane & 31);
  const int h = lane >> 5;
  const double* dm = w.dm + (size_t)b * m.K;
  // 32x32 product over k-steps [k_lo, k_hi): A = path-matrix fragments (rs) of blocks
  // row0 + k, B = the packed hi/lo rows 16k.. of the LDS array src at this wave's
  // column.  The fragments go in two groups of two steps: one group's loads are in
  // flight while the other group's products run.  Every iteration issues the same
  // loads (steps past k_hi read the next row block's fragments, or zeros past the
  // buffer's range, and are never used), so the waits count only the older group.
  auto kloop = [&](__amdgpu_buffer_rsrc_t rs, int row0, int k_lo, int k_hi, const uint32_t* src) {
    f32x16 acc = {};
    bf16x8 ga[2][2], gb[2][2];   // [step][hi, lo]
    auto load = [&](bf16x8 (&g)[2][2], int k) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        g[u][0] = frag(rs, row0 + k + u, 0);
        g[u][1] = frag(rs, row0 + k + u, lo_plane);
      }
    };
    auto product = [&](const bf16x8 (&g)[2][2], int k0) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int k = k0 + u;
        if (k >= k_hi) break;
        bf16x8 bh, bl;
        {
          const uint4 x0 = *reinterpret_cast<const uint4*>(src + col * ld + 16 * k + 8 * h);
          const uint4 x1 = *reinterpret_cast<const uint4*>(src + col * ld + 16 * k + 8 * h + 4);
          const uint32_t x[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
          frag_hl(x, bh, bl);
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(g[u][1], bh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(g[u][0], bl, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(g[u][0], bh, acc, 0, 0, 0);
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

  // Pbar tiles (32x32, column block >= row block), round-robin over the waves
  int pt_mi[kPSlotsA], pt_nl[kPSlotsA];
  {
    int t = 0;
    for (int q = 0; q < kPSlotsA; ++q) pt_mi[q] = pt_nl[q] = -1;
    for (int mi = 0; mi < MBe; ++mi)
      for (int nl = mi; nl < MBe; ++nl, ++t)
        if (t % kWavesA == wv && t / kWavesA < kPSlotsA) {
          pt_mi[t / kWavesA] = mi;
          pt_nl[t / kWavesA] = nl;
        }
#pragma unroll
    for (int q = 0; q < kPSlotsA; ++q) {
      pt_mi[q] = __builtin_amdgcn_readfirstlane(pt_mi[q]);
      pt_nl[q] = __builtin_amdgcn_readfirstlane(pt_nl[q]);
    }
  }
  f32x16 abar_acc[kSlots], pbar_acc[kPSlotsA];
#pragma unroll
  for (int q = 0; q < kSlots; ++q) abar_acc[q] = f32x16{};
#pragma unroll
  for (int q = 0; q < kPSlotsA; ++q) pbar_acc[q] = f32x16{};

  // this sample's stored optical depths and dtau_bar ([L_pad][n_nu_pad], rebased per tile)
  const float* dtau_b = aw.dtau + (size_t)b * Lp * npad;
  float* dtb_b = aw.dtb + (size_t)b * Lp * npad;
  const int ntiles = m.n_nu_pad / kTileA;
  const int t0 = chunk * ntiles / C, t1 = (chunk + 1) * ntiles / C;

  // the stored optical depths of a tile are fetched into registers while the
  // previous tile's Pbar product runs, then written to LDS as packed hi/lo:
  // items (layer octet o, half of the tile), a lane takes one wavenumber of the half
  uint32_t pf[kItemsA][8];   // packed bf16 hi | lo << 16, as the forward stored them
  // row offsets go in the scalar offset (wave-uniform, recomputed per tile); rows
  // [L, 32 MBe) lie inside the sample's L_pad rows and are replaced by zero when staged
  const __amdgpu_buffer_rsrc_t rs_dt = make_rsrc(dtau_b, (size_t)Lp * npad * 4);
  const uint32_t rowb = (uint32_t)npad * 4u;
  // layers below the tile's opaque frontier feed only chords whose seeds are zero
  // (nothing below reads them): they are neither fetched nor staged
  auto front_row = [&](int tile) { return 32 * w.front[(size_t)b * m.n_tiles + tile * kTileA / kTileNu]; };
  auto fetch = [&](int tile) {
    const int lo_row = front_row(tile);
#pragma unroll
    for (int q = 0; q < kItemsA; ++q) {
      const int it = wv + kWavesA * q;
      if (it >= 4 * kHalves * MBe) continue;   // 4 MBe layer octets per half
      const int o = it / kHalves;
      if (8 * o + 8 <= lo_row) {
#pragma unroll
        for (int j = 0; j < 8; ++j) pf[q][j] = 0u;
        continue;
      }
      const uint32_t voff = (uint32_t)(64 * (it % kHalves) + lane) * 4u;
      const uint32_t soff = (uint32_t)((8 * o * npad + (size_t)tile * kTileA) * 4);
#pragma unroll
      for (int j = 0; j < 8; ++j)
        pf[q][j] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rs_dt, voff, soff + j * rowb, kCpolStream);
    }
  };
  auto stage = [&](int tile) {
    // L passed through an empty asm: the row tests below are then formed where
    // they are used, instead of being hoisted out of the tile loop as 32 masks
    int Lq = L;
    asm volatile("" : "+s"(Lq));
    const int lo_row = front_row(tile);
#pragma unroll
    for (int q = 0; q < kItemsA; ++q) {
      const int it = wv + kWavesA * q;
      if (it >= 4 * kHalves * MBe) continue;   // 4 MBe layer octets per half
      const int o = it / kHalves, nu = 64 * (it % kHalves) + lane;
      uint32_t d[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) d[j] = (8 * o + j < Lq && 8 * o + j >= lo_row) ? pf[q][j] : 0u;
      uint32_t* dst = s_dt + nu * ld + 8 * o;
      *reinterpret_cast<uint4*>(dst) = make_uint4(d[0], d[1], d[2], d[3]);
      *reinterpret_cast<uint4*>(dst + 4) = make_uint4(d[4], d[5], d[6], d[7]);
    }
  };
  // ---- phase A of the first tile
  if (t0 < t1) {
    fetch(t0);
    stage(t0);
  }
  __syncthreads();

  for (int tile = t0; tile < t1; ++tile) {
    const int nu0 = tile * kTileA;
    // row blocks below mi0 hold only opaque chords (tau > kOpaqueTau across the
    // forward pass's 128-wavenumber tile): their seeds are exactly zero, so their
    // products are skipped and the results are those of the full computation
    const int mi0 = __builtin_amdgcn_readfirstlane(w.front[(size_t)b * m.n_tiles + nu0 / kTileNu]);

    // ---- phases B, C: tau = P dtau; seeds; tau_bar -> LDS [nu][i]; abar accumulation
    {
      const int nu_g = nu0 + col;
      const int bin = w.bin_of[nu_g];
      const float dbar = bin >= 0 ? (float)(dm[bin] * w.inv_cnt[bin]) : 0.0f;
#pragma unroll
      for (int q = 0; q < kSlots; ++q) {
        const int mi = t_mi[q];
        if (mi < 0) continue;
        if (mi < mi0) {
          // e^-tau = 0: abar takes dbar (1 - 0), tau_bar is 0
#pragma unroll
          for (int j = 0; j < 16; ++j) abar_acc[q][j] += dbar;
#pragma unroll
          for (int qd = 0; qd < 4; ++qd)
            *reinterpret_cast<uint4*>(s_tt + col * ld + 32 * mi + 8 * qd + 4 * h) = make_uint4(0u, 0u, 0u, 0u);
          continue;
        }
        const f32x16 acc = kloop(rs_p, mi * KB, 2 * mi, KBe, s_dt);
#pragma unroll
        for (int qd = 0; qd < 4; ++qd) {
          float tv[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int j = 4 * qd + r;
            const int row = 32 * mi + 8 * qd + 4 * h + r;
            const float e = exp2_fast(-1.4426950408889634f * acc[j]);
            abar_acc[q][j] = fmaf(dbar, one_minus_exp(acc[j], e), abar_acc[q][j]);
            tv[r] = dbar * s_area[row] * e;
          }
          *reinterpret_cast<uint4*>(s_tt + col * ld + 32 * mi + 8 * qd + 4 * h) =
              make_uint4(pack_hl(tv[0]), pack_hl(tv[1]), pack_hl(tv[2]), pack_hl(tv[3]));
        }
      }
    }
    __syncthreads();
    // ---- phase A of the next tile, part 1: its optical depths are in flight
    // while phase E (LDS and MFMA only) runs
    const bool more = tile + 1 < t1;
    if (more) fetch(tile + 1);

    // ---- phase E: Pbar += tau_bar dtau^T over the tile's wavenumbers (bf16x3 MFMA, k = wavenumber);
    // operands gathered from eight wavenumber rows of the packed hi/lo LDS arrays
#pragma unroll
    for (int q = 0; q < kPSlotsA; ++q) {
      const int mi = pt_mi[q], nl = pt_nl[q];
      if (mi < mi0) continue;   // also the empty slots (mi = -1): zero seeds add nothing
      const uint32_t* pa = s_tt + 8 * h * ld + 32 * mi + (lane & 31);
      const uint32_t* pbp = s_dt + 8 * h * ld + 32 * nl + (lane & 31);
#pragma unroll 1
      for (int ks = 0; ks < kTileA / 16; ++ks) {
        // the step's row offset kept opaque in a scalar register: each operand's eight
        // rows are then one address plus immediate offsets (the arrays lie past 64 KB)
        int off = 16 * ks * ld;
        asm volatile("" : "+s"(off));
        uint32_t va[8], vb[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          va[e] = pa[off + e * ld];
          vb[e] = pbp[off + e * ld];
        }
        bf16x8 ah, al, bh, bl;
        frag_hl(va, ah, al);
        frag_hl(vb, bh, bl);
        pbar_acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, pbar_acc[q], 0, 0, 0);
        pbar_acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, pbar_acc[q], 0, 0, 0);
        pbar_acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, pbar_acc[q], 0, 0, 0);
      }
    }
    // ---- phase A of the next tile, part 2: every wave is past phase E, the last
    // reader of this tile's dtau
    __syncthreads();
    if (more) stage(tile + 1);
    // ---- phase D: dtau_bar = P^T tau_bar (rows l, this wave's column block) -> HBM
    {
      const __amdgpu_buffer_rsrc_t rs_db = make_rsrc(dtb_b + nu0, ((size_t)Lp * npad - nu0) * 4);
#pragma unroll
      for (int q = 0; q < kSlots; ++q) {
        const int ml = d_ml[q];
        // rows below the opaque frontier would be exact zeros: the readers of
        // dtau_bar consult the frontier instead, so they are not stored
        if (ml < mi0) continue;
        const int kend = min(2 * ml + 2, KBe);
        // the seed rows of blocks below mi0 are zero: the sum starts at row 32 mi0
        const int kbeg = min(2 * mi0, kend);
        const f32x16 acc = kloop(rs_pt, ml * KB, kbeg, kend, s_tt);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int row = 32 * ml + 8 * (j >> 2) + 4 * h + (j & 3);
          // rows [L, 32 MBe) land in this sample's padding rows, which nothing reads
          // element copied to a scalar first: a bit_cast of a vector element lowers to element 0
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint((float)acc[j]), rs_db,
                                                (uint32_t)((row * npad + col) * 4), 0, kCpolStream);
        }
      }
    }
    __syncthreads();   // the next tile reads the staged dtau and overwrites tau_bar
  }

  // ---- write this chunk's partials
  const size_t pair = (size_t)b * C + chunk;
  float* pb = reinterpret_cast<float*>(aw.pbar) + pair * Lp * Lp;
#pragma unroll
  for (int q = 0; q < kPSlotsA; ++q) {
    const int mi = pt_mi[q], nl = pt_nl[q];
    if (mi < 0) continue;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int row = 32 * mi + 8 * (j >> 2) + 4 * h + (j & 3);
      pb[(size_t)row * Lp + 32 * nl + (lane & 31)] = pbar_acc[q][j];
    }
  }
  // abar: reduce over the 32 columns of each lane half, then over the column blocks
#pragma unroll
  for (int q = 0; q < kSlots; ++q) {
    const int mi = t_mi[q];
    if (mi < 0) continue;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      float v = abar_acc[q][j];
      for (int off = 16; off > 0; off >>= 1) v += __shfl_xor(v, off);
      abar_acc[q][j] = v;
    }
  }
  double* s_ab = reinterpret_cast<double*>(lds);   // [kNbA][Lp], all waves are past the loop
#pragma unroll
  for (int q = 0; q < kSlots; ++q) {
    const int mi = t_mi[q];
    if (mi < 0) continue;
    if ((lane & 31) == 0) {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int row = 32 * mi + 8 * (j >> 2) + 4 * h + (j & 3);
        s_ab[nb * Lp + row] = (double)abar_acc[q][j];
      }
    }
  }
  __syncthreads();
  double* ab = aw.abar + pair * Lp;
  for (int i = tid; i < Lp; i += kBlockA) {
    double v = 0.0;
    if (i < 32 * MBe)
#pragma unroll
      for (int n = 0; n < kNbA; ++n) v += s_ab[n * Lp + i];
    ab[i] = v;
  }
}

// a * h.x + c and a * h.y + c with the FP16 half taken as an operand of the FMA
// (v_fma_mix_f32): the same single rounding as converting it first, without a
// converted copy of the table pairs held in registers across a group's layers
__device__ inline float fma_f16lo(float a, half2_t h, float c) {
  float d;
  asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel_hi:[0,1,0]" : "=v"(d) : "v"(a), "v"(h), "v"(c));
  return d;
}
__device__ inline float fma_f16hi(float a, half2_t h, float c) {
  float d;
  asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel:[0,1,0] op_sel_hi:[0,1,0]" : "=v"(d) : "v"(a), "v"(h), "v"(c));
  return d;
}

// Line terms of one layer (and its CIA terms) for two wavenumbers with the
// derivative of each exponent with respect to the T weight: the arithmetic of
// eval_terms_deriv, with the line pairs entering their FMAs as FP16 operands
template <int S, bool CIA>
__device__ inline void eval_terms_deriv_f16(const LayerCoef<S>& c, const LaneConst<S>& k, const LayerRaw<S, CIA>& r,
                                            float* t0, float* t1, float* dw0, float* dw1) {
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const half2_t h00 = r.h[4 * s], h10 = r.h[4 * s + 1], h01 = r.h[4 * s + 2], h11 = r.h[4 * s + 3];
    const float cl0 = k.c0[s] + c.lam[s], cl1 = k.c1[s] + c.lam[s];
    const float u00 = fma_f16lo(c.omp, h00, fma_f16lo(c.wp, h01, cl0));
    const float u10 = fma_f16lo(c.omp, h10, fma_f16lo(c.wp, h11, cl0));
    const float u01 = fma_f16hi(c.omp, h00, fma_f16hi(c.wp, h01, cl1));
    const float u11 = fma_f16hi(c.omp, h10, fma_f16hi(c.wp, h11, cl1));
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

// ============================================================================
// reduced-precision per-layer sums: one wave per (sample, layer group, ls_tiles tiles),
// a layer group being a run of up to kLsGroup consecutive layers in one table cell
// (listed by the profile kernel), whose table pairs are fetched once per tile,
// together with the tile's dtau_bar; lanes hold two wavenumbers, partial sums stay
// in registers across the tiles and are reduced over the wave once

template <int S, bool CIA, bool NGC>
__global__ __launch_bounds__(kBlock) void k_layer_sums_mixed(Model m, Work w, Tables tb, AdjWork aw, int B) {
  constexpr int NS = n_sums(S);
  constexpr int kLs = kLsGroup;
  const int lane = threadIdx.x & 63;
  // consecutive waves (one wavenumber chunk) on one XCD: its L2 holds that chunk's table columns
  const int gw = xcd_logical_block(blockIdx.x, gridDim.x) * (kBlock / 64) +
                 __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int NG = m.L_max;   // groups per sample: at most one per layer
  const int per_chunk = B * NG;
  const int chunk = gw / per_chunk;
  if (chunk >= aw.lsum_chunks) return;
  const int rem = gw - chunk * per_chunk;
  const int b = rem / NG, lg = rem - b * NG;
  if (w.status[b]) return;
  const int Lp = m.L_pad;
  const int32_t* grp = w.lsg + (size_t)b * (Lp + 1);
  if (lg >= grp[0]) return;
  const int l0 = grp[1 + lg] & 0xffff, cnt = grp[1 + lg] >> 16;
  const size_t npad = (size_t)m.n_nu_pad;
  TableGeom g;
  g.row_bytes = (uint32_t)npad * 2u;
  g.tstep = (uint32_t)m.n_p * g.row_bytes;
  g.pstep = g.row_bytes;
  const __amdgpu_buffer_rsrc_t rh = make_rsrc(tb.h, (size_t)S * m.n_t * m.n_p * npad * 2);
  const __amdgpu_buffer_rsrc_t rhc = make_rsrc(CIA ? (const void*)tb.hc : (const void*)tb.h,
                                               CIA ? (size_t)2 * m.n_tc * npad * 2 : 0);
  const uint32_t voff = (uint32_t)lane * 4u;
  const float* rec = reinterpret_cast<const float*>(w.rec) + (size_t)b * Lp * rec_len_wide(S);
  const int32_t* cells = w.cells + (size_t)b * Lp;
  const float* dtb = aw.dtb + (size_t)b * Lp * npad;

  float acc[kLs][NS];
#pragma unroll
  for (int q = 0; q < kLs; ++q)
#pragma unroll
    for (int k = 0; k < NS; ++k) acc[q][k] = 0.0f;
  // non-grey cloud: Q_ext at the lane's two wavenumbers weights the cloud sum (its
  // spectral parameters are summed by k_cloud_spectral: more live registers here
  // would cost this kernel its load pipelining)
  const float* cq = NGC ? w.cloud_q + (size_t)b * (1 + kCloudSpec) * npad : nullptr;

  const int t0 = chunk * aw.ls_tiles, t1 = min(t0 + aw.ls_tiles, m.n_tiles);
  for (int tile = t0; tile < t1; ++tile) {
    const int nu0 = tile * kTileNu;
    // every chord through the group's layers opaque across the tile: dtau_bar is
    // exactly zero there and the tile adds nothing (the deep layers of most
    // atmospheres).  Rows below the reverse pass's opaque frontier are not stored.
    const int lo_row = 32 * w.front[(size_t)b * m.n_tiles + tile];
    if (l0 + cnt <= lo_row) continue;
    float2 dbq[kLs];
#pragma unroll
    for (int q = 0; q < kLs; ++q)
      dbq[q] = (q < cnt && l0 + q >= lo_row) ? ld_stream2(dtb + (size_t)(l0 + q) * npad + nu0 + 2 * lane)
                                             : make_float2(0.0f, 0.0f);
    // the group's table pairs, fetched with dtau_bar (one memory round trip per tile)
    // before the test that skips a tile whose dtau_bar is zero
    const LayerCoef<S> c0 = load_layer<S>(m, cells, rec, l0, (uint32_t)nu0 * 2u, g);
    LayerRaw<S, CIA> raw;
    fetch_terms<S, CIA>(c0, g, rh, rhc, voff, raw);
    const LaneConst<S> kc = load_lane<S, CIA>(m, tb, nu0 + 2 * lane);
    bool live = false;
#pragma unroll
    for (int q = 0; q < kLs; ++q) live |= dbq[q].x != 0.0f || dbq[q].y != 0.0f;
    if (__builtin_amdgcn_ballot_w64(live) == 0) continue;
    float q0 = 1.0f, q1 = 1.0f;
    if constexpr (NGC) {
      const float2 q = *reinterpret_cast<const float2*>(cq + nu0 + 2 * lane);
      q0 = q.x;
      q1 = q.y;
    }
#pragma unroll
    for (int q = 0; q < kLs; ++q) {
      if (q >= cnt) continue;
      const float2 db = dbq[q];
      const LayerCoef<S> c = q == 0 ? c0 : load_layer<S>(m, cells, rec, l0 + q, (uint32_t)nu0 * 2u, g);
      float t0_[S + 2], t1_[S + 2], dw0[S + 2], dw1[S + 2];
      eval_terms_deriv_f16<S, CIA>(c, kc, raw, t0_, t1_, dw0, dw1);
      // G_s += db t_s per wavenumber; the T-weight sums take db once per wavenumber
      // times z = sum_s t_s dw_s
      float z0 = 0.0f, z1 = 0.0f;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        acc[q][s] = fmaf(db.x, t0_[s], fmaf(db.y, t1_[s], acc[q][s]));
        z0 = fmaf(t0_[s], dw0[s], z0);
        z1 = fmaf(t1_[s], dw1[s], z1);
      }
      acc[q][S] = fmaf(db.x, z0, fmaf(db.y, z1, acc[q][S]));
      if (CIA) {
        float y0 = 0.0f, y1 = 0.0f;
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          acc[q][S + 1 + p] = fmaf(db.x, t0_[S + p], fmaf(db.y, t1_[S + p], acc[q][S + 1 + p]));
          y0 = fmaf(t0_[S + p], dw0[S + p], y0);
          y1 = fmaf(t1_[S + p], dw1[S + p], y1);
        }
        acc[q][S + 3] = fmaf(db.x, y0, fmaf(db.y, y1, acc[q][S + 3]));
      }
      acc[q][S + 4] = fmaf(db.x, kc.nu4_0, fmaf(db.y, kc.nu4_1, acc[q][S + 4]));
      if constexpr (NGC) {
        acc[q][S + 5] = fmaf(db.x, q0, fmaf(db.y, q1, acc[q][S + 5]));
      } else {
        acc[q][S + 5] += db.x + db.y;
      }
    }
  }
  float* out = aw.lsum + ((size_t)b * aw.lsum_stride + chunk) * Lp * NS;
#pragma unroll
  for (int q = 0; q < kLs; ++q) {
    const int l = l0 + q;
    if (q >= cnt) continue;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const float tot = wave_sum(acc[q][k]);
      if (lane == 0) out[(size_t)l * NS + k] = tot;
    }
  }
}

// Non-grey cloud: sums over wavenumber of G(nu) dQ_ext/dp_k with
// G(nu) = sum_l D_l dtau_bar_l(nu), the derivative of lnL along the cloud's
// spectral shape; one wave per (sample, layer-sum chunk), two wavenumbers per lane.
__global__ __launch_bounds__(kBlock) void k_cloud_spectral(Model m, Work w, AdjWork aw, int B) {
  const int lane = threadIdx.x & 63;
  const int gw = blockIdx.x * (kBlock / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int b = gw / aw.lsum_chunks, chunk = gw - b * aw.lsum_chunks;
  if (b >= B || w.status[b]) return;
  const int L = w.nlay[b], Lp = m.L_pad;
  const size_t npad = (size_t)m.n_nu_pad;
  const float* rec = reinterpret_cast<const float*>(w.rec) + (size_t)b * Lp * rec_len_wide(m.S);
  const float* dtb = aw.dtb + (size_t)b * Lp * npad;
  const float* cq = w.cloud_q + (size_t)b * (1 + kCloudSpec) * npad;
  float hq[kCloudSpec] = {};
  const int t0 = chunk * aw.ls_tiles, t1 = min(t0 + aw.ls_tiles, m.n_tiles);
  for (int tile = t0; tile < t1; ++tile) {
    const int nu = tile * kTileNu + 2 * lane;
    float g0 = 0.0f, g1 = 0.0f;
    // rows below the opaque frontier are zero (and not stored)
    for (int l = 32 * w.front[(size_t)b * m.n_tiles + tile]; l < L; ++l) {
      const float dl = rec[(size_t)l * rec_len_wide(m.S) + 4];
      const float2 d = *reinterpret_cast<const float2*>(dtb + (size_t)l * npad + nu);
      g0 = fmaf(dl, d.x, g0);
      g1 = fmaf(dl, d.y, g1);
    }
#pragma unroll
    for (int k = 0; k < kCloudSpec; ++k) {
      const float2 d = *reinterpret_cast<const float2*>(cq + (size_t)(1 + k) * npad + nu);
      hq[k] = fmaf(g0, d.x, fmaf(g1, d.y, hq[k]));
    }
  }
#pragma unroll
  for (int k = 0; k < kCloudSpec; ++k) {
    const float tot = wave_sum(hq[k]);
    if (lane == 0) aw.hq[((size_t)b * aw.lsum_stride + chunk) * kCloudSpec + k] = tot;
  }
}

// ============================================================================
// FP64 reverse kernel: 512 threads, 64-wavenumber tiles, VALU chord products,
// FP64 MFMA (16x16x4) for Pbar
template <int S, bool CIA>
__device__ inline void opacity_fp64_terms(const Model& m, const Tables& tb, int cl, const double* __restrict__ rl,
                                          int nu, double nu4, double& dtau, double* t, double* dw, double qext = 1.0) {
  const int it = cl & 255, ip = (cl >> 8) & 255, itc = cl >> 16;
  const double wt = rl[0], wp = rl[1];
  const size_t npad = (size_t)m.n_nu_pad;
  double acc = rl[3] * nu4 + rl[4] * qext;   // the non-grey cloud's column times Q_ext(nu)
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const double* p = tb.t64 + (((size_t)s * m.n_t + it) * m.n_p + ip) * npad + nu;
    const double t00 = p[0], t10 = p[(size_t)m.n_p * npad], t01 = p[npad], t11 = p[(size_t)(m.n_p + 1) * npad];
    const double v = (1.0 - wt) * (1.0 - wp) * t00 + wt * (1.0 - wp) * t10 + (1.0 - wt) * wp * t01 + wt * wp * t11;
    const double e = exp2(v * kLog2_10 + rl[kRecFixed + s]);
    acc += e;
    if (t) {
      t[s] = e;
      dw[s] = ((1.0 - wp) * (t10 - t00) + wp * (t11 - t01)) * kLog2_10;   // log2 units
    }
  }
  if (CIA) {
    const double wtc = rl[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const double* p = tb.tc64 + ((size_t)c * m.n_tc + itc) * npad + nu;
      const double e = exp2(((1.0 - wtc) * p[0] + wtc * p[npad]) * kLog2_10 + rl[5 + c]);
      acc += e;
      if (t) {
        t[S + c] = e;
        dw[S + c] = (p[npad] - p[0]) * kLog2_10;
      }
    }
  }
  dtau = acc;
}

// Two instances: TILE = 64 wavenumbers with ROWS = 16 rows per wave (L_pad <= 128),
// and TILE = 32 with ROWS = 20 (L_pad <= 160: the tile's dtau and tau_bar, 2 TILE
// (L_pad + 1) doubles, then fit in LDS; lanes 32-63 hold no wavenumber and add zeros).
// PSLOTS: 16x16 Pbar tiles per wave.
template <int S, bool CIA, int TILE, int ROWS, int PSLOTS>
__global__ __launch_bounds__(kBlockT) void k_trans_adj_fp64(Model m, Work w, Tables tb, AdjWork aw, int B, int C) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int logical = xcd_logical_block(blockIdx.x, gridDim.x);
  const int chunk = logical % C, b = logical / C;   // a sample's chunks on one XCD, as above
  if (w.status[b]) return;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int Lp = m.L_pad, L = w.nlay[b];
  constexpr int NS = n_sums(S);
  const int ld = Lp + 1;                              // padded row length (doubles)
  double* s_dt = reinterpret_cast<double*>(lds);      // dtau [nu][ld]
  double* s_tb = s_dt + TILE * ld;                    // tau_bar [nu][ld], later dtau_bar
  double* s_sums = s_tb + TILE * ld;                  // [Lp][NS]
  const bool act = lane < TILE;                       // this lane holds a wavenumber of the tile
  for (int i = tid; i < Lp * NS; i += kBlockT) s_sums[i] = 0.0;

  const double* rec = reinterpret_cast<const double*>(w.rec) + (size_t)b * Lp * rec_len(S);
  const int32_t* cells = w.cells + (size_t)b * Lp;
  const double* pm = w.pm64 + (size_t)b * Lp * Lp;
  const double* area = reinterpret_cast<const double*>(w.area) + (size_t)b * Lp;
  const double* dm = w.dm + (size_t)b * m.K;

  double abar_r[ROWS];
#pragma unroll
  for (int k = 0; k < ROWS; ++k) abar_r[k] = 0.0;
  // 16x16 Pbar tiles with column block >= row block, round-robin over waves
  const int MB16 = (L + 15) >> 4;
  int pt_mi[PSLOTS], pt_nl[PSLOTS];
  {
    int t = 0;
    for (int q = 0; q < PSLOTS; ++q) pt_mi[q] = pt_nl[q] = -1;
    for (int mi = 0; mi < MB16; ++mi)
      for (int nl = mi; nl < MB16; ++nl, ++t)
        if (t % 8 == wv && t / 8 < PSLOTS) {
          pt_mi[t / 8] = mi;
          pt_nl[t / 8] = nl;
        }
  }
  f64x4 pacc[PSLOTS];
#pragma unroll
  for (int q = 0; q < PSLOTS; ++q) pacc[q] = f64x4{0.0, 0.0, 0.0, 0.0};

  // non-grey cloud: Q_ext(nu) and its spectral derivatives, and (wave 0) the sums over
  // nu of G(nu) dQ/dp_k with G = sum_l D_l dtau_bar_l
  double hq[kCloudSpec] = {};
  CloudCoef<double> cc{};
  if (m.cloud_ng) cc = load_cloud<double>(w.cloud + (size_t)b * kCloudSpec);
  const int ntiles = m.n_nu_pad / TILE;
  const int t0 = chunk * ntiles / C, t1 = (chunk + 1) * ntiles / C;
  for (int tile = t0; tile < t1; ++tile) {
    const int nu = tile * TILE + (act ? lane : 0);
    const double nu4 = tb.nu4d[nu];
    double dqx[kCloudSpec];
    const double qx = m.cloud_ng ? cloud_q<double>(m.cloud_qext, cc, m.nu[nu], dqx) : 1.0;
    for (int l = wv; l < Lp; l += 8) {
      double d = 0.0;
      if (l < L && act) opacity_fp64_terms<S, CIA>(m, tb, cells[l], rec + (size_t)l * rec_len(S), nu, nu4, d, nullptr, nullptr, qx);
      if (act) s_dt[lane * ld + l] = d;
    }
    const int bin = w.bin_of[nu];
    const double dbar = bin >= 0 && act ? dm[bin] * w.inv_cnt[bin] : 0.0;
    __syncthreads();
    // tau_i, seeds, tau_bar
#pragma unroll
    for (int k = 0; k < ROWS; ++k) {
      const int i = wv + 8 * k;
      if (i < Lp) {
        double tbv = 0.0;
        if (i < L && act) {
          double tau = 0.0;
          for (int l = i; l < L; ++l) tau = fma(pm[(size_t)i * Lp + l], s_dt[lane * ld + l], tau);
          const double one_m_e = -expm1(-tau);
          abar_r[k] += dbar * one_m_e;
          tbv = dbar * area[i] * (1.0 - one_m_e);
        }
        if (act) s_tb[lane * ld + i] = tbv;
      }
    }
    __syncthreads();
    // Pbar += tau_bar dtau^T (FP64 MFMA, k = wavenumber)
#pragma unroll
    for (int q = 0; q < PSLOTS; ++q) {
      const int mi = pt_mi[q], nl = pt_nl[q];
      if (mi < 0) continue;
      const int ri = 16 * mi + (lane & 15), cl = 16 * nl + (lane & 15);
#pragma unroll 1
      for (int ks = 0; ks < TILE / 4; ++ks) {
        const int nr = 4 * ks + (lane >> 4);
        pacc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(s_tb[nr * ld + ri], s_dt[nr * ld + cl], pacc[q], 0, 0, 0);
      }
    }
    // dtau_bar_l = sum_{i <= l} P_il tau_bar_i
    double dtb[ROWS];
#pragma unroll
    for (int k = 0; k < ROWS; ++k) {
      const int l = wv + 8 * k;
      double acc = 0.0;
      if (l < L && act)
        for (int i = 0; i <= l; ++i) acc = fma(pm[(size_t)i * Lp + l], s_tb[lane * ld + i], acc);
      dtb[k] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < ROWS; ++k) {
      const int l = wv + 8 * k;
      if (l < Lp && act) s_tb[lane * ld + l] = dtb[k];
    }
    __syncthreads();
    if (m.cloud_ng && wv == 0) {
      double g = 0.0;
      if (act)
        for (int l = 0; l < L; ++l) g = fma(rec[(size_t)l * rec_len(S) + 4], s_tb[lane * ld + l], g);
#pragma unroll
      for (int k = 0; k < kCloudSpec; ++k) hq[k] = fma(g, dqx[k], hq[k]);
    }
    // per-layer sums
    for (int l = wv; l < L; l += 8) {
      double d, t[S + 2], dw[S + 2];
      opacity_fp64_terms<S, CIA>(m, tb, cells[l], rec + (size_t)l * rec_len(S), nu, nu4, d, t, dw, qx);
      const double db = act ? s_tb[lane * ld + l] : 0.0;
      double sums[NS];
      double ht = 0.0, htc = 0.0;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        sums[s] = db * t[s];
        ht += db * t[s] * dw[s];
      }
      sums[S] = ht;
      if (CIA) {
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          sums[S + 1 + p] = db * t[S + p];
          htc += db * t[S + p] * dw[S + p];
        }
      } else {
        sums[S + 1] = sums[S + 2] = 0.0;
      }
      sums[S + 3] = htc;
      sums[S + 4] = db * nu4;
      sums[S + 5] = db * qx;   // the cloud column: Q_ext weights the non-grey cloud (1 for the grey deck)
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const double tot = wave_sum(sums[k]);
        if (lane == 0) s_sums[l * NS + k] += tot;
      }
    }
    __syncthreads();
  }

  const size_t pair = (size_t)b * C + chunk;
  double* ls = aw.layer_sums + pair * Lp * NS;
  for (int i = tid; i < Lp * NS; i += kBlockT) ls[i] = s_sums[i];
  if (m.cloud_ng && wv == 0) {
#pragma unroll
    for (int k = 0; k < kCloudSpec; ++k) {
      const double tot = wave_sum(hq[k]);
      if (lane == 0) aw.hq64[pair * kCloudSpec + k] = tot;
    }
  }
  double* pb = reinterpret_cast<double*>(aw.pbar) + pair * Lp * Lp;
#pragma unroll
  for (int q = 0; q < PSLOTS; ++q) {
    const int mi = pt_mi[q], nl = pt_nl[q];
    if (mi < 0) continue;
#pragma unroll
    // v_mfma_f64_16x16x4f64 result: D[i][j] at lane j + 16 (i % 4), element i / 4
    for (int j = 0; j < 4; ++j) pb[(size_t)(16 * mi + (lane >> 4) + 4 * j) * Lp + 16 * nl + (lane & 15)] = pacc[q][j];
  }
  double* ab = aw.abar + pair * Lp;
#pragma unroll
  for (int k = 0; k < ROWS; ++k) {
    const int i = wv + 8 * k;
    const double v = wave_sum(abar_r[k]);
    if (lane == 0 && i < Lp) ab[i] = v;
  }
}

// ============================================================================
// FP64 chain: one workgroup per sample
__device__ inline void block_sum(double* s_red, int tid, int n) {
  // s_red[n][kBlock]: tree over the second index, result in s_red[k][0]
  for (int hh = kBlock / 2; hh > 0; hh >>= 1) {
    __syncthreads();
    if (tid < hh)
      for (int k = 0; k < n; ++k) s_red[k * kBlock + tid] += s_red[k * kBlock + tid + hh];
  }
  __syncthreads();
}

// derivatives of P_il with respect to r_l, r_{l+1} and b_i (l > i), or the
// full derivatives with respect to r_i, r_{i+1} on the diagonal
__device__ inline void path_derivs(const double* r, int i, int l, double& d_lo, double& d_up, double& d_b) {
  if (l == i) {
    const double dr = r[i + 1] - r[i];
    const double q = (3.0 * r[i + 1] + r[i]) / dr;
    const double sq = sqrt(q);
    d_up = (3.0 - q) / (2.0 * dr * sq);
    d_lo = (1.0 + q) / (2.0 * dr * sq);
    d_b = 0.0;
    return;
  }
  const double bb = 0.5 * (r[i] + r[i + 1]);
  const double rup = r[l + 1], rlo = r[l];
  const double sup = sqrt((rup - bb) * (rup + bb)), slo = sqrt((rlo - bb) * (rlo + bb));
  const double nn = 2.0 * (rup + rlo), den = sup + slo;
  const double f = nn / (den * den);
  d_up = 2.0 / den - f * rup / sup;
  d_lo = 2.0 / den - f * rlo / slo;
  d_b = f * bb * (1.0 / sup + 1.0 / slo);
}

// Slopes of the monotone cubic Hermite interpolant through (xk, yk) and their
// Jacobian J[k][j] = d slope_k / d y_j, following the branches of the slope rule
// used by the profile kernel (Fritsch-Butland weighted harmonic mean inside,
// three-point shape-preserving ends).
__device__ void pchip_slopes_jac(const double* xk, const double* yk, int n, double* d, double* J) {
  double h[kMaxKnots], del[kMaxKnots];
  for (int k = 0; k < n - 1; ++k) { h[k] = xk[k + 1] - xk[k]; del[k] = (yk[k + 1] - yk[k]) / h[k]; }
  for (int i = 0; i < n * n; ++i) J[i] = 0.0;
  // d del_k / d y_k = -1/h_k, d del_k / d y_{k+1} = 1/h_k
  auto add_del = [&](int row, int k, double c) {
    J[row * n + k] -= c / h[k];
    J[row * n + k + 1] += c / h[k];
  };
  if (n == 2) {
    d[0] = d[1] = del[0];
    add_del(0, 0, 1.0);
    add_del(1, 0, 1.0);
    return;
  }
  for (int k = 1; k < n - 1; ++k) {
    const double a = del[k - 1], b = del[k];
    if (a == 0.0 || b == 0.0 || (a > 0.0) != (b > 0.0)) {
      d[k] = 0.0;
    } else {
      const double w1 = 2.0 * h[k] + h[k - 1], w2 = h[k] + 2.0 * h[k - 1];
      const double den = w1 / a + w2 / b;
      d[k] = (w1 + w2) / den;
      add_del(k, k - 1, (w1 + w2) * w1 / (a * a * den * den));
      add_del(k, k, (w1 + w2) * w2 / (b * b * den * den));
    }
  }
  auto end = [&](int row, int i0, int i1) {
    const double h0 = h[i0], h1 = h[i1], m0 = del[i0], m1 = del[i1];
    const double dd = ((2.0 * h0 + h1) * m0 - h0 * m1) / (h0 + h1);
    auto sgn = [](double v) { return (v > 0.0) - (v < 0.0); };
    if (sgn(dd) != sgn(m0)) return 0.0;
    if (sgn(m0) != sgn(m1) && fabs(dd) > fabs(3.0 * m0)) {
      add_del(row, i0, 3.0);
      return 3.0 * m0;
    }
    add_del(row, i0, (2.0 * h0 + h1) / (h0 + h1));
    add_del(row, i1, -h0 / (h0 + h1));
    return dd;
  };
  d[0] = end(0, 0, 1);
  d[n - 1] = end(n - 1, n - 2, n - 3);
}

template <typename PbarT>
__global__ __launch_bounds__(kBlock) void k_chain(Model m, Work w, AdjWork aw, int C, int Cn, const double* __restrict__ params,
                                                  const uint8_t* __restrict__ mask, double* __restrict__ grad) {
  const int b = blockIdx.x, tid = threadIdx.x;
  const int Lp = m.L_pad;
  const int NS = n_sums(m.S);
  const int NT = sizeof(PbarT) == 8 ? NS : n_lsums(m);   // stride of the stored layer sums
  double* gout = grad + (size_t)b * m.P;
  if (w.status[b]) {
    for (int k = tid; k < m.P; k += kBlock) gout[k] = 0.0;
    return;
  }
  const int L = w.nlay[b];
  // virtual sample b of real sample real_sample(m, b); a clear one has no cloud terms
  const double* th = params + (size_t)real_sample(m, b) * m.P;
  const bool cloudy = m.has_cloud && !clear_sample(m, b);
  const bool ng = m.cloud_ng && cloudy;
  __shared__ double s_r[kMaxLayers + 1], s_rb[kMaxLayers + 1], s_ub[kMaxLayers + 1];
  __shared__ double s_t[kMaxLayers], s_tb[kMaxLayers], s_lndr[kMaxLayers];
  __shared__ double s_clo[kMaxLayers], s_cup[kMaxLayers], s_bb[kMaxLayers];
  __shared__ double s_red[16 * kBlock];
  __shared__ double s_scal[8];

  const double* rl = w.r_lev + (size_t)b * (Lp + 1);
  const double* tl = w.t_lay + (size_t)b * Lp;
  for (int j = tid; j <= L; j += kBlock) s_r[j] = rl[j];
  for (int l = tid; l < L; l += kBlock) s_t[l] = tl[l];

  // chemistry and constants (every thread)
  double x[kMaxSpecies];
  double sx = 0.0;
  for (int s = 0; s < m.S; ++s) { x[s] = exp10(th[m.n_tp + s]); sx += x[s]; }
  const double xh2 = (1.0 - sx) / (1.0 + kHeH2), xhe = kHeH2 * xh2;
  const bool mu_free = !(m.mu_fixed > 0.0);
  double mu = m.mu_fixed;
  if (mu_free) {
    mu = xh2 * kMH2 + xhe * kMHe;
    for (int s = 0; s < m.S; ++s) mu += x[s] * m.mass[s];
  }
  const double scale = m.has_scale ? th[m.idx_scale] : 1.0;
  const double g_ref = m.has_bd ? exp10(th[m.idx_bd]) : m.g_ref;
  const double r_ref = m.has_bd ? sqrt(kGrav * th[m.idx_bd + 1] * kMJup / g_ref) : m.r_p * scale;
  const double kk = kB / (mu * kMu * g_ref * r_ref * r_ref);
  const double step = (m.log10_ptop - m.log10_pbot) / L;
  const double ln10 = 2.302585092994045684017991454684;
  const double dlnp = -step * ln10;
  auto logp_lev = [&](int j) { return j == L ? m.log10_ptop : m.log10_pbot + j * step; };
  const double rs2 = m.r_s * m.r_s;
  const double log10_pc = m.has_cloud ? th[m.idx_cloud] : 0.0;
  // non-grey cloud: D_l = q_l rho_l dr_l 3 / (4 r_eff); profile parameters start at q_first
  const int q_first = m.idx_cloud + (m.cloud_qext == kQextGrey ? 1 : 3);
  const double r_eff = m.cloud_ng ? 1.0e-4 * exp10(th[m.idx_cloud]) : 1.0;
  auto layer_sum = [&](int l, int k) {
    double v = 0.0;
    if constexpr (sizeof(PbarT) == 8) {
      if (m.mode == kEmission) {
        for (int c = 0; c < aw.lsum_chunks; ++c) v += aw.lsum64[(((size_t)b * aw.lsum_stride + c) * Lp + l) * NS + k];
      } else {
        for (int c = 0; c < Cn; ++c) v += aw.layer_sums[(((size_t)b * C + c) * Lp + l) * NS + k];
      }
    } else {
      for (int c = 0; c < aw.lsum_chunks; ++c) v += (double)aw.lsum[(((size_t)b * aw.lsum_stride + c) * Lp + l) * NT + k];
    }
    return v;
  };
  __syncthreads();

  // per-layer sums reduced over chunks, and the per-layer chain through
  // n = p/kT, dr, the Rayleigh and cloud prefactors; accumulators for chemistry
  // go to s_red rows: [0,S) lnX_s, S lnXH2, S+1 lnXHe, S+2 XH2 direct,
  // S+3 XHe direct, S+4 ln mu, S+5 theta_cloud
  const int NR = m.S + 6;
  for (int k = 0; k < NR; ++k) s_red[k * kBlock + tid] = 0.0;
  for (int l = tid; l < L; l += kBlock) {
    constexpr int kMaxNS = kMaxSpecies + kExtraSums;
    double sm[kMaxNS];
    if constexpr (sizeof(PbarT) == 8) {
      for (int k = 0; k < NS; ++k) sm[k] = layer_sum(l, k);
    } else {
      // chunk by chunk with a chunk's sums loaded together; each sum still adds
      // its chunks in chunk order
      for (int k = 0; k < NS; ++k) sm[k] = 0.0;
      for (int c = 0; c < aw.lsum_chunks; ++c) {
        const float* src = aw.lsum + (((size_t)b * aw.lsum_stride + c) * Lp + l) * NT;
        float v[kMaxNS];
#pragma unroll
        for (int k = 0; k < kMaxNS; ++k) v[k] = k < NS ? src[k] : 0.0f;
#pragma unroll
        for (int k = 0; k < kMaxNS; ++k)
          if (k < NS) sm[k] += (double)v[k];
      }
    }
    const double t = s_t[l];
    const double lp_bar = 0.5 * (logp_lev(l) + logp_lev(l + 1));
    const double n = exp10(lp_bar) * kBar / (kB * t);
    const double dr = s_r[l + 1] - s_r[l];
    const double rr = (m.has_ray ? n * (xh2 * m.ray_h2 + xhe * m.ray_he) * dr : 0.0);
    double f = 0.0, dd = 0.0;
    if (ng) {
      dd = condensate_q(m.cloud_profile, th + q_first, logp_lev(l), logp_lev(l + 1), lp_bar, nullptr) * mu * kMu * n *
           dr * 0.75 / r_eff;
    } else if (cloudy) {
      f = (logp_lev(l) - log10_pc) * ln10 / dlnp;
      f = f < 0.0 ? 0.0 : (f > 1.0 ? 1.0 : f);
      dd = m.kappa_cloud * mu * kMu * n * f * dr;
    }
    double gline = 0.0;
    for (int s = 0; s < m.S; ++s) gline += sm[s];
    const double gc1 = sm[m.S + 1], gc2 = sm[m.S + 2], gr = sm[m.S + 4], gd = sm[m.S + 5];
    const double lnn_bar = gline + 2.0 * gc1 + 2.0 * gc2 + gr * rr + gd * dd;
    const double lndr_bar = gline + gc1 + gc2 + gr * rr + gd * dd;
    s_lndr[l] = lndr_bar / dr;
    // dT from n = p/kT and from the table weights (interior cells only)
    double tbar = -lnn_bar / t;
    const double ln2 = 0.69314718055994530941723212145818;
    if (t > m.t_grid[0] && t < m.t_grid[m.n_t - 1]) {
      int lo = 0, hi = m.n_t - 1;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (m.t_grid[mid] <= t) lo = mid; else hi = mid;
      }
      tbar += ln2 * sm[m.S] / (m.t_grid[lo + 1] - m.t_grid[lo]);
    }
    if (m.has_cia && t > m.tc_grid[0] && t < m.tc_grid[m.n_tc - 1]) {
      int lo = 0, hi = m.n_tc - 1;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (m.tc_grid[mid] <= t) lo = mid; else hi = mid;
      }
      tbar += ln2 * sm[m.S + 3] / (m.tc_grid[lo + 1] - m.tc_grid[lo]);
    }
    s_tb[l] = tbar;
    for (int s = 0; s < m.S; ++s) s_red[s * kBlock + tid] += sm[s];
    s_red[(m.S) * kBlock + tid] += 2.0 * gc1 + gc2;
    s_red[(m.S + 1) * kBlock + tid] += gc2;
    s_red[(m.S + 2) * kBlock + tid] += gr * n * dr * m.ray_h2;
    s_red[(m.S + 3) * kBlock + tid] += gr * n * dr * m.ray_he;
    s_red[(m.S + 4) * kBlock + tid] += gd * dd;
    if (cloudy && !m.cloud_ng && f > 0.0 && f < 1.0)
      s_red[(m.S + 5) * kBlock + tid] += gd * m.kappa_cloud * mu * kMu * n * dr * (-ln10 / dlnp);
  }
  block_sum(s_red, tid, NR);
  double chem[kMaxSpecies + 6];
  for (int k = 0; k < NR; ++k) chem[k] = s_red[k * kBlock];
  __syncthreads();

  // non-grey cloud parameters: rows [0, kCloudSpec) the spectral parameters
  // (log10 r also through the column's 1/r_eff), then the three profile parameters
  __shared__ double s_cloud[kCloudSpec + 3];
  if (m.cloud_ng) {
    constexpr int NC = kCloudSpec + 3;
    for (int k = 0; k < NC; ++k) s_red[k * kBlock + tid] = 0.0;
    for (int l = tid; l < (ng ? L : 0); l += kBlock) {   // a clear virtual sample keeps zeros
      const double gd = layer_sum(l, m.S + 5);
      const double lp_bar = 0.5 * (logp_lev(l) + logp_lev(l + 1));
      const double n = exp10(lp_bar) * kBar / (kB * s_t[l]);
      const double col = mu * kMu * n * (s_r[l + 1] - s_r[l]) * 0.75 / r_eff;
      double dq[3];
      const double q = condensate_q(m.cloud_profile, th + q_first, logp_lev(l), logp_lev(l + 1), lp_bar, dq);
      s_red[tid] -= ln10 * gd * q * col;
      for (int k = 0; k < 3; ++k) s_red[(kCloudSpec + k) * kBlock + tid] += gd * col * dq[k];
    }
    // spectral parameters: the per-chunk sums of k_cloud_spectral
    if constexpr (sizeof(PbarT) == 8) {
      for (int i = tid; i < (ng ? C * kCloudSpec : 0); i += kBlock)
        s_red[(i % kCloudSpec) * kBlock + tid] += aw.hq64[(size_t)b * C * kCloudSpec + i];
    } else {
      for (int i = tid; i < (ng ? aw.lsum_chunks * kCloudSpec : 0); i += kBlock)
        s_red[(i % kCloudSpec) * kBlock + tid] += (double)aw.hq[((size_t)b * aw.lsum_stride) * kCloudSpec + i];
    }
    block_sum(s_red, tid, NC);
    if (tid < NC) s_cloud[tid] = s_red[tid * kBlock];
    __syncthreads();
  }

  // path-matrix adjoint: column pass (r_l, r_{l+1}) and row pass (b_i); four entries'
  // loads are issued together, each entry summed over the chunks in chunk order.  Each
  // column's (row's) entries are split into nseg contiguous segments on different
  // threads (the longest column set the pace of the whole block); the segments'
  // partial sums, kept in s_red (free here), are added in segment order
  const PbarT* pbar = reinterpret_cast<const PbarT*>(aw.pbar) + (size_t)b * C * Lp * Lp;
  const size_t pst = (size_t)Lp * Lp;
  const bool trans = m.mode == kTransmission;
  constexpr int kMaxSeg = 4;
  const int nseg = trans ? max(1, min(kMaxSeg, kBlock / max(L, 1))) : 1;
  double* s_plo = s_red;                              // [kMaxSeg][kMaxLayers]
  double* s_pup = s_red + kMaxSeg * kMaxLayers;
  double* s_pb = s_red + 2 * kMaxSeg * kMaxLayers;
  for (int t = tid; t < (trans ? nseg * L : 0); t += kBlock) {
    const int l = t % L, sg = t / L;
    const int ia = sg * (l + 1) / nseg, ib = (sg + 1) * (l + 1) / nseg;   // rows i <= l
    double clo = 0.0, cup = 0.0;
    for (int i0 = ia; i0 < ib; i0 += 4) {
      double p[4] = {0.0, 0.0, 0.0, 0.0};
      for (int c = 0; c < Cn; ++c)
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (i0 + u < ib) p[u] += (double)pbar[c * pst + (size_t)(i0 + u) * Lp + l];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (i0 + u >= ib) break;
        double dlo, dup, db;
        path_derivs(s_r, i0 + u, l, dlo, dup, db);
        clo += p[u] * dlo;
        cup += p[u] * dup;
      }
    }
    s_plo[sg * kMaxLayers + l] = clo;
    s_pup[sg * kMaxLayers + l] = cup;
  }
  for (int t = tid; t < (trans ? nseg * L : 0); t += kBlock) {
    const int i = t % L, sg = t / L, n = L - 1 - i;   // columns l = i + 1 .. L - 1
    const int la = i + 1 + sg * n / nseg, lb = i + 1 + (sg + 1) * n / nseg;
    double acc = 0.0;
    for (int l0 = la; l0 < lb; l0 += 4) {
      double p[4] = {0.0, 0.0, 0.0, 0.0};
      for (int c = 0; c < Cn; ++c)
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (l0 + u < lb) p[u] += (double)pbar[c * pst + (size_t)i * Lp + l0 + u];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (l0 + u >= lb) break;
        double dlo, dup, db;
        path_derivs(s_r, i, l0 + u, dlo, dup, db);
        acc += p[u] * db;
      }
    }
    s_pb[sg * kMaxLayers + i] = acc;
  }
  __syncthreads();
  for (int l = tid; l < (trans ? L : 0); l += kBlock) {
    double clo = 0.0, cup = 0.0, bb = 0.0;
    for (int sg = 0; sg < nseg; ++sg) {
      clo += s_plo[sg * kMaxLayers + l];
      cup += s_pup[sg * kMaxLayers + l];
      bb += s_pb[sg * kMaxLayers + l];
    }
    s_clo[l] = clo;
    s_cup[l] = cup;
    s_bb[l] = bb;
  }
  __syncthreads();   // s_red is reused below
  // emission: no chord; the levels move the optical depths only through dr
  for (int l = tid; l < (trans ? 0 : L); l += kBlock) s_clo[l] = s_cup[l] = s_bb[l] = 0.0;
  // seed of the core term: the bins' d lnL / d depth summed over the block
  // (s_red is free between the cloud sums and the T-p sums)
  double cb = 0.0;
  for (int k = tid; k < m.K; k += kBlock) cb += w.dm[(size_t)b * m.K + k];
  s_red[tid] = cb;
  block_sum(s_red, tid, 1);
  const double core_bar = s_red[0];
  for (int j = tid; j <= L; j += kBlock) {
    double rb = 0.0;
    double ab_j = 0.0, ab_jm = 0.0;
    for (int c = 0; c < (trans ? Cn : 0); ++c) {
      if (j < L) ab_j += aw.abar[((size_t)b * C + c) * Lp + j];
      if (j >= 1) ab_jm += aw.abar[((size_t)b * C + c) * Lp + j - 1];
    }
    if (j < L) rb += s_clo[j] + 0.5 * s_bb[j] - 2.0 * s_r[j] * ab_j / rs2 - s_lndr[j];
    if (j >= 1) rb += s_cup[j - 1] + 0.5 * s_bb[j - 1] + 2.0 * s_r[j] * ab_jm / rs2 + s_lndr[j - 1];
    if (j == 0 && trans) rb += 2.0 * s_r[0] * core_bar / rs2;
    s_rb[j] = rb;
    s_ub[j] = -rb * s_r[j] * s_r[j];
  }
  __syncthreads();

  // hydrostatic recursion in reverse (sequential over levels)
  if (tid == 0) {
    const double lpref = log10(m.p_ref / kBar);
    int cnt = 0;
    for (int j = 0; j <= L; ++j) cnt += logp_lev(j) > lpref;
    const int lref = min(max(cnt - 1, 0), L - 1);
    const double a1 = (logp_lev(lref) - lpref) * ln10, a2 = (lpref - logp_lev(lref + 1)) * ln10;
    double ub_ref = 0.0, kbar = 0.0;
    // Q_j = (u_j - u_ref)/K from the same recursion
    double q = s_t[lref] * a1;
    double pre = 0.0;   // sum_{j <= l} ub_j, built from the bottom
    for (int j = 0; j <= L; ++j) ub_ref += s_ub[j];
    // levels at and below lref
    double qj = q;
    kbar += s_ub[lref] * qj;
    for (int j = lref - 1; j >= 0; --j) {
      qj += s_t[j] * dlnp;
      kbar += s_ub[j] * qj;
    }
    qj = -s_t[lref] * a2;
    kbar += s_ub[lref + 1] * qj;
    for (int j = lref + 2; j <= L; ++j) {
      qj -= s_t[j - 1] * dlnp;
      kbar += s_ub[j] * qj;
    }
    // temperatures
    double below = 0.0;
    for (int j = 0; j <= lref; ++j) below += s_ub[j];
    double above = ub_ref - below;
    s_tb[lref] += kk * (a1 * below - a2 * above);
    pre = 0.0;
    for (int l = 0; l < lref; ++l) {
      pre += s_ub[l];
      s_tb[l] += kk * dlnp * pre;
    }
    double suf = 0.0;
    for (int l = L - 1; l > lref; --l) {
      suf += s_ub[l + 1];
      s_tb[l] -= kk * dlnp * suf;
    }
    s_scal[0] = -ub_ref / (r_ref * r_ref) - 2.0 * kbar * kk / r_ref;   // d lnL / d R_ref
    // emission: the ratio carries (R_ref/R_s)^2, and sum_nu dlnL/dspec spec = mdot
    if (!trans) s_scal[0] += 2.0 * w.mdot[b] / r_ref;
    s_scal[1] = -kbar * kk;                                            // d lnL / d ln mu (hydrostatics)
  }
  __syncthreads();

  // T-p profile: layer temperatures (opacity, hydrostatics) and, in emission, the
  // level temperatures of the Planck sources, each at its own pressure
  __shared__ double s_kx[kMaxKnots], s_ky[kMaxKnots], s_kd[kMaxKnots], s_kj[kMaxKnots * kMaxKnots];
  if (m.tp_kind == kTpPchip && tid == 0) {
    for (int k = 0; k < m.n_knots; ++k) {
      s_kx[k] = m.n_knots == 1 ? m.log10_ptop : m.log10_ptop + k * ((m.log10_pbot - m.log10_ptop) / (m.n_knots - 1));
      s_ky[k] = th[k];
    }
    s_kx[m.n_knots - 1] = m.log10_pbot;
    pchip_slopes_jac(s_kx, s_ky, m.n_knots, s_kd, s_kj);
  }
  // slot n_tp: the profile's share of d lnL / d log10 g (tau = kappa_ir p / g) for an isolated object
  const int n_red = m.n_tp + m.has_bd;
  for (int k = 0; k < n_red; ++k) s_red[k * kBlock + tid] = 0.0;
  __syncthreads();
  auto tp_grad = [&](double lp, double t, double tbar) {
    if (m.tp_kind == kTpIso) {
      s_red[tid] += tbar;
    } else if (m.tp_kind == kTpGuillot3) {
      const double tau = m.kappa_ir * exp10(lp) * kBar / g_ref;
      const double t3 = t * t * t;
      const double s3 = 1.7320508075688772935274463415059;
      const double gam = exp10(th[2]);
      const double e = exp(-gam * tau * s3);
      const double bk = 2.0 / 3.0 + 1.0 / (gam * s3) + (gam / s3 - 1.0 / (gam * s3)) * e;
      const double dbk = -1.0 / (gam * gam * s3) + (1.0 / s3 + 1.0 / (gam * gam * s3)) * e +
                         (gam / s3 - 1.0 / (gam * s3)) * e * (-tau * s3);
      const double ti = th[0], te = th[1];
      s_red[tid] += tbar * 3.0 * ti * ti * ti * (2.0 / 3.0 + tau) / (4.0 * t3);
      s_red[kBlock + tid] += tbar * 12.0 * m.f_hem * te * te * te * bk / (4.0 * t3);
      s_red[2 * kBlock + tid] += tbar * 3.0 * m.f_hem * te * te * te * te * dbk * gam * ln10 / (4.0 * t3);
      if (m.has_bd) {
        // d T^4 / d tau times d tau / d log10 g = -tau ln 10
        const double dt4 = 0.75 * ti * ti * ti * ti - 3.0 * m.f_hem * te * te * te * te * (gam / s3 - 1.0 / (gam * s3)) * e * gam * s3;
        s_red[3 * kBlock + tid] -= tbar * dt4 * tau * ln10 / (4.0 * t3);
      }
    } else if (m.tp_kind == kTpBarstow) {
      s_red[tid] += tbar * barstow_factor(lp);
    } else if (m.tp_kind == kTpMilne || m.tp_kind == kTpGuillot7) {
      double d4[7];
      if (m.tp_kind == kTpMilne) milne_t4(th, lp, g_ref, d4);
      else guillot7_t4(th, lp, g_ref, m.f_hem, d4);
      const double inv = tbar / (4.0 * t * t * t);
      for (int k = 0; k < m.n_tp; ++k) s_red[k * kBlock + tid] += d4[k] * inv;
      // tau depends on kappa_ir / g: d/d log10 g = -d/d log10 kappa_ir
      if (m.has_bd) s_red[m.n_tp * kBlock + tid] -= d4[m.tp_kind == kTpMilne ? 1 : 2] * inv;
    } else {
      // T = h00 y_k + h10 h d_k + h01 y_k+1 + h11 h d_k+1 on the knot interval holding lp
      const int n = m.n_knots;
      int k = 0;
      while (k < n - 2 && s_kx[k + 1] <= lp) ++k;
      const double hk = s_kx[k + 1] - s_kx[k];
      const double u = (lp - s_kx[k]) / hk, omu = 1.0 - u;
      const double h00 = (1.0 + 2.0 * u) * omu * omu, h10 = u * omu * omu, h01 = u * u * (3.0 - 2.0 * u),
                   h11 = u * u * (u - 1.0);
      for (int j = 0; j < n; ++j) {
        double dtdy = hk * (h10 * s_kj[k * n + j] + h11 * s_kj[(k + 1) * n + j]);
        if (j == k) dtdy += h00;
        if (j == k + 1) dtdy += h01;
        s_red[j * kBlock + tid] += tbar * dtdy;
      }
    }
  };
  for (int l = tid; l < L; l += kBlock) tp_grad(0.5 * (logp_lev(l) + logp_lev(l + 1)), s_t[l], s_tb[l]);
  if (!trans) {
    const double* tlev = w.t_lev + (size_t)b * (Lp + 1);
    for (int j = tid; j <= L; j += kBlock) {
      double tb = 0.0;
      const size_t i0 = (size_t)b * m.n_tiles64 * (Lp + 1) + j;
      for (int t0 = 0; t0 < m.n_tiles64; t0 += 4) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const size_t i = i0 + (size_t)(t0 + u) * (Lp + 1);
          if (t0 + u >= m.n_tiles64) v[u] = 0.0;
          else if constexpr (sizeof(PbarT) == 8) v[u] = aw.psum64[i];
          else v[u] = (double)aw.psum[i];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (t0 + u < m.n_tiles64) tb += v[u];
      }
      tp_grad(logp_lev(j), tlev[j], tb);
    }
  }
  block_sum(s_red, tid, n_red);
  if (tid == 0) {
    for (int k = 0; k < m.n_tp; ++k) gout[k] = s_red[k * kBlock];
    if (m.has_bd) {
      // g R_ref^2 = G M fixes the hydrostatic constant: ln g enters at fixed R_ref like ln mu
      // (s_scal[1]) and through R_ref = sqrt(G M / g) (s_scal[0] = d lnL / d R_ref)
      gout[m.idx_bd] = (s_scal[1] - 0.5 * r_ref * s_scal[0]) * ln10 + s_red[m.n_tp * kBlock];
      gout[m.idx_bd + 1] = 0.5 * r_ref * s_scal[0] / th[m.idx_bd + 1];
    }
    // chemistry: X_H2 = (1 - sum X)/1.164, X_He = 0.164 X_H2, mu = sum X m
    const double lnmu_bar = chem[m.S + 4] + s_scal[1];
    const double mu_bar = mu_free ? lnmu_bar / mu : 0.0;
    const double xhe_bar = chem[m.S + 1] / xhe + chem[m.S + 3] + mu_bar * kMHe;
    const double xh2_bar = chem[m.S] / xh2 + chem[m.S + 2] + mu_bar * kMH2 + kHeH2 * xhe_bar;
    for (int s = 0; s < m.S; ++s) {
      const double xb = chem[s] / x[s] + mu_bar * m.mass[s] - xh2_bar / (1.0 + kHeH2);
      gout[m.n_tp + s] = xb * x[s] * ln10;
    }
    if (m.has_cloud && !m.cloud_ng) gout[m.idx_cloud] = chem[m.S + 5];
    if (m.cloud_ng) {
      // theta order: log10 r, [a, log10 Q0], profile (1 or 3), [A, lambda0, log10 omega, xi]
      int k = m.idx_cloud;
      gout[k++] = s_cloud[0];
      if (m.cloud_qext != kQextGrey) { gout[k++] = s_cloud[1]; gout[k++] = s_cloud[2]; }
      const int np = m.cloud_profile == kQprofUniform ? 1 : 3;
      for (int j = 0; j < np; ++j) gout[k++] = s_cloud[kCloudSpec + j];
      if (m.cloud_qext == kQextFeature)
        for (int j = 3; j < kCloudSpec; ++j) gout[k++] = s_cloud[j];
    }
    if (m.has_scale) gout[m.idx_scale] = s_scal[0] * m.r_p;
    if (m.has_offset) {
      double o = 0.0;
      for (int k = 0; k < m.K; ++k)
        if (mask && mask[k]) o += w.dm[(size_t)b * m.K + k];
      gout[m.idx_offset] = o * 1.0e-6;
    }
  }
}

// ============================================================================
// sum of the reverse kernel's per-chunk partials into chunk 0 of each sample
// (path-matrix adjoint, annulus-area adjoint and, in FP64, the layer sums), so
// the chain reads one slot; one thread per (sample, element)
template <typename PbarT>
__global__ __launch_bounds__(kBlock) void k_reduce_chunks(Model m, Work w, AdjWork aw, int B, int C) {
  const int Lp = m.L_pad, NS = n_sums(m.S);
  const long n_p = (long)Lp * Lp, n_a = Lp, n_s = sizeof(PbarT) == 8 ? (long)Lp * NS : 0;
  const long per = n_p + n_a + n_s;
  const long gid = (long)blockIdx.x * kBlock + threadIdx.x;
  if (gid >= per * B) return;
  const int b = (int)(gid / per);
  if (w.status[b]) return;
  const long e = gid - (long)b * per;
  const size_t p0 = (size_t)b * C;
  if (e < n_p) {
    PbarT* pb = reinterpret_cast<PbarT*>(aw.pbar);
    double v = 0.0;
    for (int c = 0; c < C; ++c) v += (double)pb[(p0 + c) * n_p + e];
    pb[p0 * n_p + e] = (PbarT)v;
  } else if (e < n_p + n_a) {
    const long i = e - n_p;
    double v = 0.0;
    for (int c = 0; c < C; ++c) v += aw.abar[(p0 + c) * n_a + i];
    aw.abar[p0 * n_a + i] = v;
  } else {
    const long i = e - n_p - n_a;
    double v = 0.0;
    for (int c = 0; c < C; ++c) v += aw.layer_sums[(p0 + c) * (size_t)Lp * NS + i];
    aw.layer_sums[p0 * (size_t)Lp * NS + i] = v;
  }
}

// ============================================================================
// host side
// reduced-precision reverse kernel shapes: (tile, row blocks)
static int adj_tile(int variant) { return variant == kAdjT128M4 ? 128 : 64; }
// FP64 reverse kernel: instance 0 (64-wavenumber tiles) up to 128 padded layers, 1 (32) up to 160
static int adj_fp64_instance(const Model& m) { return m.L_pad <= 128 ? 0 : 1; }
static int adj_tile64(const Model& m) { return adj_fp64_instance(m) == 0 ? 64 : 32; }
static int adj_mb(int variant) { return variant == kAdjT64M5 ? 5 : 4; }
// row-block parts per column block: the 64-wavenumber shapes run eight waves, two per
// SIMD, each with a quarter of the row blocks
static int adj_parts(int variant) { return variant == kAdjT128M4 ? 2 : 4; }
static int adj_threads(int variant) { return 64 * adj_parts(variant) * (adj_tile(variant) / 32); }
static int adj_slots(int variant) {
  return adj_parts(variant) == 2 ? (adj_mb(variant) + 1) / 2 : (adj_mb(variant) <= 4 ? 1 : 2);
}

int adjoint_chunks(const Model& m, const AdjWork& aw, int B, bool fp64) {
  if (m.mode == kEmission) return 1;   // the emission reverse pass keeps no per-chunk partials
  // the FP64 reverse kernel walks 64-wavenumber tiles
  const int tiles = m.n_nu_pad / (fp64 ? adj_tile64(m) : adj_tile(aw.variant));
  const int target = fp64 ? 1024 : aw.chunk_target;
  int c = (target + B - 1) / B;
  return c < 1 ? 1 : (c > tiles ? tiles : c);
}

bool adjoint_supported(const Model& m, bool fp64) {
  if (m.ck) return false;   // the correlated-k path is a forward model only
  return m.L_pad <= 160;
}

// A ragged context of more than kShortLayers padded layers with a 4-row-block shape (128 x 4
// or 64 x 4) runs its samples in two layer-count classes: that shape for those of at most
// kShortLayers layers, 64 x 5 for the rest.  Both launches split every sample into the
// same number of wavenumber chunks (bounded by the wider shape's tile count), so the
// per-chunk partials and their reduction are those of a single launch.
static bool adj_split(const Model& m, int variant) {
  return layer_classes_used(m) && (variant == kAdjT64M4 || variant == kAdjT128M4);
}

int adjoint_default_variant(const Model& m) { return m.L_pad <= 128 ? kAdjT128M4 : kAdjT64M4; }

bool adjoint_variant_fits(const Model& m, int variant) {
  const bool split = adj_split(m, variant);
  if (m.L_pad > 32 * adj_mb(split ? kAdjT64M5 : variant)) return false;
  // the greedy row-block split must never give a wave more blocks than it has slots
  for (int L = 1; L <= m.L_max; ++L) {
    const int KBe = (L + 15) >> 4, MBe = (L + 31) >> 5;
    const int v = split && L > kShortLayers ? (int)kAdjT64M5 : variant;
    for (int part = 0; part < adj_parts(v); ++part)
      for (int rev = 0; rev < 2; ++rev)
        if (__builtin_popcount(split_blocks(part, adj_parts(v), MBe, KBe, rev != 0)) > adj_slots(v)) return false;
  }
  return true;
}

bool adjoint_alloc(AdjWork& aw, const Model& m, int B_max, bool fp64, const std::function<void*(size_t)>& alloc) {
  aw = AdjWork{};
  if (!adjoint_supported(m, fp64)) return true;
  // chunk counts of the narrowest tile and the largest target bound those of every
  // launch choice the context may switch to
  aw.variant = fp64 ? kAdjT128M4 : (adjoint_variant_fits(m, kAdjT64M4) ? kAdjT64M4 : kAdjT64M5);
  aw.chunk_target = kChunkTargets[sizeof(kChunkTargets) / sizeof(int) - 1];
  int pairs = 0;
  for (int B = 1; B <= B_max; ++B) pairs = std::max(pairs, B * adjoint_chunks(m, aw, B, fp64));
  aw.variant = adjoint_default_variant(m);
  aw.chunk_target = 1024;
  aw.ls_tiles = 8;
  aw.max_pairs = pairs;
  const size_t Lp = m.L_pad;
  if (m.mode == kEmission && fp64) {
    aw.lsum_stride = (m.n_tiles + kLsTileChoices[0] - 1) / kLsTileChoices[0];
    aw.lsum_chunks = (m.n_tiles + aw.ls_tiles - 1) / aw.ls_tiles;
    aw.dtb64 = (double*)alloc((size_t)B_max * m.L_pad * m.n_nu_pad * sizeof(double));
    aw.dtau64 = (double*)alloc((size_t)B_max * m.L_pad * m.n_nu_pad * sizeof(double));
    aw.lsum64 = (double*)alloc((size_t)B_max * aw.lsum_stride * Lp * n_lsums(m) * sizeof(double));
    aw.psum64 = (double*)alloc((size_t)B_max * m.n_tiles64 * (Lp + 1) * sizeof(double));
    return aw.dtb64 && aw.dtau64 && aw.lsum64 && aw.psum64;
  }
  if (m.mode == kEmission) {
    aw.lsum_stride = (m.n_tiles + kLsTileChoices[0] - 1) / kLsTileChoices[0];
    aw.lsum_chunks = (m.n_tiles + aw.ls_tiles - 1) / aw.ls_tiles;
    aw.dtb = (float*)alloc((size_t)B_max * m.L_pad * m.n_nu_pad * sizeof(float));
    aw.dtau = (float*)alloc((size_t)B_max * m.L_pad * m.n_nu_pad * sizeof(float));
    aw.lsum = (float*)alloc((size_t)B_max * aw.lsum_stride * Lp * n_lsums(m) * sizeof(float));
    aw.psum = (float*)alloc((size_t)B_max * m.n_tiles64 * (Lp + 1) * sizeof(float));
    return aw.dtb && aw.dtau && aw.lsum && aw.psum;
  }
  aw.pbar = alloc((size_t)pairs * Lp * Lp * (fp64 ? sizeof(double) : sizeof(float)));
  aw.abar = (double*)alloc((size_t)pairs * Lp * sizeof(double));
  if (!aw.pbar || !aw.abar) return false;
  if (fp64) {
    aw.layer_sums = (double*)alloc((size_t)pairs * Lp * n_sums(m.S) * sizeof(double));
    if (m.cloud_ng) aw.hq64 = (double*)alloc((size_t)pairs * kCloudSpec * sizeof(double));
    return aw.layer_sums != nullptr && (!m.cloud_ng || aw.hq64 != nullptr);
  }
  aw.lsum_stride = (m.n_tiles + kLsTileChoices[0] - 1) / kLsTileChoices[0];   // bound over the choices
  aw.lsum_chunks = (m.n_tiles + aw.ls_tiles - 1) / aw.ls_tiles;
  aw.dtb = (float*)alloc((size_t)B_max * m.L_pad * m.n_nu_pad * sizeof(float));
  aw.dtau = (float*)alloc((size_t)B_max * m.L_pad * m.n_nu_pad * sizeof(float));
  aw.lsum = (float*)alloc((size_t)B_max * aw.lsum_stride * Lp * n_lsums(m) * sizeof(float));
  if (m.cloud_ng) {
    aw.hq = (float*)alloc((size_t)B_max * aw.lsum_stride * kCloudSpec * sizeof(float));
    if (!aw.hq) return false;
  }
  return aw.dtb && aw.dtau && aw.lsum;
}

static size_t adj_lds_bytes(const Model& m, bool fp64, int variant) {
  const size_t Lp = m.L_pad, ns = n_sums(m.S);
  if (fp64) return (size_t)2 * adj_tile64(m) * (Lp + 1) * 8 + Lp * ns * 8;
  const size_t tile = adj_tile(variant), rows = std::min(Lp, (size_t)32 * adj_mb(variant));
  return std::max(2 * tile * (32 * adj_mb(variant) + 4) * 4 + rows * 4, tile / 32 * Lp * 8);
}

template <int S, bool CIA>
const void* adj_mixed_kernel(int variant) {
  switch (variant) {
    case kAdjT128M4: return (const void*)k_trans_adj_mixed<S, CIA, 128, 4, 2>;
    case kAdjT64M4: return (const void*)k_trans_adj_mixed<S, CIA, 64, 4, 4>;
    case kAdjT64M5: return (const void*)k_trans_adj_mixed<S, CIA, 64, 5, 4>;
  }
  return nullptr;
}

template <bool F64, int S, bool CIA>
const void* adj_kernel(int variant) {
  if constexpr (F64)
    return variant == 0 ? (const void*)k_trans_adj_fp64<S, CIA, 64, 16, 5> : (const void*)k_trans_adj_fp64<S, CIA, 32, 20, 7>;
  else return adj_mixed_kernel<S, CIA>(variant);
}

template <bool F64>
const void* adj_kernel_for(int S, bool cia, int variant) {
#define EXOFWD_CASE(n) \
  case n: return cia ? adj_kernel<F64, n, true>(variant) : adj_kernel<F64, n, false>(variant);
  switch (S) {
    EXOFWD_CASE(1) EXOFWD_CASE(2) EXOFWD_CASE(3) EXOFWD_CASE(4)
    EXOFWD_CASE(5) EXOFWD_CASE(6) EXOFWD_CASE(7) EXOFWD_CASE(8)
  }
#undef EXOFWD_CASE
  return nullptr;
}

const void* ls_kernel_for(int S, bool cia, bool ng) {
#define EXOFWD_CASE(n) \
  case n:                                                                                          \
    return ng ? (cia ? (const void*)k_layer_sums_mixed<n, true, true> : (const void*)k_layer_sums_mixed<n, false, true>) \
              : (cia ? (const void*)k_layer_sums_mixed<n, true, false> : (const void*)k_layer_sums_mixed<n, false, false>);
  switch (S) {
    EXOFWD_CASE(1) EXOFWD_CASE(2) EXOFWD_CASE(3) EXOFWD_CASE(4)
    EXOFWD_CASE(5) EXOFWD_CASE(6) EXOFWD_CASE(7) EXOFWD_CASE(8)
  }
#undef EXOFWD_CASE
  return nullptr;
}

hipError_t adjoint_configure(const Model& m, bool fp64) {
  if (!adjoint_supported(m, fp64) || m.mode == kEmission) return hipSuccess;
  if (fp64) {
    const void* k = adj_kernel_for<true>(m.S, m.has_cia, adj_fp64_instance(m));
    const size_t bytes = adj_lds_bytes(m, true, 0);
    if (!k || bytes > 160 * 1024) return hipErrorInvalidValue;
    return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  }
  bool any = false;
  for (int v = 0; v < kAdjVariants; ++v) {
    if (!adjoint_variant_fits(m, v)) continue;
    // a split shape also launches 64 x 5 for the long class
    for (int u : {v, adj_split(m, v) ? (int)kAdjT64M5 : v}) {
      const size_t bytes = adj_lds_bytes(m, false, u);
      if (bytes > 160 * 1024) continue;
      const void* k = adj_kernel_for<false>(m.S, m.has_cia, u);
      if (!k) return hipErrorInvalidValue;
      const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
      if (e != hipSuccess) return e;
      any = true;
    }
  }
  return any ? hipSuccess : hipErrorInvalidValue;
}

bool adjoint_set_tuning(AdjWork& aw, const Model& m, int variant, int chunk_target, int ls_tiles) {
  if (variant < 0 || variant >= kAdjVariants || !adjoint_variant_fits(m, variant) ||
      adj_lds_bytes(m, false, variant) > 160 * 1024)
    return false;
  bool ok_t = false, ok_l = false;
  for (int t : kChunkTargets) ok_t |= t == chunk_target;
  for (int t : kLsTileChoices) ok_l |= t == ls_tiles;
  if (!ok_t || !ok_l) return false;
  aw.variant = variant;
  aw.chunk_target = chunk_target;
  aw.ls_tiles = ls_tiles;
  aw.lsum_chunks = (m.n_tiles + ls_tiles - 1) / ls_tiles;
  return true;
}

void launch_trans_adjoint(const Model& m, const Work& w, const Tables& tb, const AdjWork& aw, int B, bool fp64,
                          hipStream_t st) {
  int C = adjoint_chunks(m, aw, B, fp64);
  if (fp64) {
    void* args[] = {(void*)&m, (void*)&w, (void*)&tb, (void*)&aw, (void*)&B, (void*)&C};
    hipLaunchKernel(adj_kernel_for<true>(m.S, m.has_cia, adj_fp64_instance(m)), dim3((unsigned)(B * C)), dim3(kBlockT),
                    args, adj_lds_bytes(m, true, 0), st);
    return;
  }
  const int32_t* cls = adj_split(m, aw.variant) ? w.cls : nullptr;   // the forward built the classes
  for (int cl = 0; cl < (cls ? 2 : 1); ++cl) {
    const int v = cl == 1 ? (int)kAdjT64M5 : aw.variant;
    void* args[] = {(void*)&m, (void*)&w, (void*)&tb, (void*)&aw, (void*)&B, (void*)&C, (void*)&cls, (void*)&cl};
    hipLaunchKernel(adj_kernel_for<false>(m.S, m.has_cia, v), dim3((unsigned)(B * C)), dim3(adj_threads(v)), args,
                    adj_lds_bytes(m, false, v), st);
  }
}

void launch_layer_sums(const Model& m, const Work& w, const Tables& tb, const AdjWork& aw, int B, bool fp64,
                       hipStream_t st) {
  if (m.mode == kEmission) {
    launch_layer_sums_emis(m, w, tb, aw, B, fp64, st);
    return;
  }
  const int NG = m.L_max;   // layer groups per sample: at most one per layer
  const long waves = (long)aw.lsum_chunks * B * NG;
  void* args2[] = {(void*)&m, (void*)&w, (void*)&tb, (void*)&aw, (void*)&B};
  // a whole number of blocks per XCD; the waves past the last chunk return at once
  const long blocks = ((waves + 3) / 4 + 7) / 8 * 8;
  hipLaunchKernel(ls_kernel_for(m.S, m.has_cia, m.cloud_ng), dim3((unsigned)blocks), dim3(kBlock), args2, 0, st);
  if (m.cloud_ng) {
    const long cw = (long)B * aw.lsum_chunks;
    hipLaunchKernelGGL(k_cloud_spectral, dim3((unsigned)((cw + 3) / 4)), dim3(kBlock), 0, st, m, w, aw, B);
  }
}

void launch_chain(const Model& m, const Work& w, const AdjWork& aw, int B, const double* params, const uint8_t* mask,
                  double* grad, bool fp64, hipStream_t st) {
  const int C = adjoint_chunks(m, aw, B, fp64);
  int Cn = C;
  if (C > 1) {
    // the chunk partials are summed by a wide kernel first; the chain then reads one slot
    const long per = (long)m.L_pad * m.L_pad + m.L_pad + (fp64 ? (long)m.L_pad * n_sums(m.S) : 0);
    const unsigned grid = (unsigned)((per * B + kBlock - 1) / kBlock);
    if (fp64)
      hipLaunchKernelGGL(k_reduce_chunks<double>, dim3(grid), dim3(kBlock), 0, st, m, w, aw, B, C);
    else
      hipLaunchKernelGGL(k_reduce_chunks<float>, dim3(grid), dim3(kBlock), 0, st, m, w, aw, B, C);
    Cn = 1;
  }
  if (fp64)
    hipLaunchKernelGGL(k_chain<double>, dim3(B), dim3(kBlock), 0, st, m, w, aw, C, Cn, params, mask, grad);
  else
    hipLaunchKernelGGL(k_chain<float>, dim3(B), dim3(kBlock), 0, st, m, w, aw, C, Cn, params, mask, grad);
}

}  // namespace exofwd
