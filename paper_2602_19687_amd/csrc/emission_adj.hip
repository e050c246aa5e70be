// Adjoint of the reduced-precision emission path (Eq. 45 with the
// linear-in-tau sweep): d lnL / d dtau_l(nu) for every layer and wavenumber,
// the per-level sums over wavenumber of d lnL / d B_j times dB/dT_j, and the
// per-layer opacity sums of the FP32 tables.  The chain kernel of the
// transmission adjoint then carries both to the parameters.
//
// One wave per (sample, 64-wavenumber tile), one wavenumber per lane.  The
// sweep is linear in the intensity: through a slab of optical depth x = dtau/mu,
//   I' = I e + B_t om + (B_b - B_t) src,   e = e^-x, om = 1 - e^-x,
// so the adjoint of the intensity leaving layer l upward is the top seed times the
// transmission exp(-X_l / mu) of everything above it (X_l = sum of dtau over the
// layers above l).  A first pass walks down the column storing X_l (one float per
// layer, the same for every angle) in the dtau_bar buffer; the second walks up
// with the forward recurrence, which is stable, and overwrites each X_l with
// dtau_bar_l.  Walking the intensity back down instead would divide by e^-x and
// lose all precision under thick layers.
#include "adjoint.h"
#include "emission.h"
#include "kernels.h"
#include "opacity.h"

namespace exofwd {

__device__ inline float wave_sum_f(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// d src / dx of src = (1 - e^-x)/x - e^-x (series below x = 0.1 as in slab_terms)
__device__ inline float slab_dsrc(float x, float e, float om) {
  if (x < 0.1f)
    return 0.5f + x * (-2.0f / 3.0f + x * (0.375f + x * (-2.0f / 15.0f + x * (5.0f / 144.0f + x * (-1.0f / 140.0f)))));
  const float r = __builtin_amdgcn_rcpf(x);
  return e * (1.0f + r) - om * r * r;
}

__global__ __launch_bounds__(kBlock) void k_emis_adj_mixed(Model m, Work w, AdjWork aw, int B) {
  const int logical = xcd_logical_block(blockIdx.x, gridDim.x);
  const int b = logical % B;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tile = (logical / B) * 4 + wv;
  if (tile >= m.n_tiles64 || w.status[b]) return;
  const int nu = tile * kTile64 + lane;
  const int L = w.nlay[b], Lp = m.L_pad;
  const size_t npad = (size_t)m.n_nu_pad;
  const float* dt = aw.dtau + (size_t)b * Lp * npad + nu;
  float* dtb = aw.dtb + (size_t)b * Lp * npad + nu;
  float* ps = aw.psum + ((size_t)b * m.n_tiles64 + tile) * (Lp + 1);
  const double* t_lev = w.t_lev + (size_t)b * (Lp + 1);
  const double* inv_t = w.inv_tlev + (size_t)b * (Lp + 1);

  // seed: d lnL / d spectrum(nu) = dm_k / n_k for the bin holding nu, times the
  // flux-to-ratio factor s (R/R_s)^2 / (pi B_*) and each angle's 2 pi w mu
  const int kb = w.bin_of[nu];
  float seed = 0.0f;
  if (kb >= 0) {
    const double nd = m.nu[nu];
    const double fstar =
        m.has_bd ? 1.0 : M_PI * 2.0 * kHpl * kC * kC * nd * nd * nd / expm1(kHpl * kC * nd / (kB * m.t_star));
    seed = (float)(w.dm[(size_t)b * m.K + kb] * w.inv_cnt[kb] * m.dilution * w.core[b] / fstar);
  }
  const double nud = m.nu[nu];
  const float c1n3 = (float)(2.0 * kHpl * kC * kC * nud * nud * nud);
  const double c2n_log2e = kHpl * kC / kB * 1.4426950408889634074 * nud;
  // Planck intensity at level j (as the forward kernel forms it) and its temperature
  // derivative B y e^y / ((e^y - 1) T)
  auto planck_at = [&](int j, float& dbdt) {
    const float t = (float)t_lev[j];
    float y, em1;
    const float bv = planck_split(c1n3, c2n_log2e, inv_t[j], y, em1);
    dbdt = bv * y * (em1 + 1.0f) * __builtin_amdgcn_rcpf(em1 * t);
    return bv;
  };
  const int n_mu = m.n_mu;
  float inv_mu[kMaxMu], inten[kMaxMu], ibar_top[kMaxMu];
  // pass 1: optical depth above each layer, top down
  float above = 0.0f;
  for (int l = L - 1; l >= 0; --l) {
    dtb[(size_t)l * npad] = above;
    above += dt[(size_t)l * npad];
  }
  float dbdt_bot;
  float b_bot = planck_at(0, dbdt_bot);
#pragma unroll
  for (int k = 0; k < kMaxMu; ++k) {
    inv_mu[k] = k < n_mu ? (float)(1.0 / m.mu_nodes[k]) : 0.0f;
    ibar_top[k] = k < n_mu ? seed * (float)(2.0 * M_PI * m.mu_weights[k] * m.mu_nodes[k]) : 0.0f;
    inten[k] = b_bot;
  }
  // the bottom boundary intensity is B_0, seen through the whole column
  float bb_lev = 0.0f;
#pragma unroll
  for (int k = 0; k < kMaxMu; ++k)
    if (k < n_mu) bb_lev = fmaf(ibar_top[k], exp2_fast(-1.4426950408889634f * above * inv_mu[k]), bb_lev);
  // pass 2: up the column; bb_lev collects d lnL / d B at the current bottom level
  for (int l = 0; l < L; ++l) {
    const float d = dt[(size_t)l * npad];
    const float x_above = dtb[(size_t)l * npad];
    float dbdt_top;
    const float b_top = planck_at(l + 1, dbdt_top);
    const float db = b_bot - b_top;
    float dsum = 0.0f, bt_bar = 0.0f;
#pragma unroll
    for (int k = 0; k < kMaxMu; ++k) {
      if (k >= n_mu) break;
      const float x = d * inv_mu[k];
      const float e = exp2_fast(-1.4426950408889634f * x);
      float om, src;
      slab_terms(x, e, om, src);
      // adjoint of the intensity leaving the layer: seed x transmission above it
      const float ib = ibar_top[k] * exp2_fast(-1.4426950408889634f * x_above * inv_mu[k]);
      dsum = fmaf(ib * fmaf(b_top - inten[k], e, db * slab_dsrc(x, e, om)), inv_mu[k], dsum);
      bt_bar = fmaf(ib, om - src, bt_bar);
      bb_lev = fmaf(ib, src, bb_lev);
      inten[k] = fmaf(om, b_top - inten[k], fmaf(db, src, inten[k]));
    }
    __builtin_nontemporal_store(dsum, &dtb[(size_t)l * npad]);   // read once, by the layer sums
    const float lev = wave_sum_f(bb_lev * dbdt_bot);
    if (lane == 0) ps[l] = lev;
    bb_lev = bt_bar;
    b_bot = b_top;
    dbdt_bot = dbdt_top;
  }
  const float lev_top = wave_sum_f(bb_lev * dbdt_bot);
  if (lane == 0) ps[L] = lev_top;
}

// Per-layer opacity sums of the emission tables (FP32 entries, one
// wavenumber per lane, 64-wavenumber tiles): the same sums, in the same order,
// as the transmission layer sums, with no Rayleigh or cloud term.
template <int S, bool CIA>
__global__ __launch_bounds__(kBlock) void k_layer_sums_emis(Model m, Work w, Tables tb, AdjWork aw, int B) {
  constexpr int NS = n_sums(S);
  constexpr int kLayers = kLsGroup;
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
  // a run of up to kLayers consecutive layers in one table cell: the table entries
  // are fetched once per tile for all of them
  const int32_t* grp = w.lsg + (size_t)b * (Lp + 1);
  if (lg >= grp[0]) return;
  const int l0 = grp[1 + lg] & 0xffff, cnt = grp[1 + lg] >> 16;
  const size_t npad = (size_t)m.n_nu_pad;
  const uint32_t row_bytes = (uint32_t)npad * 4u, tstep = (uint32_t)m.n_p * row_bytes;
  const __amdgpu_buffer_rsrc_t rh = make_rsrc(tb.h, (size_t)S * m.n_t * m.n_p * npad * 4);
  const __amdgpu_buffer_rsrc_t rhc = make_rsrc(CIA ? (const void*)tb.hc : (const void*)tb.h,
                                               CIA ? (size_t)2 * m.n_tc * npad * 4 : 0);
  const uint32_t voff = (uint32_t)lane * 4u;
  constexpr int RL = rec_len(S);
  const float* rec = reinterpret_cast<const float*>(w.rec) + (size_t)b * Lp * RL;
  const float* dtb = aw.dtb + (size_t)b * Lp * npad;
  const int cl = w.cells[(size_t)b * Lp + l0];
  const int it = cl & 255, ip = (cl >> 8) & 255, itc = cl >> 16;

  float acc[kLayers][NS];
#pragma unroll
  for (int q = 0; q < kLayers; ++q)
#pragma unroll
    for (int k = 0; k < NS; ++k) acc[q][k] = 0.0f;

  // the chunk's 128-wavenumber tiles, as 64-wavenumber halves
  const int t0 = 2 * chunk * aw.ls_tiles, t1 = min(t0 + 2 * aw.ls_tiles, m.n_tiles64);
  for (int tile = t0; tile < t1; ++tile) {
    const int nu0 = tile * kTile64, nu = nu0 + lane;
    const uint32_t nu0_bytes = (uint32_t)nu0 * 4u;
    // a layer seen through no transmission at any wavenumber of the tile adds
    // nothing (the skip is per layer: the opaque depth varies across a tile)
    float dbv[kLayers];
#pragma unroll
    for (int q = 0; q < kLayers; ++q)
      dbv[q] = q < cnt ? __builtin_nontemporal_load(&dtb[(size_t)(l0 + q) * npad + nu]) : 0.0f;
    // the table entries are fetched together with dtau_bar (one memory round trip per
    // tile), before the test that skips a tile whose dtau_bar is zero
    float cs[S], ccs[2];
#pragma unroll
    for (int s = 0; s < S; ++s) cs[s] = tb.c[(size_t)s * npad + nu];
#pragma unroll
    for (int p = 0; p < 2; ++p) ccs[p] = CIA ? tb.cc[(size_t)p * npad + nu] : 0.0f;
    float tp[4 * S + 4];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const uint32_t row = (uint32_t)((s * m.n_t + it) * m.n_p + ip) * row_bytes + nu0_bytes;
      tp[4 * s] = load_f32(rh, voff, row);
      tp[4 * s + 1] = load_f32(rh, voff, row + tstep);
      tp[4 * s + 2] = load_f32(rh, voff, row + row_bytes);
      tp[4 * s + 3] = load_f32(rh, voff, row + tstep + row_bytes);
    }
    if (CIA) {
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const uint32_t row = (uint32_t)(p * m.n_tc + itc) * row_bytes + nu0_bytes;
        tp[4 * S + 2 * p] = load_f32(rhc, voff, row);
        tp[4 * S + 2 * p + 1] = load_f32(rhc, voff, row + row_bytes);
      }
    }
    bool live = false;
#pragma unroll
    for (int q = 0; q < kLayers; ++q) live |= dbv[q] != 0.0f;
    if (__builtin_amdgcn_ballot_w64(live) == 0) continue;
#pragma unroll
    for (int q = 0; q < kLayers; ++q) {
      if (q >= cnt) continue;
      const float db = dbv[q];
      if (__builtin_amdgcn_ballot_w64(db != 0.0f) == 0) continue;
      const float* rl = rec + (size_t)(l0 + q) * RL;
      const float wt = rl[0], wp = rl[1], omp = 1.0f - wp;
      float z = 0.0f;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const float p00 = tp[4 * s], p10 = tp[4 * s + 1], p01 = tp[4 * s + 2], p11 = tp[4 * s + 3];
        const float base = cs[s] + rl[kRecFixed + s];
        const float u0 = fmaf(omp, p00, fmaf(wp, p01, base));
        const float u1 = fmaf(omp, p10, fmaf(wp, p11, base));
        const float dw = u1 - u0;
        const float t = exp2_fast(fmaf(wt, dw, u0));
        acc[q][s] = fmaf(db, t, acc[q][s]);
        z = fmaf(t, dw, z);
      }
      acc[q][S] = fmaf(db, z, acc[q][S]);
      if (CIA) {
        const float wtc = rl[2];
        float y = 0.0f;
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          const float a = tp[4 * S + 2 * p], c2 = tp[4 * S + 2 * p + 1];
          const float va = a + (ccs[p] + rl[5 + p]);
          const float dw = c2 - a;
          const float t = exp2_fast(fmaf(wtc, dw, va));
          acc[q][S + 1 + p] = fmaf(db, t, acc[q][S + 1 + p]);
          y = fmaf(t, dw, y);
        }
        acc[q][S + 3] = fmaf(db, y, acc[q][S + 3]);
      }
    }
  }
  float* out = aw.lsum + ((size_t)b * aw.lsum_stride + chunk) * Lp * NS;
#pragma unroll
  for (int q = 0; q < kLayers; ++q) {
    if (q >= cnt) continue;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const float tot = wave_sum_f(acc[q][k]);
      if (lane == 0) out[(size_t)(l0 + q) * NS + k] = tot;
    }
  }
}

// ============================================================================
// plain FP64 emission adjoint: the same two passes and sums in double, from the
// FP64 forward's stored layer optical depths and the FP64 log10 sigma tables
__global__ __launch_bounds__(kBlock) void k_emis_adj_fp64(Model m, Work w, AdjWork aw, int B) {
  const int logical = xcd_logical_block(blockIdx.x, gridDim.x);
  const int b = logical % B;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tile = (logical / B) * 4 + wv;
  if (tile >= m.n_tiles64 || w.status[b]) return;
  const int nu = tile * kTile64 + lane;
  const int L = w.nlay[b], Lp = m.L_pad;
  const size_t npad = (size_t)m.n_nu_pad;
  const double* dt = aw.dtau64 + (size_t)b * Lp * npad + nu;
  double* dtb = aw.dtb64 + (size_t)b * Lp * npad + nu;
  double* ps = aw.psum64 + ((size_t)b * m.n_tiles64 + tile) * (Lp + 1);
  const double* t_lev = w.t_lev + (size_t)b * (Lp + 1);
  const int kb = w.bin_of[nu];
  const double nd = m.nu[nu];
  double seed = 0.0;
  if (kb >= 0) {
    const double fstar =
        m.has_bd ? 1.0 : M_PI * 2.0 * kHpl * kC * kC * nd * nd * nd / expm1(kHpl * kC * nd / (kB * m.t_star));
    seed = w.dm[(size_t)b * m.K + kb] * w.inv_cnt[kb] * m.dilution * w.core[b] / fstar;
  }
  const double c1n3 = 2.0 * kHpl * kC * kC * nd * nd * nd, c2n = kHpl * kC / kB * nd;
  auto planck_at = [&](int j, double& dbdt) {
    const double t = t_lev[j], y = c2n / t, em1 = expm1(y);
    const double bv = c1n3 / em1;
    dbdt = bv * y * (em1 + 1.0) / (em1 * t);
    return bv;
  };
  // 1 - e^-x, (1 - e^-x)/x - e^-x and its derivative, by series for thin slabs
  auto slab = [](double x, double& e, double& om, double& src, double& dsrc) {
    e = exp(-x);
    om = -expm1(-x);
    if (x < 1.0e-4) src = x * (0.5 + x * (-1.0 / 3.0 + x * (0.125 + x * (-1.0 / 30.0))));
    else src = om / x - e;
    if (x < 1.0e-3) dsrc = 0.5 + x * (-2.0 / 3.0 + x * (0.375 + x * (-2.0 / 15.0 + x * (5.0 / 144.0))));
    else dsrc = e * (1.0 + 1.0 / x) - om / (x * x);
  };
  const int n_mu = m.n_mu;
  double inv_mu[kMaxMu], inten[kMaxMu], ibar_top[kMaxMu];
  double above = 0.0;
  for (int l = L - 1; l >= 0; --l) {
    dtb[(size_t)l * npad] = above;
    above += dt[(size_t)l * npad];
  }
  double dbdt_bot;
  double b_bot = planck_at(0, dbdt_bot);
  for (int k = 0; k < kMaxMu; ++k) {
    inv_mu[k] = k < n_mu ? 1.0 / m.mu_nodes[k] : 0.0;
    ibar_top[k] = k < n_mu ? seed * 2.0 * M_PI * m.mu_weights[k] * m.mu_nodes[k] : 0.0;
    inten[k] = b_bot;
  }
  double bb_lev = 0.0;
  for (int k = 0; k < n_mu; ++k) bb_lev += ibar_top[k] * exp(-above * inv_mu[k]);
  for (int l = 0; l < L; ++l) {
    const double d = dt[(size_t)l * npad];
    const double x_above = dtb[(size_t)l * npad];
    double dbdt_top;
    const double b_top = planck_at(l + 1, dbdt_top);
    const double db = b_bot - b_top;
    double dsum = 0.0, bt_bar = 0.0;
    for (int k = 0; k < n_mu; ++k) {
      double e, om, src, dsrc;
      slab(d * inv_mu[k], e, om, src, dsrc);
      const double ib = ibar_top[k] * exp(-x_above * inv_mu[k]);
      dsum += ib * ((b_top - inten[k]) * e + db * dsrc) * inv_mu[k];
      bt_bar += ib * (om - src);
      bb_lev += ib * src;
      inten[k] += om * (b_top - inten[k]) + db * src;
    }
    dtb[(size_t)l * npad] = dsum;
    double lev = bb_lev * dbdt_bot;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) lev += __shfl_xor(lev, off);
    if (lane == 0) ps[l] = lev;
    bb_lev = bt_bar;
    b_bot = b_top;
    dbdt_bot = dbdt_top;
  }
  double lev = bb_lev * dbdt_bot;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) lev += __shfl_xor(lev, off);
  if (lane == 0) ps[L] = lev;
}

// FP64 per-layer opacity sums of the emission path (log10 sigma tables, one
// wavenumber per lane, layers whose dtau_bar is zero across the tile skipped)
__global__ __launch_bounds__(kBlock) void k_layer_sums_emis_fp64(Model m, Work w, Tables tb, AdjWork aw, int B) {
  constexpr int kLayers = 5;
  const int S = m.S, NS = n_sums(S);
  const int lane = threadIdx.x & 63;
  const int gw = blockIdx.x * (kBlock / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int NG = (m.L_max + kLayers - 1) / kLayers;
  const int per_chunk = B * NG;
  const int chunk = gw / per_chunk;
  if (chunk >= aw.lsum_chunks) return;
  const int rem = gw - chunk * per_chunk;
  const int b = rem / NG, lg = rem - b * NG;
  if (w.status[b]) return;
  const int L = w.nlay[b];
  const int l0 = lg * kLayers;
  if (l0 >= L) return;
  const int Lp = m.L_pad, RL = rec_len(S);
  const size_t npad = (size_t)m.n_nu_pad;
  const double* rec = reinterpret_cast<const double*>(w.rec) + (size_t)b * Lp * RL;
  const int32_t* cells = w.cells + (size_t)b * Lp;
  const double* dtb = aw.dtb64 + (size_t)b * Lp * npad;
  double acc[kLayers][kMaxSpecies + kExtraSums];
  for (int q = 0; q < kLayers; ++q)
    for (int k = 0; k < NS; ++k) acc[q][k] = 0.0;
  const int t0 = 2 * chunk * aw.ls_tiles, t1 = min(t0 + 2 * aw.ls_tiles, m.n_tiles64);
  for (int tile = t0; tile < t1; ++tile) {
    const int nu = tile * kTile64 + lane;
    for (int q = 0; q < kLayers; ++q) {
      const int l = l0 + q;
      if (l >= L) continue;
      const double db = dtb[(size_t)l * npad + nu];
      if (__builtin_amdgcn_ballot_w64(db != 0.0) == 0) continue;
      const int cl = cells[l];
      const int it = cl & 255, ip = (cl >> 8) & 255, itc = cl >> 16;
      const double* rl = rec + (size_t)l * RL;
      const double wt = rl[0], wp = rl[1];
      double z = 0.0;
      for (int s2 = 0; s2 < S; ++s2) {
        const double* p = tb.t64 + (((size_t)s2 * m.n_t + it) * m.n_p + ip) * npad + nu;
        const double t00 = p[0], t10 = p[(size_t)m.n_p * npad], t01 = p[npad], t11 = p[(size_t)(m.n_p + 1) * npad];
        const double v = (1.0 - wt) * (1.0 - wp) * t00 + wt * (1.0 - wp) * t10 + (1.0 - wt) * wp * t01 + wt * wp * t11;
        const double t = exp2(v * kLog2_10 + rl[kRecFixed + s2]);
        const double dw = ((1.0 - wp) * (t10 - t00) + wp * (t11 - t01)) * kLog2_10;   // log2 units
        acc[q][s2] += db * t;
        z += t * dw;
      }
      acc[q][S] += db * z;
      if (m.has_cia) {
        const double wtc = rl[2];
        double y = 0.0;
        for (int c = 0; c < 2; ++c) {
          const double* p = tb.tc64 + ((size_t)c * m.n_tc + itc) * npad + nu;
          const double t = exp2(((1.0 - wtc) * p[0] + wtc * p[npad]) * kLog2_10 + rl[5 + c]);
          acc[q][S + 1 + c] += db * t;
          y += t * (p[npad] - p[0]) * kLog2_10;
        }
        acc[q][S + 3] += db * y;
      }
    }
  }
  double* out = aw.lsum64 + ((size_t)b * aw.lsum_stride + chunk) * Lp * NS;
  for (int q = 0; q < kLayers; ++q) {
    const int l = l0 + q;
    if (l >= L) continue;
    for (int k = 0; k < NS; ++k) {
      double v = acc[q][k];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
      if (lane == 0) out[(size_t)l * NS + k] = v;
    }
  }
}

const void* ls_emis_kernel_for(int S, bool cia) {
#define EXOFWD_CASE(n) \
  case n: return cia ? (const void*)k_layer_sums_emis<n, true> : (const void*)k_layer_sums_emis<n, false>;
  switch (S) {
    EXOFWD_CASE(1) EXOFWD_CASE(2) EXOFWD_CASE(3) EXOFWD_CASE(4)
    EXOFWD_CASE(5) EXOFWD_CASE(6) EXOFWD_CASE(7) EXOFWD_CASE(8)
  }
#undef EXOFWD_CASE
  return nullptr;
}

void launch_emis_adjoint(const Model& m, const Work& w, const AdjWork& aw, int B, bool fp64, hipStream_t st) {
  // four 64-wavenumber tiles (one per wave) of one sample per workgroup
  const dim3 grid((unsigned)((m.n_tiles64 + 3) / 4 * B));
  if (fp64) hipLaunchKernelGGL(k_emis_adj_fp64, grid, dim3(kBlock), 0, st, m, w, aw, B);
  else hipLaunchKernelGGL(k_emis_adj_mixed, grid, dim3(kBlock), 0, st, m, w, aw, B);
}

void launch_layer_sums_emis(const Model& m, const Work& w, const Tables& tb, const AdjWork& aw, int B, bool fp64,
                            hipStream_t st) {
  // FP64: fixed groups of 5 layers; reduced precision: one wave per (chunk, sample, layer group)
  const long waves = (long)aw.lsum_chunks * B * (fp64 ? (m.L_max + 4) / 5 : m.L_max);
  // a whole number of blocks per XCD; the waves past the last chunk return at once
  const dim3 grid((unsigned)(((waves + 3) / 4 + 7) / 8 * 8));
  if (fp64) {
    hipLaunchKernelGGL(k_layer_sums_emis_fp64, grid, dim3(kBlock), 0, st, m, w, tb, aw, B);
    return;
  }
  void* args[] = {(void*)&m, (void*)&w, (void*)&tb, (void*)&aw, (void*)&B};
  hipLaunchKernel(ls_emis_kernel_for(m.S, m.has_cia), grid, dim3(kBlock), args, 0, st);
}

}  // namespace exofwd
