// Adjoint of the transmission path: per-(sample, wavenumber chunk) partial
// sums from the fused reverse kernels, and the FP64 chain to d lnL / d params.
#pragma once
#include "common.h"

#include <functional>

namespace exofwd {

// Per-layer sums over wavenumber produced by the reverse kernels, in this order:
//   [0, S)  G_s   = sum_nu dtau_bar_l t_ls           (t_ls: line term of source s)
//   S       HT    = sum_nu dtau_bar_l sum_s t_ls dv_ls/dwT   (log2 units)
//   S+1,2   Gc_p  = sum_nu dtau_bar_l t_lp           (CIA pairs H2-H2, H2-He)
//   S+3     HTc   = sum_nu dtau_bar_l sum_p t_lp dv_lp/dwTc
//   S+4     GR    = sum_nu dtau_bar_l (nu/1e4)^4
//   S+5     GD    = sum_nu dtau_bar_l               (non-grey cloud: sum_nu dtau_bar_l Q_ext(nu))
constexpr int kExtraSums = 6;
__host__ __device__ constexpr int n_sums(int s) { return s + kExtraSums; }
__host__ __device__ inline int n_lsums(const Model& m) { return n_sums(m.S); }

// shapes of the reduced-precision reverse kernel: wavenumber tile x 32-row blocks
enum : int { kAdjT128M4 = 0, kAdjT64M4 = 1, kAdjT64M5 = 2, kAdjVariants = 3 };

// launch choices the autotuner may change (every value is valid for any workload)
constexpr int kChunkTargets[] = {512, 1024, 2048, 4096, 8192};   // (sample, chunk) work items per reverse launch
constexpr int kLsTileChoices[] = {4, 8, 16, 32, 64};           // 128-wavenumber tiles per layer-sum wave

struct AdjWork {
  int variant;         // reduced-precision reverse kernel shape (kAdj*)
  int chunk_target;    // the reverse kernel splits each sample's wavenumbers into ~chunk_target / B chunks
  int ls_tiles;        // tiles per wave of the layer-sum kernel
  int max_pairs;       // allocated (sample, chunk) pairs of the fused reverse kernel
  double* layer_sums;  // FP64 path: [pair][L_pad][n_sums]
  void* pbar;          // [pair][L_pad][L_pad] d lnL / d P_il (row i, column l), float (mixed) or double (FP64)
  double* abar;        // [pair][L_pad] d lnL / d area_i
  // reduced-precision path: the fused kernel stores dtau_bar, a second kernel forms the layer sums
  float* dtau;         // [B_max][L_pad][n_nu_pad] layer optical depths stored by the forward kernel:
                       //   transmission as packed bf16 pairs (hi | lo << 16), emission as FP32
  float* dtb;          // [B_max][L_pad][n_nu_pad] d lnL / d dtau_l(nu)
  float* lsum;         // [B_max][lsum_chunks][L_pad][n_lsums] partial layer sums
  float* hq;           // non-grey cloud: [B_max][lsum_stride][kCloudSpec] per-chunk sums over nu of
                       //   (sum_l D_l dtau_bar_l) dQ_ext/dp_k
  float* psum;         // emission: [B_max][n_tiles64][L_pad+1] per-tile sums over nu of d lnL/dB_j dB_j/dT_j
  // FP64 emission: the same buffers in double (dtau, dtau_bar, per-level and per-layer sums)
  double* dtau64;
  double* dtb64;
  double* psum64;
  double* lsum64;      // [B_max][lsum_chunks][L_pad][n_sums]
  double* hq64;        // FP64 transmission, non-grey cloud: [pair][kCloudSpec] the sums of hq
  int lsum_chunks;     // wavenumber chunks of the layer-sum kernel (n_tiles / ls_tiles, rounded up)
  int lsum_stride;     // allocated chunks per sample (the bound over the ls_tiles choices)
};

// wavenumber chunks per sample for a batch of B (pair index = b * chunks + chunk)
int adjoint_chunks(const Model& m, const AdjWork& aw, int B, bool fp64);
bool adjoint_alloc(AdjWork& aw, const Model& m, int B_max, bool fp64, const std::function<void*(size_t)>& alloc);
hipError_t adjoint_configure(const Model& m, bool fp64);
void launch_trans_adjoint(const Model& m, const Work& w, const Tables& tb, const AdjWork& aw, int B, bool fp64,
                          hipStream_t st);
// per-layer sums from the stored dtau_bar (reduced-precision transmission, emission in both precisions)
void launch_layer_sums(const Model& m, const Work& w, const Tables& tb, const AdjWork& aw, int B, bool fp64,
                       hipStream_t st);
void launch_chain(const Model& m, const Work& w, const AdjWork& aw, int B, const double* params, const uint8_t* mask,
                  double* grad, bool fp64, hipStream_t st);
// whether the adjoint supports this workload: transmission with L_pad <= 160 in
// reduced precision, <= 128 and no non-grey cloud in FP64; emission with L_pad <= 160
// in reduced precision, <= 128 in FP64
void launch_emis_adjoint(const Model& m, const Work& w, const AdjWork& aw, int B, bool fp64, hipStream_t st);
void launch_layer_sums_emis(const Model& m, const Work& w, const Tables& tb, const AdjWork& aw, int B, bool fp64,
                            hipStream_t st);
bool adjoint_supported(const Model& m, bool fp64);
// default reverse-kernel shape, whether a shape serves this model, and switching shapes
int adjoint_default_variant(const Model& m);
bool adjoint_variant_fits(const Model& m, int variant);
// switch the reduced-precision launch choices (reverse shape, chunk target, layer-sum
// tiles); false, with nothing changed, if a choice does not serve this model
bool adjoint_set_tuning(AdjWork& aw, const Model& m, int variant, int chunk_target, int ls_tiles);

}  // namespace exofwd
