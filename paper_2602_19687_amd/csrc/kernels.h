// Launch entry points of the gfx950 kernels (host side of each .hip file).
#pragma once
#include "common.h"

namespace exofwd {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

// block id -> logical id such that consecutive logical ids share an XCD
// (the dispatcher deals workgroups round-robin over the 8 XCDs)
__device__ inline int xcd_logical_block(int bid, int nblk) {
  if ((nblk & 7) != 0) return bid;
  return (bid & 7) * (nblk >> 3) + (bid >> 3);
}

// Position in a layer-count class's sample list of sample slot s of a launch whose
// logical blocks (xcd_logical_block over n_slots * per_slot blocks) give each XCD a
// contiguous run of n_slots / 8 slots: the positions are dealt round the XCDs
// (slot s of XCD k holds position 8 (s - k n_slots / 8) + k), so a class that fills
// only part of the grid still spreads over every XCD, longest samples first on each.
__device__ inline int class_position(int s, int n_slots, int per_slot) {
  if ((n_slots & 7) != 0 || (((long)n_slots * per_slot) & 7) != 0) return s;
  const int spx = n_slots >> 3;
  return (s % spx) * 8 + s / spx;
}

void launch_profile(const Model& m, const Work& w, int B, const double* params, const int32_t* n_layers,
                    bool fp64, hipStream_t st);
// dtau_out (reduced precision only, may be null): layer optical depths [B][L_pad][n_nu_pad] for the reverse pass
void launch_trans_fwd(const Model& m, const Work& w, const Tables& tb, int B, void* spec, bool fp64,
                      hipStream_t st, float* dtau_out = nullptr);
// B real samples; with the cloudy/clear mixing spec holds the 2B virtual spectra and the
// mixed spectrum goes to spec_out (may be null)
void launch_loglike(const Model& m, const Work& w, int B, const double* params, const void* spec, void* spec_out,
                    bool spec_f64, const int32_t* bin_lo, const int32_t* bin_hi, const double* y, const double* yerr,
                    const uint8_t* mask, double* lnl, int32_t* status_out, hipStream_t st);
// cloudy/clear mixing: grad[b] = gv[2b] + gv[2b+1], with d lnL / d f_cld from the likelihood kernel
void launch_mix_grad(const Model& m, const Work& w, int B, double* grad, hipStream_t st);
size_t trans_fwd_lds_bytes(const Model& m, bool fp64);
// Layer-count classes of a reduced-precision transmission call whose padded layer count
// exceeds kShortLayers: w.cls = [count0, count1, samples of class 0 (at most kShortLayers
// layers, and invalid ones) longest first, then class 1 longest first, each list B long]
inline bool layer_classes_used(const Model& m) { return m.mode == kTransmission && !m.ck && m.L_pad > kShortLayers; }
void launch_layer_classes(const Model& m, const Work& w, int B, hipStream_t st);
hipError_t trans_fwd_configure(const Model& m, bool fp64);

}  // namespace exofwd
