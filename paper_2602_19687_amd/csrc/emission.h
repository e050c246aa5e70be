#pragma once
#include "common.h"

namespace exofwd {
// dtau_out (may be null): layer optical depths [B][L_pad][n_nu_pad] for the reverse pass, float in reduced
// precision, double in FP64
void launch_emission(const Model& m, const Work& w, const Tables& tb, int B, void* spec, bool fp64, hipStream_t st,
                     void* dtau_out = nullptr);
hipError_t emission_configure(const Model& m, bool fp64);
size_t emission_lds_bytes(const Model& m, bool fp64);

// Planck intensity per unit wavenumber at temperature t, 2 h c^2 nu^3 / (exp(y) - 1)
// with y = h c nu / k t, from c1n3 = 2 h c^2 nu^3 and c2n = h c nu / k; below
// y = 0.01, exp(y) - 1 is taken from its series.  em1 returns exp(y) - 1.
__device__ inline float planck_f32(float c1n3, float c2n, float t, float& y, float& em1) {
  y = c2n * __builtin_amdgcn_rcpf(t);
  em1 = y < 0.01f ? y * (1.0f + y * (0.5f + y * (1.0f / 6.0f)))
                  : __builtin_amdgcn_exp2f(1.4426950408889634f * y) - 1.0f;
  return c1n3 * __builtin_amdgcn_rcpf(em1);
}

// Terms of the linear-in-tau slab of optical depth x along the ray (e = e^-x):
// om = 1 - e^-x and src = (1 - e^-x)/x - e^-x, by their Taylor series below
// x = 0.1 where the differences cancel in FP32 (a thin hot layer above a cold
// one can carry most of the emergent intensity).  Through the slab
// I' = I e^-x + B_top om + (B_bot - B_top) src.
__device__ inline void slab_terms(float x, float e, float& om, float& src) {
  if (x < 0.1f) {
    om = x * (1.0f + x * (-0.5f + x * (1.0f / 6.0f + x * (-1.0f / 24.0f + x * (1.0f / 120.0f + x * (-1.0f / 720.0f))))));
    src = x * (0.5f + x * (-1.0f / 3.0f + x * (0.125f + x * (-1.0f / 30.0f + x * (1.0f / 144.0f + x * (-1.0f / 840.0f))))));
  } else {
    om = 1.0f - e;
    src = om * __builtin_amdgcn_rcpf(x) - e;
  }
}

}  // namespace exofwd
