#pragma once
#include "common.h"

namespace exofwd {
// dtau_out (may be null): layer optical depths [B][L_pad][n_nu_pad] for the reverse pass, float in reduced
// precision, double in FP64
void launch_emission(const Model& m, const Work& w, const Tables& tb, int B, void* spec, bool fp64, hipStream_t st,
                     void* dtau_out = nullptr);
hipError_t emission_configure(const Model& m, bool fp64);
size_t emission_lds_bytes(const Model& m, bool fp64);

// Planck intensity per unit wavenumber, 2 h c^2 nu^3 / (e^y - 1) with y = h c nu / k T,
// from c1n3 = 2 h c^2 nu^3, c2n_log2e = log2(e) h c nu / k and inv_t = 1/T; em1
// returns e^y - 1.  FP32 holds y only to about 1e-6 absolute at y ~ 20, and e^y
// inherits that as a relative error in B, which the emitted flux, and through the
// likelihood residuals near the best fit the gradient, would carry.  So the exponent
// a = log2(e) y is formed in FP64 and split as a = a_hi + a_lo with a_hi exactly a
// float: e^y = 2^a_hi (1 + a_lo ln 2) (a_lo < 2^-24 a_hi, so the first-order term is
// exact to FP32).  Below y = 0.1, e^y - 1 comes from its series (through y^5).
__device__ inline float planck_split(float c1n3, double c2n_log2e, double inv_t, float& y, float& em1) {
  const double a = c2n_log2e * inv_t;
  y = (float)(a * 0.69314718055994530942);
  if (y < 0.1f) {
    em1 = y * (1.0f + y * (0.5f + y * (1.0f / 6.0f + y * (1.0f / 24.0f + y * (1.0f / 120.0f)))));
  } else {
    const float ah = (float)a;
    const float al = (float)(a - (double)ah);
    em1 = fmaf(__builtin_amdgcn_exp2f(ah), fmaf(al, 0.69314718055994530942f, 1.0f), -1.0f);
  }
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
