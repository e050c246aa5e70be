// Correlated-k path: mixing of the absorbers' k-tables and the spectrum per bin.
#pragma once
#include "common.h"

namespace exofwd {
hipError_t ck_configure(const Model& m);
// RORR: the mixed layer optical depths into w.ckmix (nothing for the product of transmissions)
void launch_ck_mix(const Model& m, const Work& w, const Tables& tb, int B, hipStream_t st);
// the transit depth or F_p/F_* per bin into spec
void launch_ck_spectrum(const Model& m, const Work& w, const Tables& tb, int B, void* spec, hipStream_t st);
}  // namespace exofwd
