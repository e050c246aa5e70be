#pragma once
#include "common.h"

namespace exofwd {
void launch_emission(const Model& m, const Work& w, const Tables& tb, int B, void* spec, bool fp64, hipStream_t st);
hipError_t emission_configure(const Model& m, bool fp64);
size_t emission_lds_bytes(const Model& m, bool fp64);
}  // namespace exofwd
