// Adjoint of the transmission path: per-sample partial sums from the fused
// reverse kernel and the FP64 chain to d lnL / d params.
#pragma once
#include "common.h"

#include <functional>

namespace exofwd {

struct AdjWork {
  int n_chunks;        // wavenumber chunks per sample in the reverse kernel
  double* layer_sums;  // [B][n_chunks][L_pad][n_sums] per-layer sums over nu
  double* pbar;        // [B][n_chunks][L_pad][L_pad] d lnL / d P_il partials
  double* abar;        // [B][n_chunks][L_pad + 1] d lnL / d area_i, last = d lnL / d core
};

bool adjoint_alloc(AdjWork& aw, const Model& m, int B, bool fp64, const std::function<void*(size_t)>& alloc);
hipError_t adjoint_configure(const Model& m, bool fp64);
void launch_trans_adjoint(const Model& m, const Work& w, const Tables& tb, const AdjWork& aw, int B, bool fp64,
                          hipStream_t st);
void launch_chain(const Model& m, const Work& w, const AdjWork& aw, int B, const double* params, const uint8_t* mask,
                  double* grad, bool fp64, hipStream_t st);
bool adjoint_ready();

}  // namespace exofwd
