// Binned Gaussian log-likelihood in FP64 (Eq. 1-3): box-car bin means of the
// spectrum, the instrument offset on masked bins, lnL and d lnL / d m_k.
// One workgroup per sample; the sum over bins is a fixed-order tree.
#include "kernels.h"

namespace exofwd {

template <typename SpecT>
__global__ __launch_bounds__(kBlock) void k_loglike(Model m, Work w, const double* __restrict__ params,
                                                    const SpecT* __restrict__ spec, const int32_t* __restrict__ lo,
                                                    const int32_t* __restrict__ hi, const double* __restrict__ y,
                                                    const double* __restrict__ yerr, const uint8_t* __restrict__ mask,
                                                    double* __restrict__ lnl, int32_t* __restrict__ status_out) {
  const int b = blockIdx.x, tid = threadIdx.x;
  __shared__ double s_part[kBlock];
  int status = w.status[b];
  double* dm = w.dm + (size_t)b * m.K;
  if (status) {
    for (int k = tid; k < m.K; k += kBlock) dm[k] = 0.0;
    if (tid == 0) {
      if (lnl) lnl[b] = kInvalidLnL;
      if (status_out) status_out[b] = status;
    }
    return;
  }
  const double offset = m.has_offset ? params[(size_t)b * m.P + m.idx_offset] * 1.0e-6 : 0.0;
  const double infl = exp10(2.0 * m.err_c);
  const double half_ln2pi = 0.91893853320467274178032973640562;
  const SpecT* sp = spec + (size_t)b * m.n_nu;
  double part = 0.0;
  for (int k = tid; k < m.K; k += kBlock) {
    double sum = 0.0;
    for (int i = lo[k]; i < hi[k]; ++i) sum += (double)sp[i];
    const double mk = sum / (double)(hi[k] - lo[k]) + (mask && mask[k] ? offset : 0.0);
    const double s2 = yerr[k] * yerr[k] + infl;
    const double r = y[k] - mk;
    part += -0.5 * log(s2) - half_ln2pi - 0.5 * r * r / s2;
    dm[k] = r / s2;
  }
  s_part[tid] = part;
  __syncthreads();
  for (int h = kBlock / 2; h > 0; h >>= 1) {
    if (tid < h) s_part[tid] += s_part[tid + h];
    __syncthreads();
  }
  if (tid == 0) {
    double v = s_part[0];
    if (!isfinite(v)) {
      v = kInvalidLnL;
      status = kNonfinite;
      w.status[b] = status;
    }
    if (lnl) lnl[b] = v;
    w.lnl_tmp[b] = v;
    if (status_out) status_out[b] = status;
  }
}

void launch_loglike(const Model& m, const Work& w, int B, const double* params, const void* spec, bool spec_f64,
                    const int32_t* bin_lo, const int32_t* bin_hi, const double* y, const double* yerr,
                    const uint8_t* mask, double* lnl, int32_t* status_out, hipStream_t st) {
  if (spec_f64)
    hipLaunchKernelGGL(k_loglike<double>, dim3(B), dim3(kBlock), 0, st, m, w, params, (const double*)spec, bin_lo,
                       bin_hi, y, yerr, mask, lnl, status_out);
  else
    hipLaunchKernelGGL(k_loglike<float>, dim3(B), dim3(kBlock), 0, st, m, w, params, (const float*)spec, bin_lo,
                       bin_hi, y, yerr, mask, lnl, status_out);
}

}  // namespace exofwd
