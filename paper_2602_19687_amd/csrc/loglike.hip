// Binned Gaussian log-likelihood in FP64 (Eq. 1-3): box-car bin means of the
// spectrum, the instrument offset on masked bins, lnL and d lnL / d m_k; with
// the cloudy/clear mixing (Eq. 26) also the mixed spectrum and d lnL / d f_cld.
// One workgroup per sample.  A group of lanes (8 to 64, after the mean bin width)
// sums one bin at a time: its lanes stride through the bin's wavenumbers
// (coalesced) and their partial sums meet in a fixed butterfly; then one thread
// per bin forms the bin's terms, and the sum over bins is a fixed-order tree.
#include "kernels.h"

namespace exofwd {

constexpr int kBlockLL = 1024;   // threads per sample: 16 waves (a small batch still fills the chip)

// sum over the aligned group of g lanes holding v (every lane of the group gets it)
__device__ inline double group_sum_d(double v, int g) {
  for (int off = g >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

template <typename SpecT>
__global__ __launch_bounds__(kBlockLL) void k_loglike(Model m, Work w, const double* __restrict__ params,
                                                    const SpecT* __restrict__ spec, SpecT* __restrict__ spec_out,
                                                    const int32_t* __restrict__ lo, const int32_t* __restrict__ hi,
                                                    const double* __restrict__ y, const double* __restrict__ yerr,
                                                    const uint8_t* __restrict__ mask, double* __restrict__ lnl,
                                                    int32_t* __restrict__ status_out) {
  const int b = blockIdx.x, tid = threadIdx.x;
  __shared__ double s_part[kBlockLL], s_fpart[kBlockLL], s_mpart[kBlockLL];
  __shared__ double s_sum[kBlockLL], s_sumcf[kBlockLL];
  // cloudy/clear mixing (Eq. 26): virtual samples 2b (cloudy) and 2b+1 (clear) give
  // the spectrum f Phi_cld + (1 - f) Phi_cf; their dm carry the factors f and 1 - f
  const bool mix = m.has_fcld;
  const int bc = mix ? 2 * b : b;
  int status = mix ? (w.status[bc] | w.status[bc + 1]) : w.status[b];
  double* dm = w.dm + (size_t)bc * m.K;
  double* dm_cf = mix ? dm + m.K : nullptr;
  if (status) {
    for (int k = tid; k < m.K; k += kBlockLL) {
      dm[k] = 0.0;
      if (mix) dm_cf[k] = 0.0;
    }
    if (mix && spec_out)
      for (int i = tid; i < m.n_nu; i += kBlockLL) spec_out[(size_t)b * m.n_nu + i] = (SpecT)__builtin_nan("");
    if (tid == 0) {
      if (lnl) lnl[b] = kInvalidLnL;
      if (status_out) status_out[b] = status;
      if (mix) w.fbar[b] = 0.0;
      w.mdot[b] = 0.0;
    }
    return;
  }
  const double* th = params + (size_t)b * m.P;
  const double offset = m.has_offset ? th[m.idx_offset] * 1.0e-6 : 0.0;
  const double f = mix ? th[m.idx_fcld] : 1.0;
  const double infl = exp10(2.0 * m.err_c);
  const double half_ln2pi = 0.91893853320467274178032973640562;
  const SpecT* sp = spec + (size_t)bc * m.n_nu;
  const SpecT* sp_cf = mix ? sp + m.n_nu : nullptr;
  if (mix && spec_out)
    for (int i = tid; i < m.n_nu; i += kBlockLL)
      spec_out[(size_t)b * m.n_nu + i] = (SpecT)(f * (double)sp[i] + (1.0 - f) * (double)sp_cf[i]);
  double part = 0.0, fpart = 0.0, mpart = 0.0;
  const int gl = m.ll_lanes, glane = tid & (gl - 1), grp = tid / gl, ngrp = kBlockLL / gl;
  for (int k0 = 0; k0 < m.K; k0 += kBlockLL) {
    const int kn = min(kBlockLL, m.K - k0);
    // bin sums, a group of lanes per bin
    for (int kk = grp; kk < kn; kk += ngrp) {
      const int k = k0 + kk;
      double sum = 0.0, sum_cf = 0.0;
      const int i1 = hi[k];
      for (int i = lo[k] + glane; i < i1; i += gl) {
        sum += (double)sp[i];
        if (mix) sum_cf += (double)sp_cf[i];
      }
      sum = group_sum_d(sum, gl);
      if (mix) sum_cf = group_sum_d(sum_cf, gl);
      if (glane == 0) {
        s_sum[kk] = sum;
        s_sumcf[kk] = sum_cf;
      }
    }
    __syncthreads();
    // the bin's terms, a thread per bin
    if (tid < kn) {
      const int k = k0 + tid;
      const double cnt = (double)(hi[k] - lo[k]);
      const double m_cld = s_sum[tid] / cnt, m_cf = s_sumcf[tid] / cnt;
      const double mk = (mix ? f * m_cld + (1.0 - f) * m_cf : m_cld) + (mask && mask[k] ? offset : 0.0);
      const double s2 = yerr[k] * yerr[k] + infl;
      const double r = y[k] - mk;
      part += -0.5 * log(s2) - half_ln2pi - 0.5 * r * r / s2;
      if (mix) {
        dm[k] = f * r / s2;
        dm_cf[k] = (1.0 - f) * r / s2;
        fpart += r / s2 * (m_cld - m_cf);
      } else {
        dm[k] = r / s2;
      }
      mpart += r / s2 * (mix ? f * m_cld + (1.0 - f) * m_cf : m_cld);
    }
    __syncthreads();   // the next chunk of bins overwrites the sums
  }
  s_part[tid] = part;
  s_fpart[tid] = fpart;
  s_mpart[tid] = mpart;
  __syncthreads();
  for (int h = kBlockLL / 2; h > 0; h >>= 1) {
    if (tid < h) {
      s_part[tid] += s_part[tid + h];
      s_fpart[tid] += s_fpart[tid + h];
      s_mpart[tid] += s_mpart[tid + h];
    }
    __syncthreads();
  }
  if (tid == 0) {
    double v = s_part[0];
    if (!isfinite(v)) {
      v = kInvalidLnL;
      status = kNonfinite;
      w.status[bc] = status;
      if (mix) w.status[bc + 1] = status;
    }
    if (lnl) lnl[b] = v;
    w.lnl_tmp[b] = v;
    if (mix) w.fbar[b] = status ? 0.0 : s_fpart[0];
    w.mdot[b] = status ? 0.0 : s_mpart[0];
    if (status_out) status_out[b] = status;
  }
}

__global__ __launch_bounds__(kBlock) void k_mix_grad(Model m, Work w, int B, double* __restrict__ grad) {
  const long i = (long)blockIdx.x * kBlock + threadIdx.x;
  if (i >= (long)B * m.P) return;
  const int b = (int)(i / m.P), j = (int)(i % m.P);
  grad[i] = j == m.idx_fcld ? w.fbar[b] : w.gv[(size_t)(2 * b) * m.P + j] + w.gv[(size_t)(2 * b + 1) * m.P + j];
}

void launch_loglike(const Model& m, const Work& w, int B, const double* params, const void* spec, void* spec_out,
                    bool spec_f64, const int32_t* bin_lo, const int32_t* bin_hi, const double* y, const double* yerr,
                    const uint8_t* mask, double* lnl, int32_t* status_out, hipStream_t st) {
  if (spec_f64)
    hipLaunchKernelGGL(k_loglike<double>, dim3(B), dim3(kBlockLL), 0, st, m, w, params, (const double*)spec,
                       (double*)spec_out, bin_lo, bin_hi, y, yerr, mask, lnl, status_out);
  else
    hipLaunchKernelGGL(k_loglike<float>, dim3(B), dim3(kBlockLL), 0, st, m, w, params, (const float*)spec,
                       (float*)spec_out, bin_lo, bin_hi, y, yerr, mask, lnl, status_out);
}

void launch_mix_grad(const Model& m, const Work& w, int B, double* grad, hipStream_t st) {
  const long n = (long)B * m.P;
  hipLaunchKernelGGL(k_mix_grad, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, m, w, B, grad);
}

}  // namespace exofwd
