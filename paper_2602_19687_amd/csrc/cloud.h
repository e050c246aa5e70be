// Extinction efficiency of the non-grey cloud's effective particle size
// (Section "Non-grey aerosol opacity", Eqs. 24 and 27-29) at one wavenumber,
// with its derivatives with respect to the spectral cloud parameters.  The
// material factor Q1 of Eq. 25 is folded into the effective mixing ratio, so
// the fitted curve carries no separate scale.
//
//   x = 2 pi r_eff nu
//   fit     : Q = 1 / (Q0 x^-a + x^0.2)                               (Eq. 24)
//   feature : Q = min(fit + W(x) F(lambda), 2),  W = exp(-x / 0.5),
//             F = 2 A exp(-z^2/2) Phi(xi z),  z = (lambda - lambda0) / omega   (Eqs. 27-29)
//   grey    : Q = 2
#pragma once
#include "common.h"

namespace exofwd {

// Per-sample constants: r_eff [cm], a, Q0, A, lambda0 [um], omega [um], xi.
template <typename Real>
struct CloudCoef {
  Real r, a, q0, amp, lam0, om, xi;
};

template <typename Real>
__device__ inline CloudCoef<Real> load_cloud(const double* __restrict__ cl) {
  CloudCoef<Real> c;
  c.r = (Real)cl[0];
  c.a = (Real)cl[1];
  c.q0 = (Real)cl[2];
  c.amp = (Real)cl[3];
  c.lam0 = (Real)cl[4];
  c.om = (Real)cl[5];
  c.xi = (Real)cl[6];
  return c;
}

__device__ inline float m_exp(float v) { return expf(v); }
__device__ inline double m_exp(double v) { return exp(v); }
__device__ inline float m_log(float v) { return logf(v); }
__device__ inline double m_log(double v) { return log(v); }
__device__ inline float m_erf(float v) { return erff(v); }
__device__ inline double m_erf(double v) { return erf(v); }

// Q_ext(nu); with dq != nullptr also dQ/d(log10 r_eff, a, log10 Q0, A, lambda0,
// log10 omega, xi) at fixed column (the column's own 1/r_eff is not included).
template <typename Real>
__device__ inline Real cloud_q(int kind, const CloudCoef<Real>& c, Real nu, Real* dq) {
  const Real ln10 = (Real)2.302585092994045684017991454684;
  if (dq) {
#pragma unroll
    for (int k = 0; k < kCloudSpec; ++k) dq[k] = (Real)0;
  }
  if (kind == kQextGrey) return (Real)2;
  const Real x = (Real)6.283185307179586476925286766559 * c.r * nu;
  const Real lx = m_log(x);
  const Real u = c.q0 * m_exp(-c.a * lx);
  const Real v = m_exp((Real)0.2 * lx);
  const Real qh = (Real)1 / (u + v);
  const Real uq = u * qh;   // u/(u+v), kept apart so that qh^2 never underflows alone
  if (dq) {
    dq[0] = ln10 * (c.a * uq - (Real)0.2 * v * qh) * qh;
    dq[1] = uq * lx * qh;
    dq[2] = -ln10 * uq * qh;
  }
  if (kind != kQextFeature) return qh;
  const Real lam = (Real)1.0e4 / nu;
  const Real z = (lam - c.lam0) / c.om;
  const Real e = m_exp((Real)-0.5 * z * z);
  const Real y = c.xi * z;
  const Real phi_cdf = (Real)0.5 * ((Real)1 + m_erf(y * (Real)0.70710678118654752440084436210485));
  const Real wgt = m_exp((Real)-2 * x);
  const Real f = (Real)2 * c.amp * e * phi_cdf;
  const Real q = qh + wgt * f;
  if (!(q < (Real)2)) {
    if (dq) {
#pragma unroll
      for (int k = 0; k < kCloudSpec; ++k) dq[k] = (Real)0;
    }
    return (Real)2;
  }
  if (dq) {
    const Real pdf = m_exp((Real)-0.5 * y * y) * (Real)0.39894228040143267793994605993438;
    const Real dfdz = (Real)2 * c.amp * e * (c.xi * pdf - z * phi_cdf);
    dq[0] -= (Real)2 * ln10 * x * wgt * f;
    dq[3] = wgt * (Real)2 * e * phi_cdf;
    dq[4] = -wgt * dfdz / c.om;
    dq[5] = -ln10 * z * wgt * dfdz;
    dq[6] = wgt * (Real)2 * c.amp * e * z * pdf;
  }
  return q;
}

// Condensate mass mixing ratio of one layer (Eqs. 18-20) and, with dq != nullptr,
// its derivatives with respect to the profile parameters thq[0..2]:
//   uniform: [log10 q]                          q_l = q
//   slab   : [log10 q, log10 p_top, log10 dp]   q between p_top and p_top + dp
//   power  : [log10 q_b, log10 p_b, alpha]      q_b (p_l / p_b)^alpha above p_b
// Pressures in log10 bar; lb > lt are the layer's bottom and top levels, lp its
// mid-layer pressure.  A layer that straddles a slab or power-law edge is
// covered by the fraction of its ln p extent inside the cloud.
__device__ inline double condensate_q(int prof, const double* __restrict__ thq, double lb, double lt, double lp,
                                      double* dq) {
  const double ln10 = 2.302585092994045684017991454684;
  const double q = exp10(thq[0]);
  if (dq) dq[0] = dq[1] = dq[2] = 0.0;
  if (prof == kQprofUniform) {
    if (dq) dq[0] = ln10 * q;
    return q;
  }
  // coverage of [lo, hi] (log10 bar), and its slopes in hi and lo
  double hi, lo, s_hi = 0.0, s_lo = 0.0, pw = 1.0;
  double dhi_1 = 0.0, dhi_2 = 0.0;   // d hi / d thq[1], d thq[2]
  if (prof == kQprofSlab) {
    const double pt = exp10(thq[1]), dp = exp10(thq[2]);
    hi = log10(pt + dp);
    lo = thq[1];
    dhi_1 = pt / (pt + dp);
    dhi_2 = dp / (pt + dp);
  } else {
    hi = thq[1];
    lo = lt - 3.0;   // no upper edge: the whole column above p_b
    pw = exp10(thq[2] * (lp - thq[1]));
    dhi_1 = 1.0;
  }
  if (hi < lb) s_hi = 1.0; else hi = lb;
  if (lo > lt) s_lo = -1.0; else lo = lt;
  double cov = (hi - lo) / (lb - lt);
  if (!(cov > 0.0)) return 0.0;
  const double val = q * pw * cov;
  if (dq) {
    dq[0] = ln10 * val;
    if (prof == kQprofSlab) {
      dq[1] = q * (s_hi * dhi_1 + s_lo) / (lb - lt);
      dq[2] = q * s_hi * dhi_2 / (lb - lt);
    } else {
      dq[1] = q * pw * (-thq[2] * ln10 * cov + s_hi * dhi_1 / (lb - lt));
      dq[2] = val * ln10 * (lp - thq[1]);
    }
  }
  return val;
}

}  // namespace exofwd
