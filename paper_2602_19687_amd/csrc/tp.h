// T-p profiles of the Barstow 2020 form (Eq. 8), the modified Milne form
// (Eqs. 9-14) and the seven-parameter modified Guillot form (Eq. 16), in FP64,
// with the derivatives of T^4 with respect to their parameters for the chain
// rule (dT/dp_k = dT^4/dp_k / (4 T^3)).  Pressures enter as log10 p [bar]; the
// infrared optical depth is tau = kappa_ir p / g (Eq. 10) with p in dyn cm^-2.
#pragma once
#include "common.h"

namespace exofwd {

// Eq. 8: T / T_strat; isotherm down to 0.1 bar, adiabat (p / 0.1 bar)^kappa down
// to 1 bar, the 1-bar value below.
__device__ inline double barstow_factor(double lp) {
  if (lp <= -1.0) return 1.0;
  if (lp < 0.0) return exp10(kKappaAd * (lp + 1.0));
  return exp10(kKappaAd);
}

// Modified Milne, th = [T_int, log10 kappa_ir, T_ratio, log10 p_t/bar, beta]:
//   T^4 = 3/4 T_int^4 (tau + q),  q = q_inf + (q0 - q_inf) exp(-(p/p_t)^beta),
//   q0 = 4/3 T_ratio^4 (Eqs. 12-14), q_inf the large-depth Hopf value.
__device__ inline double milne_t4(const double* th, double lp, double g, double* d = nullptr) {
  const double ln10 = 2.302585092994045684017991454684;
  const double ti = th[0], ti4 = ti * ti * ti * ti;
  const double tau = exp10(th[1] + lp) * kBar / g;
  const double tr = th[2], q0 = 4.0 / 3.0 * tr * tr * tr * tr;
  const double x = exp10(th[4] * (lp - th[3])), e = exp(-x);
  const double q = kQHopfInf + (q0 - kQHopfInf) * e;
  if (d) {
    d[0] = 3.0 * ti * ti * ti * (tau + q);
    d[1] = 0.75 * ti4 * tau * ln10;
    d[2] = 4.0 * ti4 * e * tr * tr * tr;
    d[3] = 0.75 * ti4 * (q0 - kQHopfInf) * e * x * th[4] * ln10;
    d[4] = -0.75 * ti4 * (q0 - kQHopfInf) * e * x * (lp - th[3]) * ln10;
  }
  return 0.75 * ti4 * (tau + q);
}

// Seven-parameter modified Guillot, th = [T_int, T_eq, log10 kappa_ir, log10 gamma_v,
// q_irr0, log10 p_t/bar, beta], mu_* = 1/sqrt 3, q_int = 2/3:
//   T^4 = 3/4 T_int^4 (2/3 + tau) + 3 f_hem T_eq^4 [q_irr + 1/(g s3) + (g/s3 - 1/(g s3)) e^(-g tau s3)]
// with q_irr = 2/3 + (q_irr0 - 2/3) exp(-(p/p_t)^beta) and g = gamma_v, s3 = sqrt 3.
__device__ inline double guillot7_t4(const double* th, double lp, double g, double f_hem, double* d = nullptr) {
  const double ln10 = 2.302585092994045684017991454684;
  const double s3 = 1.7320508075688772935274463415059;
  const double ti = th[0], te = th[1];
  const double ti4 = ti * ti * ti * ti, te4 = te * te * te * te;
  const double tau = exp10(th[2] + lp) * kBar / g;
  const double gam = exp10(th[3]);
  const double x = exp10(th[6] * (lp - th[5])), e = exp(-x);
  const double qi = 2.0 / 3.0 + (th[4] - 2.0 / 3.0) * e;
  const double ev = exp(-gam * tau * s3);
  const double cv = gam / s3 - 1.0 / (gam * s3);
  const double bk = qi + 1.0 / (gam * s3) + cv * ev;
  const double irr = 3.0 * f_hem * te4;
  if (d) {
    d[0] = 3.0 * ti * ti * ti * (2.0 / 3.0 + tau);
    d[1] = 12.0 * f_hem * te * te * te * bk;
    d[2] = (0.75 * ti4 - irr * cv * ev * gam * s3) * tau * ln10;
    const double dbk = -1.0 / (gam * gam * s3) + (1.0 / s3 + 1.0 / (gam * gam * s3)) * ev - cv * ev * tau * s3;
    d[3] = irr * dbk * gam * ln10;
    d[4] = irr * e;
    d[5] = irr * (th[4] - 2.0 / 3.0) * e * x * th[6] * ln10;
    d[6] = -irr * (th[4] - 2.0 / 3.0) * e * x * (lp - th[5]) * ln10;
  }
  return 0.75 * ti4 * (2.0 / 3.0 + tau) + irr * bk;
}

}  // namespace exofwd
