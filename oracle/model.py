"""The forward model, step by step, in FP64 (complex-step safe).

Test infrastructure only (see the package docstring).

Notation follows the paper: levels j = 0..L (0 at the bottom), layers
l = 0..L-1 between levels l and l+1, impact parameters b_i at layer mid radii,
species s, wavenumber nu [cm^-1].  Every branch (clamps, table cells, case
selections) is decided on real parts, so that a complex perturbation of the
parameters carries the derivative through unchanged (complex-step
differentiation).
"""
from __future__ import annotations

import numpy as np
from scipy import special

# CODATA 2018 / IAU 2015 constants in cgs; the paper works in cgs but gives none
K_B = 1.380649e-16          # erg K^-1
H_PL = 6.62607015e-27       # erg s
C_LIGHT = 2.99792458e10     # cm s^-1
M_U = 1.66053906660e-24     # g
BAR = 1.0e6                 # dyn cm^-2
G_GRAV = 6.67430e-8         # cm^3 g^-1 s^-2
M_JUP = 1.89813e30          # g (nominal G M_J / G)
HE_H2 = 0.164               # He/H2 number ratio (free-chemistry filling, Eq. 36)
M_H2 = 2.01588              # amu
M_HE = 4.002602             # amu

# per-sample status bits
S_BAD_VMR = 1
S_UNBOUND = 2
S_NONFINITE = 4
S_BAD_T = 8
S_BAD_LAYERS = 16
INVALID_LNL = -1.0e300      # log-likelihood of an invalid forward output (Section "Likelihood")

TP_ISOTHERMAL, TP_GUILLOT3, TP_PCHIP, TP_BARSTOW, TP_MILNE, TP_GUILLOT7 = 0, 1, 2, 3, 4, 5
TP_NPARAM = {TP_ISOTHERMAL: 1, TP_GUILLOT3: 3, TP_BARSTOW: 1, TP_MILNE: 5, TP_GUILLOT7: 7}
KAPPA_AD = 2.0 / 7.0        # adiabatic exponent of the Barstow profile (Eq. 8)
Q_HOPF_INF = 0.710446       # Hopf function at large optical depth (Milne q_inf)


def _re(x):
    return np.real(x)


# ---------------------------------------------------------------------------
# a1: pressure grid and T-p profile
def level_pressures(p_bot_bar, p_top_bar, n_layers):
    """Level and layer pressures [dyn cm^-2].

    Reading of "layers evenly log-spaced between p_bot and p_top" (WASP-17b
    setup): n_layers+1 log-uniform *levels*, level 0 at p_bot; a layer's
    pressure is the geometric mean of its two edges.
    """
    logp = np.linspace(np.log10(p_bot_bar), np.log10(p_top_bar), n_layers + 1)
    p_lev = 10.0 ** logp * BAR
    p_lay = np.sqrt(p_lev[:-1] * p_lev[1:])
    return p_lev, p_lay


def tp_isothermal(t_iso, p):
    """Isothermal profile, Eq. 7: T(p) = T_iso."""
    return t_iso * np.ones_like(p)


def tp_guillot3(t_int, t_eq, log10_gamma, p, kappa_ir, g_ref, f_hem):
    """Modified Guillot profile (Eq. 16) in its three-parameter form.

    Both Hopf-like functions are held at the Eddington value 2/3 (q_int = 2/3
    as the paper recommends for hot Jupiters; q_irr = 2/3 = q_irr,inf), the
    optical depth is tau = kappa_ir p / g (Eq. 10) and mu_* = 1/sqrt(3).
    Parameters: T_int, T_eq and log10 gamma_v.
    """
    gam = 10.0 ** log10_gamma
    tau = kappa_ir * p / g_ref
    s3 = np.sqrt(3.0)
    q = 2.0 / 3.0
    t4 = (0.75 * t_int ** 4 * (q + tau)
          + 0.75 * t_eq ** 4 * 4.0 * f_hem
          * (q + 1.0 / (gam * s3) + (gam / s3 - 1.0 / (gam * s3)) * np.exp(-gam * tau * s3)))
    return t4 ** 0.25


def tp_barstow(t_strat, p):
    """Barstow 2020 profile, Eq. 8: T_strat up to 0.1 bar, an adiabat
    T_strat (p / 0.1 bar)^kappa between 0.1 and 1 bar, and its 1-bar value
    below.  kappa = 2/7.  p in dyn cm^-2; one parameter, T_strat."""
    pb = np.asarray(p, dtype=np.float64) / BAR
    f = np.where(pb <= 0.1, 1.0, np.where(pb < 1.0, (pb / 0.1) ** KAPPA_AD, 10.0 ** KAPPA_AD))
    return t_strat * f


def hopf_stretched(q0, q_inf, p, p_t, beta):
    """Stretched-exponential Hopf-like function in pressure, Eq. 12:
    q(p) = q_inf + (q0 - q_inf) exp[-(p/p_t)^beta]."""
    return q_inf + (q0 - q_inf) * np.exp(-(p / p_t) ** beta)


def tp_milne(t_int, log10_kappa, t_ratio, log10_pt_bar, beta, p, g_ref):
    """Modified Milne profile, Eqs. 9-14: T^4 = 3/4 T_int^4 [tau + q(tau)] with
    tau = kappa_ir p / g (Eq. 10) and q the stretched exponential of Eq. 12,
    q0 = 4/3 (T_skin/T_int)^4 = 4/3 T_ratio^4 (Eqs. 13-14).

    Readings: q_inf is held at the classic large-depth Hopf value 0.710446
    (the paper names five retrieved parameters, q_inf not among them);
    kappa_ir and p_t are retrieved as log10 (cgs and bar).  Parameters:
    T_int, log10 kappa_ir, T_ratio, log10 p_t [bar], beta."""
    tau = 10.0 ** log10_kappa * p / g_ref
    q0 = 4.0 / 3.0 * t_ratio ** 4
    q = hopf_stretched(q0, Q_HOPF_INF, p, 10.0 ** log10_pt_bar * BAR, beta)
    return (0.75 * t_int ** 4 * (tau + q)) ** 0.25


def tp_guillot7(t_int, t_eq, log10_kappa, log10_gamma, q_irr0, log10_pt_bar, beta, p, g_ref, f_hem):
    """Modified Guillot profile, Eq. 16, in its seven-parameter form.

    T^4 = 3/4 T_int^4 [q_int + tau]
        + 3/4 T_eq^4 4 f_hem [q_irr(tau) + 1/(gamma sqrt 3) + (gamma/sqrt 3 - 1/(gamma sqrt 3)) e^(-gamma tau sqrt 3)]
    with mu_* = 1/sqrt 3, q_int = 2/3 (Eddington, as the paper recommends for
    hot Jupiters), q_irr the stretched exponential of Eq. 12 from q_irr,0 to
    q_irr,inf = 2/3, tau = kappa_ir p / g (Eq. 10) and f_hem a fixed workload
    constant.  Readings: kappa_ir, gamma_v and p_t are retrieved as log10 (cgs,
    -, bar).  Parameters: T_int, T_eq, log10 kappa_ir, log10 gamma_v, q_irr,0,
    log10 p_t [bar], beta.  With q_irr,0 = 2/3 this is the three-parameter form
    at kappa_ir = 10^log10_kappa."""
    gam = 10.0 ** log10_gamma
    tau = 10.0 ** log10_kappa * p / g_ref
    s3 = np.sqrt(3.0)
    q_irr = hopf_stretched(q_irr0, 2.0 / 3.0, p, 10.0 ** log10_pt_bar * BAR, beta)
    t4 = (0.75 * t_int ** 4 * (2.0 / 3.0 + tau)
          + 0.75 * t_eq ** 4 * 4.0 * f_hem
          * (q_irr + 1.0 / (gam * s3) + (gam / s3 - 1.0 / (gam * s3)) * np.exp(-gam * tau * s3)))
    return t4 ** 0.25


def pchip(xk, yk, x):
    """Monotone piecewise-cubic Hermite interpolation (Fritsch-Carlson slopes
    with the Fritsch-Butland weighted harmonic mean at interior knots and the
    shape-preserving three-point end slopes), complex-safe in ``yk``.

    This is the node interpolant the paper uses for its optical-constant nodes
    (Section "Direct (n, k) retrieval"); here it interpolates knot
    temperatures in log10 p.  ``xk`` must be strictly increasing and real.
    """
    xk = np.asarray(xk, dtype=np.float64)
    yk = np.asarray(yk)
    n = len(xk)
    h = np.diff(xk)
    delta = np.diff(yk) / h
    d = np.zeros(n, dtype=yk.dtype)
    for k in range(1, n - 1):
        a, b = _re(delta[k - 1]), _re(delta[k])
        if a == 0.0 or b == 0.0 or np.sign(a) != np.sign(b):
            d[k] = 0.0
        else:
            w1 = 2.0 * h[k] + h[k - 1]
            w2 = h[k] + 2.0 * h[k - 1]
            d[k] = (w1 + w2) / (w1 / delta[k - 1] + w2 / delta[k])

    def end(h0, h1, m0, m1):
        dd = ((2.0 * h0 + h1) * m0 - h0 * m1) / (h0 + h1)
        if np.sign(_re(dd)) != np.sign(_re(m0)):
            return 0.0 * dd
        if np.sign(_re(m0)) != np.sign(_re(m1)) and abs(_re(dd)) > abs(3.0 * _re(m0)):
            return 3.0 * m0
        return dd

    if n == 2:
        d[0] = d[1] = delta[0]
    else:
        d[0] = end(h[0], h[1], delta[0], delta[1])
        d[-1] = end(h[-1], h[-2], delta[-1], delta[-2])
    x = np.asarray(x, dtype=np.float64)
    k = np.clip(np.searchsorted(xk, x, side="right") - 1, 0, n - 2)
    t = (x - xk[k]) / h[k]
    h00 = (1 + 2 * t) * (1 - t) ** 2
    h10 = t * (1 - t) ** 2
    h01 = t * t * (3 - 2 * t)
    h11 = t * t * (t - 1)
    return h00 * yk[k] + h10 * h[k] * d[k] + h01 * yk[k + 1] + h11 * h[k] * d[k + 1]


def tp_profile(wl, tp_theta, p, g=None):
    """T at pressures p [dyn cm^-2] for the workload's profile kind; g is the
    gravity in the infrared optical depth tau = kappa_ir p / g (default: the
    workload's g_ref)."""
    kind = wl["tp"]
    g = wl["g_ref"] if g is None else g
    if kind == TP_ISOTHERMAL:
        return tp_isothermal(tp_theta[0], p)
    if kind == TP_GUILLOT3:
        return tp_guillot3(tp_theta[0], tp_theta[1], tp_theta[2], p,
                           wl["kappa_ir"], g, wl["f_hem"])
    if kind == TP_BARSTOW:
        return tp_barstow(tp_theta[0], p)
    if kind == TP_MILNE:
        return tp_milne(*tp_theta, p, g)
    if kind == TP_GUILLOT7:
        return tp_guillot7(*tp_theta, p, g, wl["f_hem"])
    # knots equally spaced in log10 p from p_top (knot 0) to p_bot (last knot)
    nk = len(tp_theta)
    xk = np.linspace(np.log10(wl["p_top"]), np.log10(wl["p_bot"]), nk)
    return pchip(xk, np.asarray(tp_theta), np.log10(p / BAR))


# ---------------------------------------------------------------------------
# a2: free chemistry with H2/He filling
def chemistry(log10_x, masses, mu_fixed=0.0):
    """Volume mixing ratios and mean molecular weight (Eq. 35-36).

    X_s = 10^theta_s; the remainder is H2 + He with X_He/X_H2 = 0.164.
    mu [amu] is the mixing-ratio weighted mass unless ``mu_fixed`` > 0.
    Returns (X_s, X_H2, X_He, mu, valid); invalid when sum X_s >= 1.
    """
    x = 10.0 ** np.asarray(log10_x)
    sx = np.sum(x)
    x_h2 = (1.0 - sx) / (1.0 + HE_H2)
    x_he = HE_H2 * x_h2
    if mu_fixed > 0.0:
        mu = mu_fixed + 0.0 * sx
    else:
        mu = x_h2 * M_H2 + x_he * M_HE + np.sum(x * np.asarray(masses))
    return x, x_h2, x_he, mu, bool(_re(sx) < 1.0)


# ---------------------------------------------------------------------------
# a3: hydrostatic altitude grid
def altitudes(t_lay, p_lev, mu, g_ref, r_ref, p_ref, constant_g=False):
    """Level radii [cm] from hydrostatic balance with inverse-square gravity.

    The paper fixes a reference radius R_ref at a reference pressure p_ref with
    gravity g_ref there (HD 209458b setup) but prints no integration rule.
    Reading: g(r) = g_ref (R_ref/r)^2 and each layer isothermal at its layer
    temperature, so u = 1/r is exactly linear in ln p inside a layer:
        du = (k_B T / (mu m_u g_ref R_ref^2)) d ln p.
    The layer holding p_ref is split at p_ref.  Returns (r_lev, valid); valid
    is False when some u <= 0 (an unbound atmosphere).
    """
    n = len(t_lay)
    if constant_g:
        # test mode: uniform gravity, dr = (k_B T / (mu m_u g_ref)) ln(p_bottom/p_top)
        hh = K_B / (mu * M_U * g_ref)
        lref = int(np.searchsorted(-p_lev, -p_ref, side="left")) - 1
        lref = min(max(lref, 0), n - 1)
        r = np.empty(n + 1, dtype=np.result_type(hh, t_lay, r_ref))
        r[lref] = r_ref - hh * t_lay[lref] * np.log(p_lev[lref] / p_ref)
        r[lref + 1] = r_ref + hh * t_lay[lref] * np.log(p_ref / p_lev[lref + 1])
        for j in range(lref - 1, -1, -1):
            r[j] = r[j + 1] - hh * t_lay[j] * np.log(p_lev[j] / p_lev[j + 1])
        for j in range(lref + 1, n):
            r[j + 1] = r[j] + hh * t_lay[j] * np.log(p_lev[j] / p_lev[j + 1])
        return r, bool(np.all(_re(r) > 0.0))
    kk = K_B / (mu * M_U * g_ref * r_ref ** 2)
    u_ref = 1.0 / r_ref
    # layer holding p_ref: p_lev[l] >= p_ref > p_lev[l+1]; outside the grid the
    # bottom or top layer extends the integration
    lref = int(np.searchsorted(-p_lev, -p_ref, side="left")) - 1
    lref = min(max(lref, 0), n - 1)
    u = np.empty(n + 1, dtype=np.result_type(kk, t_lay))
    u[lref] = u_ref + kk * t_lay[lref] * np.log(p_lev[lref] / p_ref)
    u[lref + 1] = u_ref - kk * t_lay[lref] * np.log(p_ref / p_lev[lref + 1])
    for j in range(lref - 1, -1, -1):
        u[j] = u[j + 1] + kk * t_lay[j] * np.log(p_lev[j] / p_lev[j + 1])
    for j in range(lref + 1, n):
        u[j + 1] = u[j] - kk * t_lay[j] * np.log(p_lev[j] / p_lev[j + 1])
    valid = bool(np.all(_re(u) > 0.0))
    return 1.0 / u, valid


# ---------------------------------------------------------------------------
# a5: opacity
def interp_index(grid, x):
    """Cell index and weight for linear interpolation on an increasing grid.

    x is clamped to the grid; i is the largest index with grid[i] <= x, capped
    at n-2; w = (x - grid[i]) / (grid[i+1] - grid[i]).  A clamped x has a
    real weight (zero derivative), an interior x carries its complex part.
    """
    xr = _re(x)
    if xr <= grid[0]:
        return 0, 0.0
    if xr >= grid[-1]:
        return len(grid) - 2, 1.0
    i = int(np.searchsorted(grid, xr, side="right")) - 1
    i = min(max(i, 0), len(grid) - 2)
    return i, (x - grid[i]) / (grid[i + 1] - grid[i])


def bilinear_log_table(table, t_grid, logp_grid, t, logp):
    """log10 sigma(nu) from a [nT][nP][nu] table, bilinear in (T, log10 p).

    Reading (the paper names OS tables but no interpolation rule): bilinear in
    T and log10 p on log10 sigma, clamped at the table edges.
    """
    it, wt = interp_index(t_grid, t)
    ip, wp = interp_index(logp_grid, logp)
    t00 = table[it, ip]
    t10 = table[it + 1, ip]
    t01 = table[it, ip + 1]
    t11 = table[it + 1, ip + 1]
    return ((1 - wt) * (1 - wp) * t00 + wt * (1 - wp) * t10
            + (1 - wt) * wp * t01 + wt * wp * t11)


def cia_log(table, tc_grid, t):
    """log10 k(nu) of one CIA pair, linear in T on a [nTc][nu] table (clamped)."""
    i, w = interp_index(tc_grid, t)
    return (1 - w) * table[i] + w * table[i + 1]


def cloud_fraction(p_bottom, p_top, p_cloud):
    """Fraction (in ln p) of a layer inside a grey deck whose top is p_cloud.

    Reading of the slab profile (Eq. 18) with the grey limit Q_ext = 2: the
    deck fills every pressure >= p_cloud; the layer holding p_cloud is covered
    by the fraction of its ln p extent that lies below p_cloud.
    """
    f = (np.log(p_bottom) - np.log(p_cloud)) / (np.log(p_bottom) - np.log(p_top))
    fr = _re(f)
    if fr <= 0.0:
        return 0.0
    if fr >= 1.0:
        return 1.0
    return f


# ---------------------------------------------------------------------------
# non-grey aerosol opacity (Section "Non-grey aerosol opacity")
CLOUD_GREY_DECK = 0       # slab deck from P_cloud down, Q_ext = 2, fixed kappa (R9)
CLOUD_NONGREY = 1         # q_c(p) profile and Q_ext(x, lambda), Eqs. 18-29
QPROF_UNIFORM, QPROF_SLAB, QPROF_POWER = 0, 1, 2
QEXT_FIT, QEXT_FIT_FEATURE, QEXT_GREY = 0, 1, 2
X0_FEATURE = 0.5          # transition size parameter of the feature window (Eq. 29)
Q_MAX = 2.0               # cap of the total extinction efficiency (Eq. 27)


def nongrey_param_count(wl):
    """[log10 r_eff/um, a, log10 Q0] (fit), profile parameters (1 or 3), feature (4)."""
    n = 1 if wl["cloud_qext"] == QEXT_GREY else 3
    n += 1 if wl["cloud_profile"] == QPROF_UNIFORM else 3
    n += 4 if wl["cloud_qext"] == QEXT_FIT_FEATURE else 0
    return n


def layer_coverage(p_bottom, p_top, p_hi, p_lo):
    """Fraction, in ln p, of the layer between levels p_bottom > p_top that lies
    inside the pressure range [p_lo, p_hi] (the same rule as the grey deck's
    partial layer, so the profile's edges move the optical depth continuously)."""
    lb, lt = np.log(p_bottom), np.log(p_top)
    hi = np.log(p_hi) if np.real(np.log(p_hi)) < np.real(lb) else lb
    lo = np.log(p_lo) if np.real(np.log(p_lo)) > np.real(lt) else lt
    f = (hi - lo) / (lb - lt)
    return f if np.real(f) > 0.0 else 0.0 * f


def condensate_profile(wl, cp, p_lev, p_lay):
    """Effective condensate mass mixing ratio of every layer (Eqs. 18-20).

    uniform : q_l = q                                               (Eq. 18)
    slab    : q between p_top and p_top + dp, else 0                (Eq. 19)
    power   : q_base (p / p_base)^alpha above p_base, 0 below       (Eq. 20)
    The power law is taken at the layer pressure; slab and power-law edges
    cover the layers that straddle them by their ln p fraction.
    """
    prof = wl["cloud_profile"]
    n_lay = len(p_lay)
    q = [None] * n_lay
    if prof == QPROF_UNIFORM:
        for l in range(n_lay):
            q[l] = 10.0 ** cp["q"][0] * np.ones(1)[0]
    elif prof == QPROF_SLAB:
        p_top = 10.0 ** cp["q"][1] * BAR
        p_bot = p_top + 10.0 ** cp["q"][2] * BAR
        for l in range(n_lay):
            q[l] = 10.0 ** cp["q"][0] * layer_coverage(p_lev[l], p_lev[l + 1], p_bot, p_top)
    else:
        p_base = 10.0 ** cp["q"][1] * BAR
        for l in range(n_lay):
            cov = layer_coverage(p_lev[l], p_lev[l + 1], p_base, p_lev[-1] * 1e-3)
            q[l] = 10.0 ** cp["q"][0] * (p_lay[l] / p_base) ** cp["q"][2] * cov
    return np.array(q)


def feature_efficiency(feat, lam_um):
    """Skew-normal absorption feature (Eq. 28): 2 A exp(-z^2/2) Phi(xi z),
    z = (lambda - lambda0) / omega, Phi the standard normal CDF; feat is
    (A, lambda0 [um], log10 omega [um], xi)."""
    amp, lam0, log_w, xi = feat
    z = (lam_um - lam0) / 10.0 ** log_w
    return 2.0 * amp * np.exp(-0.5 * z * z) * 0.5 * (1.0 + special.erf(xi * z / np.sqrt(2.0)))


def extinction_efficiency(wl, cp, nu):
    """Q_ext(nu) of the effective particle size r_eff (Eqs. 24, 27-29), with the
    material factor Q1 folded into the effective mixing ratio (Eq. 25):
      fit     : Q = 1 / (Q0 x^-a + x^0.2),  x = 2 pi r_eff / lambda
      feature : Q = min(fit + W(x) Q_feat(lambda), Q_max), W = exp(-x / x0),
                Q_feat = 2 A exp(-z^2/2) Phi(xi z), z = (lambda - lambda0) / omega
      grey    : Q = 2 (geometric-optics limit)."""
    r = 1.0e-4 * 10.0 ** cp["r"]
    if wl["cloud_qext"] == QEXT_GREY:
        return 2.0 + 0.0 * nu * r, r
    x = 2.0 * np.pi * r * nu
    q = 1.0 / (10.0 ** cp["q0"] * x ** (-cp["a"]) + x ** 0.2)
    if wl["cloud_qext"] == QEXT_FIT_FEATURE:
        q = q + np.exp(-x / X0_FEATURE) * feature_efficiency(cp["feat"], 1.0e4 / nu)
        q = np.where(np.real(q) < Q_MAX, q, Q_MAX + 0.0 * q)
    return q, r


def nongrey_cloud_dtau(wl, cp, p_lev, p_lay, t_lay, mu, dr, nu):
    """Cloud optical depth dtau[l, nu] = q_l rho_l dr_l 3 Q(nu) / (4 r_eff) (Eq. 23)."""
    q_lay = condensate_profile(wl, cp, p_lev, p_lay)
    q_nu, r = extinction_efficiency(wl, cp, nu)
    rho = mu * M_U * p_lay / (K_B * t_lay)
    col = q_lay * rho * dr * 0.75 / r
    return col[:, None] * q_nu[None, :]


def layer_optical_depth(wl, t_lay, p_lev, p_lay, r_lev, x, x_h2, x_he, mu, log10_pc=None,
                        tables=None):
    """Vertical optical depth of every layer, dtau[l, nu] = kappa_l(nu) dr_l.

    kappa_l = n_l sum_s X_s sigma_s(T_l, p_l)                     (line tables)
            + n_l (X_H2 sigma_R,H2 + X_He sigma_R,He)             (Rayleigh)
            + n_l^2 (X_H2^2 k_H2H2 + X_H2 X_He k_H2He)            (CIA)
            + kappa_c rho_l f_l                                   (grey deck)
    with n_l = p_l/(k_B T_l) and rho_l = mu m_u n_l.  The line and CIA
    sources are the paper's gas opacities (Section "Gas phase opacities" and
    the WASP-17b setup); the grey deck is the slab cloud (Eq. 18, 23) in the
    geometric-optics limit.
    """
    xs_tab, cia_tab = (wl["log10_xsec"], wl["log10_cia"]) if tables is None else tables
    nu = wl["nu"]
    n_lay = len(t_lay)
    dr = r_lev[1:] - r_lev[:-1]
    logp_bar = np.log10(p_lay / BAR)
    nu4 = (nu / 1.0e4) ** 4
    emission = wl["mode"] == 1
    out = np.empty((n_lay, len(nu)), dtype=np.result_type(t_lay, r_lev, x, mu))
    for l in range(n_lay):
        n_l = p_lay[l] / (K_B * t_lay[l])
        kap = np.zeros(len(nu), dtype=out.dtype)
        for s in range(len(x)):
            v = bilinear_log_table(xs_tab[s], wl["t_grid"], wl["logp_grid"], t_lay[l], logp_bar[l])
            kap = kap + n_l * x[s] * np.exp(v * np.log(10.0))
        if cia_tab is not None and wl["cia"]:
            k1 = np.exp(cia_log(cia_tab[0], wl["tc_grid"], t_lay[l]) * np.log(10.0))
            k2 = np.exp(cia_log(cia_tab[1], wl["tc_grid"], t_lay[l]) * np.log(10.0))
            kap = kap + n_l * n_l * (x_h2 * x_h2 * k1 + x_h2 * x_he * k2)
        if wl["rayleigh"] and not emission:
            kap = kap + n_l * (x_h2 * wl["ray_h2"] + x_he * wl["ray_he"]) * nu4
        if wl["cloud"] and not emission and wl.get("cloud_model", CLOUD_GREY_DECK) == CLOUD_GREY_DECK:
            f = cloud_fraction(p_lev[l], p_lev[l + 1], 10.0 ** log10_pc * BAR)
            kap = kap + wl["kappa_cloud"] * mu * M_U * n_l * f
        out[l] = kap * dr[l]
    if wl["cloud"] and not emission and wl.get("cloud_model", CLOUD_GREY_DECK) == CLOUD_NONGREY:
        out = out + nongrey_cloud_dtau(wl, log10_pc, p_lev, p_lay, t_lay, mu, dr, nu)
    return out


# ---------------------------------------------------------------------------
# a4, a6, a7: transmission
def path_matrix(r_lev):
    """Slant path matrix P_1D (Eq. 43).

    Rows i are impact parameters b_i = (r_i + r_{i+1})/2 (layer mid radii),
    columns l are layers with lower/upper radii r_l, r_{l+1}:
      0                                                 if r_{l+1} <= b_i
      (2/dr_l) sqrt(r_{l+1}^2 - b_i^2)                  if r_l < b_i < r_{l+1}
      (2/dr_l) (sqrt(r_{l+1}^2 - b_i^2) - sqrt(r_l^2 - b_i^2))   if r_l >= b_i
    """
    n = len(r_lev) - 1
    b = 0.5 * (r_lev[:-1] + r_lev[1:])
    pm = np.zeros((n, n), dtype=r_lev.dtype)
    for i in range(n):
        for l in range(n):
            r_lo, r_up = r_lev[l], r_lev[l + 1]
            dr = r_up - r_lo
            if _re(r_up) <= _re(b[i]):
                continue
            if _re(r_lo) < _re(b[i]):
                pm[i, l] = 2.0 / dr * np.sqrt(r_up ** 2 - b[i] ** 2)
            else:
                pm[i, l] = 2.0 / dr * (np.sqrt(r_up ** 2 - b[i] ** 2) - np.sqrt(r_lo ** 2 - b[i] ** 2))
    return pm


def transit_depth(pm, dtau, r_lev, r_s):
    """Transit depth from the slant optical depth tau = P . dtau (Eq. 44).

    The paper cites the transmission equation without printing it.  Reading:
    an opaque disc of radius r_0 plus annuli between consecutive levels, each
    with the transmission of its mid-radius chord:
        delta = [r_0^2 + sum_i (r_{i+1}^2 - r_i^2)(1 - exp(-tau_i))] / R_s^2.
    """
    tau = pm @ dtau
    area = r_lev[1:] ** 2 - r_lev[:-1] ** 2
    return (r_lev[0] ** 2 + area @ (1.0 - np.exp(-tau))) / r_s ** 2


# ---------------------------------------------------------------------------
# a7': emission
def planck(t, nu):
    """Planck intensity per unit wavenumber, 2 h c^2 nu^3 / (exp(h c nu / k T) - 1)."""
    return 2.0 * H_PL * C_LIGHT ** 2 * nu ** 3 / np.expm1(H_PL * C_LIGHT * nu / (K_B * t))


def gauss_legendre_01(n):
    """n-point Gauss-Legendre nodes and weights mapped to mu in [0, 1]."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def _lin_source_factor(x):
    """(1 - e^-x)/x - e^-x, with its Taylor series below 1e-4."""
    small = _re(x) < 1.0e-4
    xs = np.where(small, 1.0, x)
    full = -np.expm1(-xs) / xs - np.exp(-xs)
    series = x / 2.0 - x ** 2 / 3.0 + x ** 3 / 8.0 - x ** 4 / 30.0
    return np.where(small, series, full)


def emission_intensity(dtau, b_lev, mu):
    """Upward intensity at the top for one angle, pure absorption.

    Linear-in-tau source in every layer (the paper's emission scheme without
    scattering): going up through layer l with x = dtau_l / mu,
      I <- I e^-x + B_top (1 - e^-x) + (B_bot - B_top) [(1 - e^-x)/x - e^-x],
    starting from I = B(T_0) at the bottom level.
    """
    i_nu = b_lev[0].copy()
    for l in range(dtau.shape[0]):
        x = dtau[l] / mu
        e = np.exp(-x)
        # 1 - e^-x as -expm1(-x): a thin hot layer's emission is B (1 - e^-x)
        i_nu = i_nu * e - b_lev[l + 1] * np.expm1(-x) + (b_lev[l] - b_lev[l + 1]) * _lin_source_factor(x)
    return i_nu


def toa_flux(dtau, t_lev, nu, n_mu):
    """Outgoing flux at the top of the atmosphere, F_toa = 2 pi sum_k w_k mu_k I_k."""
    b_lev = np.stack([planck(t, nu) for t in t_lev])
    mus, ws = gauss_legendre_01(n_mu)
    flux = 0.0
    for mu_k, w_k in zip(mus, ws):
        flux = flux + 2.0 * np.pi * w_k * mu_k * emission_intensity(dtau, b_lev, mu_k)
    return flux


def emission_ratio(dtau, t_lev, nu, r_p, r_s, t_star, n_mu, dilution):
    """F_p / F_* = s F_toa / F_* (R_p/R_*)^2 (Eq. 45), F_* = pi B(T_*)."""
    return dilution * toa_flux(dtau, t_lev, nu, n_mu) / (np.pi * planck(t_star, nu)) * (r_p / r_s) ** 2


def brown_dwarf_radius(m_bd_mjup, g):
    """R_bd = sqrt(G M_bd / g) (Eq. 47), M_bd in Jupiter masses, g in cm s^-2."""
    return np.sqrt(G_GRAV * m_bd_mjup * M_JUP / g)


def brown_dwarf_flux(dtau, t_lev, nu, r_bd, distance, n_mu, dilution):
    """Flux of an isolated object at the observer, F_bd = s F_toa (R_bd/D)^2 (Eq. 46)
    [erg s^-1 cm^-2 (cm^-1)^-1]."""
    return dilution * toa_flux(dtau, t_lev, nu, n_mu) * (r_bd / distance) ** 2


# ---------------------------------------------------------------------------
# a8: binning and likelihood
def bin_means(y, lo, hi, offset_ppm, mask):
    """Box-car mean over native points [lo_k, hi_k) plus an additive offset
    (ppm) on masked bins (the paper's instrument offset)."""
    m = np.array([np.mean(y[a:b]) for a, b in zip(lo, hi)])
    return m + offset_ppm * 1.0e-6 * mask


def log_likelihood(y_obs, model, sigma, err_c=-99.0):
    """Independent-Gaussian log-likelihood (Eq. 1-3), natural logarithms,
    sigma_eff^2 = sigma^2 + 10^(2c)."""
    s_eff = np.sqrt(sigma ** 2 + 10.0 ** (2.0 * err_c))
    r = y_obs - model
    return np.sum(-np.log(s_eff) - 0.5 * np.log(2.0 * np.pi) - 0.5 * (r / s_eff) ** 2)


# ---------------------------------------------------------------------------
def split_params(wl, theta):
    """Split a parameter vector by the workload's layout."""
    k = 0
    ntp = wl.get("n_knots", 5) if wl["tp"] == TP_PCHIP else TP_NPARAM[wl["tp"]]
    out = {"tp": theta[k:k + ntp]}
    k += ntp
    out["logx"] = theta[k:k + wl["n_species"]]
    k += wl["n_species"]
    if wl["cloud"] and wl.get("cloud_model", CLOUD_GREY_DECK) == CLOUD_NONGREY:
        # non-grey cloud: the whole group travels under "log10_pc" to the opacity
        n_c = nongrey_param_count(wl)
        g = theta[k:k + n_c]
        j = 0
        cp = {}
        if wl["cloud_qext"] == QEXT_GREY:
            cp["r"] = g[0]
            j = 1
        else:
            cp["r"], cp["a"], cp["q0"] = g[0], g[1], g[2]
            j = 3
        nq = 1 if wl["cloud_profile"] == QPROF_UNIFORM else 3
        cp["q"] = g[j:j + nq]
        j += nq
        if wl["cloud_qext"] == QEXT_FIT_FEATURE:
            cp["feat"] = g[j:j + 4]
        out["log10_pc"] = cp
        k += n_c
    else:
        out["log10_pc"] = theta[k] if wl["cloud"] else None
        k += int(wl["cloud"])
    fc = bool(wl.get("fcld", False))
    out["fcld"] = theta[k] if fc else 1.0
    k += int(fc)
    bd = bool(wl.get("bd", False))
    out["log10_g"], out["m_bd"] = (theta[k], theta[k + 1]) if bd else (None, None)
    k += 2 * int(bd)
    out["scale"] = theta[k] if wl["scale"] else 1.0
    k += int(wl["scale"])
    out["offset"] = theta[k] if wl["offset"] else 0.0
    k += int(wl["offset"])
    if k != len(theta):
        raise ValueError(f"expected {k} parameters, got {len(theta)}")
    return out


def decode_tables(wl, wide=None):
    """The tables as the reduced-precision path stores them, decoded to FP64.

    Storage rule of the reduced-precision path: per species (or CIA pair) and
    wavenumber, c = float32((min + max)/2) of log2 sigma over the (T, p) grid;
    each entry is float16(log2 sigma - c).  Emission stores each entry as
    float32(log2 sigma - c) instead (``wide``, by default for emission
    workloads).  The decoded value is (c + entry) / log2(10) in log10 units, so
    forward(..., tables=...) isolates the storage error from the arithmetic error.
    """
    if wide is None:
        wide = wl["mode"] == 1
    store = np.float32 if wide else np.float16

    def dec(tab, axes):
        l2 = tab * np.log2(10.0)
        c = (0.5 * (l2.min(axis=axes, keepdims=True) + l2.max(axis=axes, keepdims=True))).astype(np.float32)
        v = l2 - c.astype(np.float64)
        h = v.astype(store).astype(np.float64)
        return (c.astype(np.float64) + h) / np.log2(10.0)
    xs = dec(wl["log10_xsec"], (1, 2))
    cia = dec(wl["log10_cia"], (1,)) if wl["log10_cia"] is not None else None
    return xs, cia


def forward(wl, theta, n_layers=None, tables=None, want_internals=False):
    """One sample through the whole path: T-p, chemistry, altitudes, opacity,
    chord (or emission), binning and log-likelihood.

    Returns dict(spectrum, binned, lnL, status[, internals]).  An invalid
    sample returns lnL = -1e300 and a NaN spectrum (Section "Likelihood").
    """
    theta = np.asarray(theta)
    n_lay = wl["n_layers"] if n_layers is None else int(n_layers)
    nan = np.full(len(wl["nu"]), np.nan)
    bad = {"spectrum": nan, "binned": np.full(len(wl["bin_lo"]), np.nan), "lnL": INVALID_LNL}
    if n_lay < 1 or n_lay > wl["n_layers"]:
        return dict(bad, status=S_BAD_LAYERS)
    if not np.all(np.isfinite(_re(theta))):
        return dict(bad, status=S_NONFINITE)
    ps = split_params(wl, theta)
    # an isolated object (Eqs. 46-47) retrieves its gravity and mass
    bd = bool(wl.get("bd", False))
    g_ref = 10.0 ** ps["log10_g"] if bd else wl["g_ref"]
    p_lev, p_lay = level_pressures(wl["p_bot"], wl["p_top"], n_lay)
    t_lay = tp_profile(wl, ps["tp"], p_lay, g_ref)
    t_lev = tp_profile(wl, ps["tp"], p_lev, g_ref) if wl["mode"] == 1 else None
    status = 0
    tt = _re(t_lay) if t_lev is None else np.concatenate([_re(t_lay), _re(t_lev)])
    if not np.all(np.isfinite(tt)) or np.any(tt <= 0.0):
        status |= S_BAD_T
    x, x_h2, x_he, mu, ok = chemistry(ps["logx"], wl["species_mass"], wl["mu_fixed"])
    if not ok:
        status |= S_BAD_VMR
    if status:
        return dict(bad, status=status)
    r_ref = brown_dwarf_radius(ps["m_bd"], g_ref) if bd else wl["r_p"] * ps["scale"]
    r_lev, ok = altitudes(t_lay, p_lev, mu, g_ref, r_ref, wl["p_ref_bar"] * BAR,
                          constant_g=wl.get("constant_g", False))
    if not ok:
        return dict(bad, status=S_UNBOUND)
    if wl.get("ck", False):
        # correlated-k tables: the spectrum is per bin, the native points of the binning
        from . import ck
        internals = dict(t_lay=t_lay, t_lev=t_lev, r_lev=r_lev, x=x, x_h2=x_h2, x_he=x_he, mu=mu,
                         p_lev=p_lev, p_lay=p_lay, r_ref=r_ref)
        spec = ck.spectrum(wl, internals, ps["log10_pc"])
        dtau = None
    else:
        dtau = layer_optical_depth(wl, t_lay, p_lev, p_lay, r_lev, x, x_h2, x_he, mu,
                                   ps["log10_pc"], tables=tables)
    if wl.get("ck", False):
        pass
    elif wl["mode"] == 0:
        pm = path_matrix(r_lev)
        spec = transit_depth(pm, dtau, r_lev, wl["r_s"])
        if wl.get("fcld", False):
            # Eq. 26: a fraction f_cld of the limb is cloudy, the rest clear
            dtau_cf = layer_optical_depth(dict(wl, cloud=False), t_lay, p_lev, p_lay, r_lev, x, x_h2, x_he, mu,
                                          None, tables=tables)
            spec_cf = transit_depth(pm, dtau_cf, r_lev, wl["r_s"])
            spec = ps["fcld"] * spec + (1.0 - ps["fcld"]) * spec_cf
    elif bd:
        spec = brown_dwarf_flux(dtau, t_lev, wl["nu"], r_ref, wl["bd_distance"], wl["n_mu"], wl["dilution"])
    else:
        spec = emission_ratio(dtau, t_lev, wl["nu"], r_ref, wl["r_s"], wl["t_star"],
                              wl["n_mu"], wl["dilution"])
    if not np.all(np.isfinite(_re(spec))):
        return dict(bad, status=S_NONFINITE)
    m = bin_means(spec, wl["bin_lo"], wl["bin_hi"], ps["offset"], wl["offset_mask"])
    lnl = log_likelihood(wl["y_obs"], m, wl["y_err"], wl["err_c"])
    out = {"spectrum": spec, "binned": m, "lnL": lnl, "status": 0}
    if want_internals:
        out["internals"] = dict(t_lay=t_lay, t_lev=t_lev, r_lev=r_lev, dtau=dtau, mu=mu,
                                x=x, x_h2=x_h2, x_he=x_he, p_lev=p_lev, p_lay=p_lay)
    return out
