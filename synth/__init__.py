"""Seeded synthetic workloads for the batched atmospheric forward model.

This module only *generates inputs*: spectral grids, line-list cross-section
tables, collision-induced-absorption (CIA) tables, Rayleigh coefficients,
bins, observational errors and parameter draws.  It holds none of the forward
model's arithmetic (no profiles, hydrostatics, interpolation, radiative
transfer or likelihood); both the FP64 oracle and the HIP library consume
exactly the arrays produced here.

The workloads stand in for the paper's opacity-sampled HELIOS-k tables and
HST/JWST spectra (Section "Gas phase opacities" and Table 2), which are not
available; their shapes follow those workloads: 100 layers, tens of thousands
of wavenumbers, 4-8 absorbers, 10-13 parameters.

Configurations (ids 0-6); config 1 at B = 1024 is the headline transmission batch:

* 0 -- plain transmission, one sample, isothermal, one absorber, 2000 nu.
* 1 -- JWST-like transmission, 6 absorbers x 20 T x 20 log p x 30000 nu,
       reduced Guillot profile, CIA, Rayleigh, grey cloud, 400 ln-lambda bins.
* 2 -- emission, 8 absorbers, 20000 nu (1-12 um), 5 PCHIP knot temperatures.
* 3 -- transmission setup of 1, used for gradients (B=128).
* 4 -- high-resolution transmission, 4 absorbers x 8 x 8 x 400000 nu,
       per-sample layer counts 60-150.
* 5 -- the setup of 1 with a non-grey cloud (power-law condensate, fitted Q_ext
       with the mid-infrared feature).
* 6 -- the setup of 1 with a partly cloudy limb (non-grey slab cloud, cloudy fraction).
* 7 -- correlated-k transmission: the species of 1 as k-tables on R = 1000 bins
       (0.6-5.3 um, 2178 bins) with 8 g-points, mixed by random overlap.
* 8 -- correlated-k emission: the species of 2 as k-tables on R = 1000 bins
       (1-12 um, 2485 bins) with 8 g-points, mixed by random overlap with
       resorting and rebinning.

Every random stream is ``numpy.random.default_rng([19687, cid, stream])``.
"""
from __future__ import annotations

import functools
import os

import numpy as np

# ----------------------------------------------------------------------------
# physical constants the generators need (cgs); the model's own constants live
# separately in the oracle and in the C library
BAR = 1.0e6            # dyn cm^-2
R_JUP = 7.1492e9       # cm
R_SUN = 6.957e10       # cm

# species order of the paper's opacity list (Section "Gas phase opacities")
# with molecular masses in atomic mass units
SPECIES = ("H2O", "CO2", "CO", "CH4", "NH3", "H2S", "SO2", "Na")
SPECIES_MASS = (18.015, 44.009, 28.010, 16.043, 17.031, 34.081, 64.066, 22.990)

TP_ISOTHERMAL = 0
TP_GUILLOT3 = 1
TP_PCHIP = 2
TP_BARSTOW = 3
TP_MILNE = 4
TP_GUILLOT7 = 5

MODE_TRANSMISSION = 0
MODE_EMISSION = 1

STREAM_LINES = 1
STREAM_CIA = 2
STREAM_PARAMS = 3
STREAM_NOISE = 4
STREAM_TRUTH = 5
STREAM_LAYERS = 6

_DATA_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")


def _rng(cid: int, stream: int, sub: int = 0) -> np.random.Generator:
    return np.random.default_rng([19687, int(cid), int(stream), int(sub)])


# ----------------------------------------------------------------------------
# line-list cross sections
def line_list(cid: int, species: int, n_lines: int, nu_min: float, nu_max: float):
    """Seeded line list: uniform centres, log-normal strengths.

    log10 S ~ N(-21, 1.5) [cm^-1 / (molecule cm^-2)]; centres ~ U(nu_min, nu_max).
    """
    g = _rng(cid, STREAM_LINES, species)
    centres = g.uniform(nu_min, nu_max, n_lines)
    log_s = g.normal(-21.0, 1.5, n_lines)
    return centres, 10.0 ** log_s


def lorentz_log10_xsec(nu, t_grid, logp_grid, centres, strengths, gamma0=0.07,
                       cutoff=25.0, continuum=1.0e-24):
    """log10 cross section [cm^2] on a (T, log10 p[bar], nu) grid.

    sigma(nu; T, p) = continuum + sum_j S_j (g/pi) / ((nu - c_j)^2 + g^2), with
    the Lorentz half width g = gamma0 (p / 1 bar) (T / 296 K)^-0.5 shared by all
    lines and each line truncated at ``cutoff`` cm^-1 from its centre.  The
    strengths do not depend on T.
    """
    nu = np.asarray(nu, dtype=np.float64)
    n = nu.size
    dnu = (nu[-1] - nu[0]) / (n - 1)
    width = int(np.ceil(2.0 * cutoff / dnu)) + 2
    i0 = np.ceil((centres - cutoff - nu[0]) / dnu).astype(np.int64)
    idx = i0[:, None] + np.arange(width)[None, :]
    inside = (idx >= 0) & (idx < n)
    idxc = np.clip(idx, 0, n - 1)
    d2 = (nu[idxc] - centres[:, None]) ** 2
    inside &= d2 <= cutoff * cutoff
    flat_idx = idxc[inside]
    d2_in = d2[inside]
    s_in = np.broadcast_to(strengths[:, None], idx.shape)[inside]
    out = np.empty((len(t_grid), len(logp_grid), n), dtype=np.float64)
    for it, t in enumerate(t_grid):
        for ip, lp in enumerate(logp_grid):
            g = gamma0 * (10.0 ** lp) * (t / 296.0) ** -0.5
            prof = s_in * (g / np.pi) / (d2_in + g * g)
            sig = continuum + np.bincount(flat_idx, weights=prof, minlength=n)
            out[it, ip] = np.log10(sig)
    return out


def cia_log10(cid: int, pair: int, nu, tc_grid, n_bands=4):
    """Smooth seeded CIA band model log10 k(T, nu) [cm^5].

    k = sum_g A_g exp(-(nu - c_g)^2 / (2 w_g^2)) (T / 1000 K)^beta_g + 1e-50,
    log10 A ~ U[-46, -44], w ~ U[200, 1500] cm^-1, beta ~ U[-1, 1],
    c ~ U(nu range).
    """
    g = _rng(cid, STREAM_CIA, pair)
    log_a = g.uniform(-46.0, -44.0, n_bands)
    w = g.uniform(200.0, 1500.0, n_bands)
    beta = g.uniform(-1.0, 1.0, n_bands)
    c = g.uniform(nu[0], nu[-1], n_bands)
    out = np.empty((len(tc_grid), len(nu)), dtype=np.float64)
    for it, t in enumerate(tc_grid):
        k = np.full(len(nu), 1.0e-50)
        for b in range(n_bands):
            k += 10.0 ** log_a[b] * np.exp(-0.5 * ((nu - c[b]) / w[b]) ** 2) * (t / 1000.0) ** beta[b]
        out[it] = np.log10(k)
    return out


def ln_lambda_bins(nu, n_bins):
    """Contiguous native-index bins [lo_k, hi_k) uniform in ln(nu) (= ln lambda).

    Bins are ordered by ascending nu and together cover every native point.
    """
    nu = np.asarray(nu)
    edges = np.exp(np.linspace(np.log(nu[0]), np.log(nu[-1]), n_bins + 1))
    lo = np.searchsorted(nu, edges[:-1], side="left")
    hi = np.searchsorted(nu, edges[1:], side="left")
    hi[-1] = len(nu)
    lo[0] = 0
    if np.any(hi <= lo):
        raise ValueError("empty bin; use fewer bins")
    return lo.astype(np.int32), hi.astype(np.int32)


# ----------------------------------------------------------------------------
# correlated-k tables (the same line lists, summarised per spectral bin)
def ck_bin_edges(nu_min: float, nu_max: float, resolution: float) -> np.ndarray:
    """Bin edges uniform in ln(nu) with nu/dnu = resolution: [n_bins + 1] ascending."""
    n = int(round(np.log(nu_max / nu_min) * resolution))
    return np.exp(np.linspace(np.log(nu_min), np.log(nu_max), n + 1))


def ck_g_quadrature(n_lo: int = 4, n_hi: int = 4, g_split: float = 0.9):
    """g-points and weights on [0, 1]: Gauss-Legendre rules of n_lo points on
    [0, g_split] and n_hi points on [g_split, 1] (the strong-absorption tail
    gets its own points).  Weights sum to 1; nodes ascend."""
    x1, w1 = np.polynomial.legendre.leggauss(n_lo)
    x2, w2 = np.polynomial.legendre.leggauss(n_hi)
    g = np.concatenate([0.5 * g_split * (x1 + 1.0), g_split + 0.5 * (1.0 - g_split) * (x2 + 1.0)])
    w = np.concatenate([0.5 * g_split * w1, 0.5 * (1.0 - g_split) * w2])
    return g, w


def ck_sub_grid(edges: np.ndarray, n_sub: int) -> np.ndarray:
    """n_sub midpoints of equal sub-intervals in every bin: [n_bins, n_sub]."""
    lo, hi = edges[:-1], edges[1:]
    f = (np.arange(n_sub) + 0.5) / n_sub
    return lo[:, None] + (hi - lo)[:, None] * f[None, :]


def lorentz_pairs(nu, centres, strengths, cutoff=25.0):
    """(point index, squared distance, strength) of every (line, point) pair within
    ``cutoff`` cm^-1, at arbitrary ascending nu."""
    lo = np.searchsorted(nu, centres - cutoff, side="left")
    hi = np.searchsorted(nu, centres + cutoff, side="right")
    cnt = hi - lo
    tot = int(cnt.sum())
    start = np.repeat(lo, cnt)
    offs = np.arange(tot) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    idx = start + offs
    line = np.repeat(np.arange(len(centres)), cnt)
    return idx, (nu[idx] - centres[line]) ** 2, strengths[line]


def lorentz_sigma_nonuniform(nu, gamma, centres, strengths, cutoff=25.0, continuum=1.0e-24, pairs=None):
    """sigma(nu) [cm^2] at arbitrary ascending nu for one Lorentz half width
    gamma (the line shape of ``lorentz_log10_xsec``, same cutoff and continuum)."""
    idx, d2, s = lorentz_pairs(nu, centres, strengths, cutoff) if pairs is None else pairs
    prof = s * (gamma / np.pi) / (d2 + gamma * gamma)
    return continuum + np.bincount(idx, weights=prof, minlength=len(nu))


def ck_log10_table(sub_nu, g_nodes, t_grid, logp_grid, centres, strengths, gamma0=0.07):
    """log10 k(g) [cm^2] per (T, log10 p[bar], bin, g-point) from the sub-grid
    cross sections: within each bin the n_sub values are sorted ascending (the
    k-distribution as a function of g, each value standing for a sub-interval of
    width 1/n_sub centred at (i + 1/2)/n_sub) and read at the g-nodes by linear
    interpolation (held constant outside the first and last centres)."""
    n_bins, n_sub = sub_nu.shape
    flat = sub_nu.ravel()
    pairs = lorentz_pairs(flat, centres, strengths)
    out = np.empty((len(t_grid), len(logp_grid), n_bins, len(g_nodes)))
    for it, t in enumerate(t_grid):
        for ip, lp in enumerate(logp_grid):
            gam = gamma0 * (10.0 ** lp) * (t / 296.0) ** -0.5
            sig = np.sort(lorentz_sigma_nonuniform(flat, gam, centres, strengths, pairs=pairs).reshape(n_bins, n_sub),
                          axis=1)
            k = np.empty((n_bins, len(g_nodes)))
            for n, gn in enumerate(g_nodes):
                pos = np.clip(gn * n_sub - 0.5, 0.0, n_sub - 1.0)
                i0 = np.minimum(np.floor(pos).astype(int), n_sub - 2)
                fr = pos - i0
                k[:, n] = (1.0 - fr) * sig[:, i0] + fr * sig[:, i0 + 1]
            out[it, ip] = np.log10(k)
    return out


# ----------------------------------------------------------------------------
# configuration descriptions
_BASE = dict(
    p_ref_bar=10.0,          # reference pressure of the altitude grid
    r_p=R_JUP,               # planet reference radius [cm]
    r_s=R_SUN,               # stellar radius [cm]
    g_ref=1000.0,            # gravity at the reference radius [cm s^-2]
    kappa_ir=1.0e-2,         # Guillot infrared opacity [cm^2 g^-1]
    f_hem=0.25,              # hemispheric redistribution factor
    kappa_cloud=60.0,        # grey deck opacity [cm^2 g^-1]: 3 q Q/(4 rho_d r) with q=1e-2, Q=2, rho_d=2.5, r=1 um
    t_star=5500.0,           # stellar blackbody temperature [K] (emission)
    dilution=1.0,            # emission dilution factor s
    err_c=-99.0,             # error inflation exponent c (off)
    ray_h2=8.0e-29,          # H2 Rayleigh cross section at 1e4 cm^-1 [cm^2], scales as nu^4
    ray_he=6.0e-30,          # He Rayleigh cross section at 1e4 cm^-1 [cm^2]
    n_mu=4,                  # Gauss-Legendre angles (emission)
    cloud_model=0,           # 0: grey deck (log10 P_cloud); 1: non-grey (profile + Q_ext)
    cloud_profile=0,         # non-grey q_c(p): 0 uniform, 1 slab, 2 base + power law
    cloud_qext=0,            # non-grey Q_ext: 0 fit, 1 fit + mid-IR feature, 2 grey Q = 2
    fcld=False,              # cloudy fraction f_cld of the limb (Eq. 26) as a parameter
    bd=False,                # isolated object (emission): log10 g and M_bd retrieved, flux at distance bd_distance
    bd_distance=10.0 * 3.0856775814913673e18,   # [cm], 10 pc
    sigma_ppm=50.0,          # observational error per bin [ppm]
)

CONFIGS = {
    0: dict(mode=MODE_TRANSMISSION, tp=TP_ISOTHERMAL, n_layers=50, p_bot=100.0, p_top=1.0e-6,
            n_species=1, n_nu=2000, nu_min=2000.0, nu_max=10000.0,
            t_grid=np.linspace(500.0, 2500.0, 8), logp_grid=np.linspace(-6.0, 2.0, 8),
            n_lines=300, cia=False, rayleigh=True, cloud=False, scale=False, offset=False,
            mu_fixed=2.3, n_bins=100, batch=1),
    1: dict(mode=MODE_TRANSMISSION, tp=TP_GUILLOT3, n_layers=100, p_bot=100.0, p_top=1.0e-7,
            n_species=6, n_nu=30000, nu_min=1.0e4 / 5.3, nu_max=1.0e4 / 0.6,
            t_grid=np.linspace(300.0, 3500.0, 20), logp_grid=np.linspace(-7.0, 2.0, 20),
            n_lines=2000, cia=True, rayleigh=True, cloud=True, scale=True, offset=True,
            mu_fixed=0.0, n_bins=400, batch=256),
    2: dict(mode=MODE_EMISSION, tp=TP_PCHIP, n_layers=100, p_bot=100.0, p_top=1.0e-7,
            n_species=8, n_nu=20000, nu_min=1.0e4 / 12.0, nu_max=1.0e4 / 1.0,
            t_grid=np.linspace(300.0, 3500.0, 20), logp_grid=np.linspace(-7.0, 2.0, 20),
            n_lines=2000, cia=True, rayleigh=False, cloud=False, scale=False, offset=False,
            mu_fixed=0.0, n_bins=400, batch=1024, n_knots=5),
    3: dict(mode=MODE_TRANSMISSION, tp=TP_GUILLOT3, n_layers=100, p_bot=100.0, p_top=1.0e-7,
            n_species=6, n_nu=30000, nu_min=1.0e4 / 5.3, nu_max=1.0e4 / 0.6,
            t_grid=np.linspace(300.0, 3500.0, 20), logp_grid=np.linspace(-7.0, 2.0, 20),
            n_lines=2000, cia=True, rayleigh=True, cloud=True, scale=True, offset=True,
            mu_fixed=0.0, n_bins=400, batch=128),
    4: dict(mode=MODE_TRANSMISSION, tp=TP_GUILLOT3, n_layers=150, p_bot=100.0, p_top=1.0e-7,
            n_species=4, n_nu=400000, nu_min=1.0e4 / 2.5, nu_max=1.0e4 / 0.95,
            t_grid=np.linspace(300.0, 3500.0, 8), logp_grid=np.linspace(-7.0, 2.0, 8),
            n_lines=2000, cia=True, rayleigh=True, cloud=True, scale=True, offset=True,
            mu_fixed=0.0, n_bins=400, batch=64, ragged=(60, 150)),
    # the transmission setup of 1 with a non-grey cloud: power-law condensate profile
    # and the fitted extinction efficiency with a mid-infrared feature
    5: dict(mode=MODE_TRANSMISSION, tp=TP_GUILLOT3, n_layers=100, p_bot=100.0, p_top=1.0e-7,
            n_species=6, n_nu=30000, nu_min=1.0e4 / 5.3, nu_max=1.0e4 / 0.6,
            t_grid=np.linspace(300.0, 3500.0, 20), logp_grid=np.linspace(-7.0, 2.0, 20),
            n_lines=2000, cia=True, rayleigh=True, cloud=True, scale=True, offset=True,
            mu_fixed=0.0, n_bins=400, batch=128, cloud_model=1, cloud_profile=2, cloud_qext=1),
    # 5 with a partly cloudy limb (Eq. 26): a slab profile and the fitted Q_ext
    6: dict(mode=MODE_TRANSMISSION, tp=TP_GUILLOT3, n_layers=100, p_bot=100.0, p_top=1.0e-7,
            n_species=6, n_nu=30000, nu_min=1.0e4 / 5.3, nu_max=1.0e4 / 0.6,
            t_grid=np.linspace(300.0, 3500.0, 20), logp_grid=np.linspace(-7.0, 2.0, 20),
            n_lines=2000, cia=True, rayleigh=True, cloud=True, scale=True, offset=True,
            mu_fixed=0.0, n_bins=400, batch=128, cloud_model=1, cloud_profile=1, cloud_qext=0, fcld=True),
    # correlated-k transmission: the six species of 1 (same line lists) as k-tables on
    # R = 1000 bins of 16 sub-points, 8 g-points; random overlap of the species
    # (ck_mix 1: product of the species' transmission functions; 0: RORR)
    7: dict(mode=MODE_TRANSMISSION, tp=TP_GUILLOT3, n_layers=100, p_bot=100.0, p_top=1.0e-7,
            n_species=6, nu_min=1.0e4 / 5.3, nu_max=1.0e4 / 0.6, ck_resolution=1000.0, ck_sub=16,
            t_grid=np.linspace(300.0, 3500.0, 20), logp_grid=np.linspace(-7.0, 2.0, 20),
            n_lines=2000, cia=True, rayleigh=True, cloud=True, scale=True, offset=True,
            mu_fixed=0.0, n_bins=400, batch=256, ck=True, ck_mix=1),
    # correlated-k emission: the eight species of 2 on R = 1000 bins, mixed by random
    # overlap with resorting and rebinning
    8: dict(mode=MODE_EMISSION, tp=TP_PCHIP, n_layers=100, p_bot=100.0, p_top=1.0e-7,
            n_species=8, nu_min=1.0e4 / 12.0, nu_max=1.0e4 / 1.0, ck_resolution=1000.0, ck_sub=16,
            t_grid=np.linspace(300.0, 3500.0, 20), logp_grid=np.linspace(-7.0, 2.0, 20),
            n_lines=2000, cia=True, rayleigh=False, cloud=False, scale=False, offset=False,
            mu_fixed=0.0, n_bins=400, batch=256, n_knots=5, ck=True, ck_mix=0),
}

CK_MIX_RORR = 0       # random overlap with resorting and rebinning, layer by layer
CK_MIX_PRODUCT = 1    # transmission: product of the species' chord transmission functions

# configs 1, 3, 5 and 6 share tables (same seeds) with the headline batch; the
# correlated-k configs summarise the line lists of 1 and 2
_TABLE_CID = {0: 0, 1: 1, 2: 2, 3: 1, 4: 4, 5: 1, 6: 1, 7: 1, 8: 2}


def param_names(cfg) -> list:
    s = cfg["n_species"]
    if cfg["tp"] == TP_ISOTHERMAL:
        names = ["T_iso"]
    elif cfg["tp"] == TP_GUILLOT3:
        names = ["T_int", "T_eq", "log10_gamma_v"]
    elif cfg["tp"] == TP_BARSTOW:
        names = ["T_strat"]
    elif cfg["tp"] == TP_MILNE:
        names = ["T_int", "log10_kappa_ir", "T_ratio", "log10_p_t_bar", "beta"]
    elif cfg["tp"] == TP_GUILLOT7:
        names = ["T_int", "T_eq", "log10_kappa_ir", "log10_gamma_v", "q_irr0", "log10_p_t_bar", "beta"]
    else:
        names = [f"T_knot{k}" for k in range(cfg["n_knots"])]
    names += [f"log10_X_{SPECIES[i]}" for i in range(s)]
    if cfg["cloud"] and cfg.get("cloud_model", 0) == 1:
        names += ["log10_r_eff_um"] + ([] if cfg["cloud_qext"] == 2 else ["a_slope", "log10_Q0"])
        names += [["log10_q"], ["log10_q", "log10_p_top_bar", "log10_dp_bar"],
                  ["log10_q_base", "log10_p_base_bar", "alpha"]][cfg["cloud_profile"]]
        if cfg["cloud_qext"] == 1:
            names += ["feature_A", "feature_lambda0_um", "log10_feature_width_um", "feature_skew"]
    elif cfg["cloud"]:
        names.append("log10_P_cloud_bar")
    if cfg.get("fcld", False):
        names.append("f_cld")
    if cfg.get("bd", False):
        names += ["log10_g_cgs", "M_bd_MJup"]
    if cfg["scale"]:
        names.append("R_p_scale")
    if cfg["offset"]:
        names.append("offset_ppm")
    return names


def param_bounds(cfg):
    """Uniform prior bounds, one (lo, hi) pair per parameter."""
    s = cfg["n_species"]
    if cfg["tp"] == TP_ISOTHERMAL:
        b = [(1200.0, 1200.0)]
    elif cfg["tp"] == TP_GUILLOT3:
        b = [(100.0, 1500.0), (500.0, 2000.0), (-3.0, 2.0)]
    elif cfg["tp"] == TP_BARSTOW:
        b = [(600.0, 2000.0)]
    elif cfg["tp"] == TP_MILNE:
        b = [(400.0, 1000.0), (-4.0, -2.5), (0.4, 0.9), (-3.0, 1.0), (0.5, 2.0)]
    elif cfg["tp"] == TP_GUILLOT7:
        b = [(100.0, 500.0), (800.0, 1800.0), (-3.0, -2.0), (-2.0, 1.0), (0.1, 0.65), (-4.0, 0.0), (0.5, 2.0)]
    else:
        b = [(800.0, 2500.0)] * cfg["n_knots"]
    b += [(-8.0, -2.0)] * s if cfg["tp"] != TP_ISOTHERMAL else [(-3.0, -3.0)] * s
    if cfg["cloud"] and cfg.get("cloud_model", 0) == 1:
        b.append((-1.5, 0.5))
        if cfg["cloud_qext"] != 2:
            b += [(2.0, 5.0), (0.5, 1.5)]
        b += [[(-7.0, -4.0)], [(-7.0, -4.0), (-4.0, 0.0), (-3.0, 0.5)],
              [(-7.0, -4.0), (-3.0, 0.0), (0.5, 3.0)]][cfg["cloud_profile"]]
        if cfg["cloud_qext"] == 1:
            # amplitude below 0.8 keeps fit + feature under the Q_max = 2 cap
            b += [(0.0, 0.8), (2.5, 4.5), (-1.0, -0.3), (-2.0, 2.0)]
    elif cfg["cloud"]:
        b.append((-6.0, 2.0))
    if cfg.get("fcld", False):
        b.append((0.0, 1.0))
    if cfg.get("bd", False):
        b += [(4.5, 5.5), (20.0, 80.0)]
    if cfg["scale"]:
        b.append((0.95, 1.05))
    if cfg["offset"]:
        b.append((-100.0, 100.0))
    return np.array(b, dtype=np.float64)


def draw_params(cid: int, batch: int, stream: int = STREAM_PARAMS) -> np.ndarray:
    """[batch, P] uniform draws; row b does not depend on ``batch``."""
    cfg = CONFIGS[cid]
    bounds = param_bounds(cfg)
    u = _rng(cid, stream).uniform(0.0, 1.0, size=(batch, len(bounds)))
    return bounds[:, 0] + u * (bounds[:, 1] - bounds[:, 0])


def draw_layers(cid: int, batch: int) -> np.ndarray | None:
    cfg = CONFIGS[cid]
    if "ragged" not in cfg:
        return None
    lo, hi = cfg["ragged"]
    return _rng(cid, STREAM_LAYERS).integers(lo, hi + 1, size=batch).astype(np.int32)


@functools.lru_cache(maxsize=2)
def _ck_tables(cid: int):
    """Bin centres, k-tables [S][nT][nP][n_bins][G] (log10), g-nodes and weights, CIA at the centres."""
    cfg = CONFIGS[cid]
    tcid = _TABLE_CID[cid]
    lcfg = CONFIGS[tcid]
    edges = ck_bin_edges(cfg["nu_min"], cfg["nu_max"], cfg["ck_resolution"])
    centres = np.sqrt(edges[:-1] * edges[1:])
    sub = ck_sub_grid(edges, cfg["ck_sub"])
    g_nodes, g_w = ck_g_quadrature()
    xs = np.empty((cfg["n_species"], len(cfg["t_grid"]), len(cfg["logp_grid"]), len(centres), len(g_nodes)))
    for s in range(cfg["n_species"]):
        c, st = line_list(tcid, s, lcfg["n_lines"], lcfg["nu_min"], lcfg["nu_max"])
        xs[s] = ck_log10_table(sub, g_nodes, cfg["t_grid"], cfg["logp_grid"], c, st)
    tc = np.linspace(300.0, 3500.0, 20)
    cia = np.stack([cia_log10(tcid, p, centres, tc) for p in range(2)]) if cfg["cia"] else None
    for a in (centres, xs, tc, g_nodes, g_w, edges) + ((cia,) if cia is not None else ()):
        a.setflags(write=False)
    return centres, xs, tc, cia, g_nodes, g_w, edges


@functools.lru_cache(maxsize=4)
def _tables(tcid: int):
    cfg = CONFIGS[tcid]
    nu = np.linspace(cfg["nu_min"], cfg["nu_max"], cfg["n_nu"])
    xs = np.empty((cfg["n_species"], len(cfg["t_grid"]), len(cfg["logp_grid"]), len(nu)))
    for s in range(cfg["n_species"]):
        c, st = line_list(tcid, s, cfg["n_lines"], cfg["nu_min"], cfg["nu_max"])
        xs[s] = lorentz_log10_xsec(nu, cfg["t_grid"], cfg["logp_grid"], c, st)
    tc = np.linspace(300.0, 3500.0, 20)
    if cfg["cia"]:
        cia = np.stack([cia_log10(tcid, p, nu, tc) for p in range(2)])
    else:
        cia = None
    for a in (nu, xs, tc) + ((cia,) if cia is not None else ()):
        a.setflags(write=False)
    return nu, xs, tc, cia


def obs_path(cid: int) -> str:
    return os.path.join(_DATA_DIR, f"obs_c{cid}.txt")


def load_obs(cid: int, n_bins: int):
    """Observed binned spectrum y_k (written beforehand from the FP64 oracle at a
    seeded truth parameter vector, plus seeded Gaussian noise)."""
    path = obs_path(cid)
    if not os.path.exists(path):
        return None
    y = np.loadtxt(path, dtype=np.float64)
    if y.shape != (n_bins,):
        raise ValueError(f"{path}: expected {n_bins} values, got {y.shape}")
    return y


def truth_params(cid: int) -> np.ndarray:
    return draw_params(cid, 1, stream=STREAM_TRUTH)[0]


def noise(cid: int, n_bins: int, sigma_ppm: float) -> np.ndarray:
    return _rng(cid, STREAM_NOISE).normal(0.0, sigma_ppm * 1.0e-6, n_bins)


def workload(cid: int, batch: int | None = None, require_obs: bool = True) -> dict:
    """Everything one configuration needs, as plain numpy arrays and scalars.

    Units are cgs except where a key says otherwise (pressures in bar).
    """
    cfg = CONFIGS[cid]
    ck = {}
    if cfg.get("ck", False):
        nu, xs, tc, cia, g_nodes, g_w, edges = _ck_tables(cid)
        ck = dict(ck_g=g_nodes, ck_w=g_w, ck_edges=edges, n_nu=len(nu))
    else:
        nu, xs, tc, cia = _tables(_TABLE_CID[cid])
    lo, hi = ln_lambda_bins(nu, cfg["n_bins"]) if cid != 0 else _uniform_bins(len(nu), cfg["n_bins"])
    b = cfg["batch"] if batch is None else int(batch)
    wl = dict(_BASE)
    wl.update({k: v for k, v in cfg.items() if k not in ("t_grid", "logp_grid")})
    wl.update(
        cid=cid, batch=b, nu=nu, t_grid=np.asarray(cfg["t_grid"], dtype=np.float64),
        logp_grid=np.asarray(cfg["logp_grid"], dtype=np.float64), log10_xsec=xs,
        species=SPECIES[: cfg["n_species"]], species_mass=np.array(SPECIES_MASS[: cfg["n_species"]]),
        tc_grid=tc, log10_cia=cia, bin_lo=lo, bin_hi=hi,
        y_err=np.full(cfg["n_bins"], _BASE["sigma_ppm"] * 1.0e-6),
        offset_mask=(0.5 * (nu[lo] + nu[hi - 1]) <= 1.0e4 / 3.0).astype(np.uint8) if cfg["offset"]
        else np.zeros(cfg["n_bins"], np.uint8),
        params=draw_params(cid, b), n_layers_per_sample=draw_layers(cid, b),
        param_names=param_names(cfg), param_bounds=param_bounds(cfg),
        n_knots=cfg.get("n_knots", 0), ck=bool(cfg.get("ck", False)), ck_mix=int(cfg.get("ck_mix", 0)),
    )
    wl.update(ck)
    y = load_obs(cid, cfg["n_bins"])
    if y is None:
        if require_obs:
            raise FileNotFoundError(f"{obs_path(cid)} missing; regenerate it with tests/golden/make_obs.py")
        y = np.zeros(cfg["n_bins"])
    wl["y_obs"] = y
    return wl


def _uniform_bins(n, k):
    edges = np.linspace(0, n, k + 1).round().astype(np.int32)
    return edges[:-1].copy(), edges[1:].copy()
