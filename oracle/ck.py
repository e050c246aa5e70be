"""Correlated-k opacities and their mixing (Section "Gas phase opacities"), in FP64.

Test infrastructure only (see the package docstring).

A k-table holds, per species, temperature, pressure and spectral bin j, the
absorption cross section k(g) at G g-points of the bin's cumulative
distribution, with quadrature weights w_g summing to 1: every bin-mean
function of the cross section over the bin becomes a g-weighted sum.  The
paper mixes the species' k-tables in one of two ways:

* random overlap with resorting and rebinning (RORR, Amundsen et al. 2017),
  layer by layer: the k-distributions of two absorbers, each expressed as
  layer optical depths, are combined on all G x G g-point pairs (sum of the
  optical depths, product of the weights), the G^2 values are sorted, and the
  sorted distribution is rebinned onto the original g-intervals; the next
  absorber is then mixed into the result, and so on;
* for transmission, random overlap through the product of the species' own
  chord transmission functions, each species keeping its own g-points.

Readings (the paper names the methods but prints neither):
  - rebinning averages k over each target g-interval: the interval
    [E_{n-1}, E_n] with E_n = w_1 + ... + w_n gets the mean of the sorted
    (quantile) function over it, so the mean sum_n w_n k_n is conserved;
  - the species are mixed in table order, absorber 0 first;
  - continuum sources (CIA, Rayleigh, a grey cloud) are grey within a bin and
    are added to every g-point after the species are mixed (RORR), or enter the
    product as one more factor exp(-tau_c) (product of transmissions);
  - the k-tables are interpolated like the cross-section tables: bilinear in
    (T, log10 p) on log10 k, clamped at the table edges.
"""
from __future__ import annotations

import numpy as np

from . import model as om


def rorr_pair(ka, kb, w):
    """Random overlap of two k-distributions with resorting and rebinning.

    ka, kb: [..., G] layer optical depths at the g-points of two absorbers (or
    of the mixture so far and the next absorber); w: [G] weights.  Returns the
    mixture's [..., G] optical depths on the same g-points: the G^2 pair sums
    ka_a + kb_b with weights w_a w_b, sorted (by real part), define a quantile
    function Q(g); point n gets the mean of Q over its interval [E_{n-1}, E_n].
    """
    w = np.asarray(w, dtype=np.float64)
    G = len(w)
    comb = (np.asarray(ka)[..., :, None] + np.asarray(kb)[..., None, :])
    comb = comb.reshape(comb.shape[:-2] + (G * G,))
    wc = (w[:, None] * w[None, :]).reshape(G * G)
    order = np.argsort(np.real(comb), axis=-1, kind="stable")
    v = np.take_along_axis(comb, order, axis=-1)
    ws = wc[order]
    c_up = np.cumsum(ws, axis=-1)            # upper end of each sorted element's g-interval
    p_up = np.cumsum(ws * v, axis=-1)        # integral of Q from 0 to c_up
    edges = np.cumsum(w)
    integ = np.empty(v.shape[:-1] + (G,), dtype=v.dtype)
    for n in range(G - 1):
        # elements lying wholly below the edge, then the part of the next one
        m = np.sum(c_up <= edges[n], axis=-1, keepdims=True)
        below = m > 0
        mm1 = np.maximum(m - 1, 0)
        p_lo = np.where(below, np.take_along_axis(p_up, mm1, axis=-1), 0.0)
        c_lo = np.where(below, np.take_along_axis(c_up, mm1, axis=-1), 0.0)
        v_m = np.take_along_axis(v, m, axis=-1)
        integ[..., n] = (p_lo + (edges[n] - c_lo) * v_m)[..., 0]
    integ[..., G - 1] = p_up[..., -1]
    return np.diff(integ, axis=-1, prepend=0.0) / w


def rorr_mix(dtau_species, w):
    """RORR mixture of all absorbers: dtau_species [S, ..., G] -> [..., G]."""
    mix = dtau_species[0]
    for s in range(1, len(dtau_species)):
        mix = rorr_pair(mix, dtau_species[s], w)
    return mix


def species_dtau(wl, t_lay, p_lay, r_lev, x, tables=None):
    """Layer optical depth of every absorber at every bin and g-point:
    dtau[s, l, j, g] = n_l X_s k_s(T_l, p_l; j, g) dr_l with n_l = p_l/(k_B T_l)."""
    tab = wl["log10_xsec"] if tables is None else tables
    dr = r_lev[1:] - r_lev[:-1]
    logp_bar = np.log10(p_lay / om.BAR)
    n_lay = len(t_lay)
    out = np.empty((len(x), n_lay) + tab.shape[3:], dtype=np.result_type(t_lay, r_lev, x))
    for s in range(len(x)):
        for l in range(n_lay):
            v = om.bilinear_log_table(tab[s], wl["t_grid"], wl["logp_grid"], t_lay[l], logp_bar[l])
            n_l = p_lay[l] / (om.K_B * t_lay[l])
            out[s, l] = n_l * x[s] * np.exp(v * np.log(10.0)) * dr[l]
    return out


def continuum_dtau(wl, t_lay, p_lev, p_lay, r_lev, x_h2, x_he, mu, log10_pc):
    """CIA, Rayleigh and grey-cloud layer optical depths at the bin centres [l, j]
    (the cross-section model's continuum terms with no absorber)."""
    return om.layer_optical_depth(wl, t_lay, p_lev, p_lay, r_lev, np.zeros(0), x_h2, x_he, mu, log10_pc)


def transit_depth_product(pm, dtau_s, dtau_c, w, r_lev, r_s):
    """Transit depth per bin with the species overlapping at random along each
    chord: T_i = exp(-tau_c,i) prod_s sum_g w_g exp(-tau_s,i,g), tau = P dtau
    (Eq. 44) for every species and g-point; then the annulus rule of the
    line-by-line path with T_i in place of exp(-tau_i)."""
    trans = np.exp(-(pm @ dtau_c))
    for s in range(len(dtau_s)):
        tau = np.tensordot(pm, dtau_s[s], axes=(1, 0))           # [i, j, g]
        trans = trans * np.sum(w * np.exp(-tau), axis=-1)
    area = r_lev[1:] ** 2 - r_lev[:-1] ** 2
    return (r_lev[0] ** 2 + area @ (1.0 - trans)) / r_s ** 2


def transit_depth_rorr(pm, dtau_mix, w, r_lev, r_s):
    """Transit depth per bin of the mixed k-distribution dtau_mix [l, j, g]: the
    g-weighted mean of the transmission of each g-point's chord."""
    tau = np.tensordot(pm, dtau_mix, axes=(1, 0))                # [i, j, g]
    trans = np.sum(w * np.exp(-tau), axis=-1)
    area = r_lev[1:] ** 2 - r_lev[:-1] ** 2
    return (r_lev[0] ** 2 + area @ (1.0 - trans)) / r_s ** 2


def toa_flux_ck(dtau_mix, t_lev, nu, w, n_mu):
    """Bin-mean outgoing flux: sum_g w_g F_toa(dtau_mix[:, :, g]) with the
    line-by-line emission solver per g-point and the Planck function at the bin
    centres."""
    flux = 0.0
    for g in range(len(w)):
        flux = flux + w[g] * om.toa_flux(dtau_mix[:, :, g], t_lev, nu, n_mu)
    return flux


def spectrum(wl, internals, log10_pc):
    """Spectrum per bin (transit depth, or F_p/F_* for emission) of one sample
    from the profile internals of ``model.forward``."""
    it = internals
    w = np.asarray(wl["ck_w"], dtype=np.float64)
    dtau_s = species_dtau(wl, it["t_lay"], it["p_lay"], it["r_lev"], it["x"])
    dtau_c = continuum_dtau(wl, it["t_lay"], it["p_lev"], it["p_lay"], it["r_lev"], it["x_h2"], it["x_he"],
                            it["mu"], log10_pc)
    r_lev = it["r_lev"]
    if wl["mode"] == 0:
        pm = om.path_matrix(r_lev)
        if wl["ck_mix"] == 1:
            return transit_depth_product(pm, dtau_s, dtau_c, w, r_lev, wl["r_s"])
        mix = rorr_mix(dtau_s, w) + dtau_c[..., None]
        return transit_depth_rorr(pm, mix, w, r_lev, wl["r_s"])
    mix = rorr_mix(dtau_s, w) + dtau_c[..., None]
    flux = toa_flux_ck(mix, it["t_lev"], wl["nu"], w, wl["n_mu"])
    return wl["dilution"] * flux / (np.pi * om.planck(wl["t_star"], wl["nu"])) * (it["r_ref"] / wl["r_s"]) ** 2
