"""Pins of the correlated-k oracle (tables summarised per bin at g-points, mixed
by random overlap with resorting and rebinning, or by the product of the
species' transmission functions), against identities, brute force on tiny
inputs and the independent line-by-line path.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth
from oracle import ck
from parity_util import reduced_ck

W8 = synth.ck_g_quadrature()[1]


def _sorted_k(rng, g, lo=-3.0, hi=1.0):
    return np.sort(10.0 ** rng.uniform(lo, hi, g))


def _rorr_event_sweep(ka, kb, w):
    """The rebinned mixture by a sweep over the merged breakpoints of the sorted
    pair distribution and the target intervals (pure Python, tiny inputs)."""
    G = len(w)
    pairs = sorted((ka[a] + kb[b], w[a] * w[b]) for a in range(G) for b in range(G))
    targets = list(itertools.accumulate(w))
    out = [0.0] * G
    g_pos, n = 0.0, 0
    for val, wt in pairs:
        left = wt
        while left > 1e-300 and n < G:
            room = targets[n] - g_pos
            take = min(left, room)
            out[n] += val * take
            g_pos += take
            left -= take
            if room - take <= 1e-15:
                n += 1
    return np.array(out) / w


def test_rorr_with_an_empty_absorber_returns_the_other():
    rng = np.random.default_rng(1)
    ka = _sorted_k(rng, 8)
    np.testing.assert_allclose(ck.rorr_pair(ka, np.zeros(8), W8), ka, rtol=1e-13)
    np.testing.assert_allclose(ck.rorr_pair(np.zeros(8), ka, W8), ka, rtol=1e-13)


def test_rorr_of_grey_absorbers_is_their_sum():
    out = ck.rorr_pair(np.full(8, 0.3), np.full(8, 1.7), W8)
    np.testing.assert_allclose(out, 2.0, rtol=1e-12)


@pytest.mark.parametrize("seed", range(5))
def test_rorr_conserves_the_mean_and_sorts(seed):
    rng = np.random.default_rng(10 + seed)
    ka, kb = _sorted_k(rng, 8), _sorted_k(rng, 8, -1.0, 2.0)
    out = ck.rorr_pair(ka, kb, W8)
    assert np.sum(W8 * out) == pytest.approx(np.sum(W8 * ka) + np.sum(W8 * kb), rel=1e-13)
    assert np.all(np.diff(out) >= 0.0)
    assert out[0] >= ka[0] + kb[0] and out[-1] <= ka[-1] + kb[-1]


@pytest.mark.parametrize("g", [3, 4, 8])
def test_rorr_matches_event_sweep(g):
    rng = np.random.default_rng(100 + g)
    w = rng.uniform(0.2, 1.0, g)
    w /= w.sum()
    for _ in range(5):
        ka, kb = _sorted_k(rng, g), _sorted_k(rng, g)
        np.testing.assert_allclose(ck.rorr_pair(ka, kb, w), _rorr_event_sweep(ka, kb, w), rtol=1e-12)
    # vectorised over leading axes like one row at a time
    ka = np.sort(rng.uniform(0, 1, (3, 4, g)), axis=-1)
    kb = np.sort(rng.uniform(0, 1, (3, 4, g)), axis=-1)
    full = ck.rorr_pair(ka, kb, w)
    for i in range(3):
        for j in range(4):
            np.testing.assert_allclose(full[i, j], _rorr_event_sweep(ka[i, j], kb[i, j], w), rtol=1e-12)


def test_product_rule_is_random_overlap_of_exact_distributions():
    """Two species on one homogeneous chord, each given by its exact
    k-distribution (its N sub-grid cross sections, sorted, weights 1/N): the
    product of the species' transmission functions equals the mean of
    exp(-sigma_1 u_1 - sigma_2 u_2) over all N^2 independent pairs."""
    rng = np.random.default_rng(3)
    n = 16
    s1, s2 = 10.0 ** rng.uniform(-2, 1, n), 10.0 ** rng.uniform(-1, 0.5, n)
    w = np.full(n, 1.0 / n)
    r_lev = np.array([1.0, 1.2])
    pm = np.array([[1.0]])
    dtau_s = np.stack([np.sort(s1)[None, None, :], np.sort(s2)[None, None, :]])   # [s, l, j, g]
    dtau_c = np.array([[0.05]])
    depth = ck.transit_depth_product(pm, dtau_s, dtau_c, w, r_lev, 1.0)[0]
    area = r_lev[1] ** 2 - r_lev[0] ** 2
    trans = 1.0 - (depth - r_lev[0] ** 2) / area
    brute = np.mean([np.exp(-a - b - 0.05) for a in s1 for b in s2])
    assert trans == pytest.approx(brute, rel=1e-13)


def _grey_ck_and_os(cid, n_ck=40):
    """A ck workload whose k-tables do not depend on g, and the line-by-line
    workload with the same cross sections at the bin centres."""
    wl = reduced_ck(cid, n_ck=n_ck, n_bins=8, batch=3, step=50, n_layers=40)
    grey = np.repeat(wl["log10_xsec"][..., 3:4], wl["log10_xsec"].shape[-1], axis=-1)
    wck = dict(wl, log10_xsec=grey)
    wos = dict(wl, ck=False, log10_xsec=np.ascontiguousarray(grey[..., 0]))
    return wck, wos


@pytest.mark.parametrize("cid,mix", [(7, synth.CK_MIX_PRODUCT), (7, synth.CK_MIX_RORR), (8, synth.CK_MIX_RORR)])
def test_grey_k_tables_reduce_to_line_by_line(cid, mix):
    wck, wos = _grey_ck_and_os(cid)
    wck["ck_mix"] = mix
    for th in wck["params"]:
        a, b = oracle.forward(wck, th), oracle.forward(wos, th)
        assert a["status"] == b["status"] == 0
        np.testing.assert_allclose(a["spectrum"], b["spectrum"], rtol=1e-11)


def test_ck_emission_isothermal_is_blackbody_ratio():
    wl = reduced_ck(8, n_ck=30, n_bins=5, batch=1, step=80, n_layers=40)
    th = wl["params"][0].copy()
    th[:5] = 1400.0
    out = oracle.forward(wl, th)
    assert out["status"] == 0
    ref = (wl["r_p"] / wl["r_s"]) ** 2 * oracle.planck(1400.0, wl["nu"]) / oracle.planck(wl["t_star"], wl["nu"])
    np.testing.assert_allclose(out["spectrum"], ref, rtol=1e-12)


@pytest.mark.parametrize("mix", [synth.CK_MIX_PRODUCT, synth.CK_MIX_RORR])
def test_ck_transmission_monotone_in_a_species_table(mix):
    wl = reduced_ck(7, n_ck=30, n_bins=5, batch=2, step=60, n_layers=40)
    wl["ck_mix"] = mix
    th = wl["params"][1].copy()
    th[3:9] = -4.0                     # every absorber visible
    th[9] = 1.9                        # cloud deck at the bottom
    base = oracle.forward(wl, th)["spectrum"]
    more = oracle.forward(dict(wl, log10_xsec=wl["log10_xsec"] + np.log10(3.0) * (np.arange(6) == 2)[:, None, None,
                                                                                                    None, None]),
                          th)["spectrum"]
    assert np.all(more >= base * (1 - 1e-14)) and np.any(more > base * (1 + 1e-6))


def test_k_table_of_a_continuum_is_flat_and_tables_ascend_in_g():
    edges = synth.ck_bin_edges(2000.0, 2100.0, 1000.0)
    sub = synth.ck_sub_grid(edges, 16)
    g, w = synth.ck_g_quadrature()
    assert w.sum() == pytest.approx(1.0, rel=1e-15) and np.all(np.diff(g) > 0)
    flat = synth.ck_log10_table(sub, g, [1000.0], [0.0], np.array([1.0e5]), np.array([0.0]))
    np.testing.assert_allclose(flat, -24.0, atol=1e-13)
    wl = synth.workload(7, batch=1, require_obs=False)
    assert np.all(np.diff(wl["log10_xsec"], axis=-1) >= 0.0)
