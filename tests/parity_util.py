"""Shared helpers for GPU parity tests: reduced workloads and error measures."""
import numpy as np

import synth


def reduced(cid, n_nu, n_bins, batch, n_layers=None, start=0, step=1):
    """Config ``cid`` cut to ``n_nu`` wavenumbers (every ``step``-th from index
    ``start``) and ``n_bins`` index-uniform bins; y_obs is the full observation's level."""
    wl = dict(synth.workload(cid, batch=batch))
    sl = slice(start, start + n_nu * step, step)
    wl["nu"] = wl["nu"][sl]
    wl["log10_xsec"] = np.ascontiguousarray(wl["log10_xsec"][..., sl])
    if wl["log10_cia"] is not None:
        wl["log10_cia"] = np.ascontiguousarray(wl["log10_cia"][..., sl])
    edges = np.linspace(0, n_nu, n_bins + 1).round().astype(np.int32)
    wl["bin_lo"], wl["bin_hi"] = edges[:-1].copy(), edges[1:].copy()
    level = float(np.mean(wl["y_obs"]))
    wl["y_obs"] = level * (1.0 + 0.01 * np.sin(np.arange(n_bins)))
    wl["y_err"] = np.full(n_bins, 5.0e-5)
    wl["offset_mask"] = (np.arange(n_bins) >= n_bins // 2).astype(np.uint8)
    if n_layers is not None:
        wl["n_layers"] = n_layers
    return wl


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.max(np.abs(a - b) / np.abs(b))


def reduced_ck(cid, n_ck, n_bins, batch, start=0, step=1, n_layers=None):
    """Correlated-k config ``cid`` cut to ``n_ck`` spectral bins (every ``step``-th
    from ``start``) and ``n_bins`` index-uniform observation bins."""
    wl = dict(synth.workload(cid, batch=batch, require_obs=False))
    sl = slice(start, start + n_ck * step, step)
    wl["nu"] = wl["nu"][sl]
    wl["log10_xsec"] = np.ascontiguousarray(wl["log10_xsec"][:, :, :, sl, :])
    if wl["log10_cia"] is not None:
        wl["log10_cia"] = np.ascontiguousarray(wl["log10_cia"][..., sl])
    edges = np.linspace(0, n_ck, n_bins + 1).round().astype(np.int32)
    wl["bin_lo"], wl["bin_hi"] = edges[:-1].copy(), edges[1:].copy()
    level = 0.012 if wl["mode"] == 0 else 1.0e-3
    wl["y_obs"] = level * (1.0 + 0.01 * np.sin(np.arange(n_bins)))
    wl["y_err"] = np.full(n_bins, 5.0e-5)
    wl["offset_mask"] = (np.arange(n_bins) >= n_bins // 2).astype(np.uint8)
    wl["n_nu"] = n_ck
    if n_layers is not None:
        wl["n_layers"] = n_layers
    return wl
