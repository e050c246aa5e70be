"""Oracle gradients of the log-likelihood (test infrastructure only).

Complex-step differentiation (Squire & Trapp 1998): g_j = Im lnL(theta + i h e_j)/h
with h = 1e-30, exact to rounding wherever no branch (table cell, clamp,
case) changes within the step.  Central finite differences are the
independent second check.
"""
from __future__ import annotations

import numpy as np

from .model import forward, INVALID_LNL


def grad_complex_step(wl, theta, n_layers=None, h=1.0e-30, tables=None):
    theta = np.asarray(theta, dtype=np.float64)
    g = np.zeros(len(theta))
    for j in range(len(theta)):
        tc = theta.astype(np.complex128)
        tc[j] += 1j * h
        out = forward(wl, tc, n_layers=n_layers, tables=tables)
        if out["status"]:
            return np.zeros(len(theta))
        g[j] = np.imag(out["lnL"]) / h
    return g


def grad_central_fd(wl, theta, n_layers=None, rel_step=1.0e-6, tables=None):
    """Central differences with h_j = rel_step * max(1, |theta_j|)."""
    theta = np.asarray(theta, dtype=np.float64)
    g = np.zeros(len(theta))
    for j in range(len(theta)):
        h = rel_step * max(1.0, abs(theta[j]))
        tp = theta.copy()
        tm = theta.copy()
        tp[j] += h
        tm[j] -= h
        fp = forward(wl, tp, n_layers=n_layers, tables=tables)["lnL"]
        fm = forward(wl, tm, n_layers=n_layers, tables=tables)["lnL"]
        if fp == INVALID_LNL or fm == INVALID_LNL:
            return np.zeros(len(theta))
        g[j] = (fp - fm) / (2.0 * h)
    return g
