"""Small hand-built workloads for oracle pins (plain dicts shaped like synth.workload)."""
import numpy as np

import synth


def constant_sigma_workload(sigma=1.0e-26, t_iso=1200.0, n_layers=50, n_nu=4, mu=2.3,
                            p_bot=100.0, p_top=1.0e-6, constant_g=True, mode=0):
    """Isothermal, one absorber with wavelength-independent sigma, nothing else."""
    wl = synth.workload(0, require_obs=False)
    nu = np.linspace(2000.0, 10000.0, n_nu)
    t_grid = np.linspace(300.0, 3500.0, 4)
    logp_grid = np.linspace(-9.0, 3.0, 4)
    # one absorber at X = 1e-3: kappa = n * 1e-3 * sigma_table = n * sigma
    tab = np.full((1, 4, 4, n_nu), np.log10(sigma / 1.0e-3))
    wl.update(mode=mode, tp=0, n_layers=n_layers, p_bot=p_bot, p_top=p_top, n_species=1,
              nu=nu, t_grid=t_grid, logp_grid=logp_grid, log10_xsec=tab, log10_cia=None,
              cia=False, rayleigh=False, cloud=False, scale=False, offset=False, mu_fixed=mu,
              bin_lo=np.array([0], np.int32), bin_hi=np.array([n_nu], np.int32),
              y_obs=np.zeros(1), y_err=np.full(1, 5e-5), offset_mask=np.zeros(1, np.uint8),
              constant_g=constant_g, params=np.array([[t_iso, -3.0]]), n_knots=0)
    wl["theta"] = np.array([t_iso, -3.0])
    return wl
