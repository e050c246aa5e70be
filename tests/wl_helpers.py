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


def continuum_workload(kind, n_layers=1000, t_iso=1200.0, mu=2.3, nu=(1.0e4, 2.0e4), k_pair=(1e-45, 1e-45),
                       ray=(8.0e-29, 6.0e-30)):
    """Isothermal, constant g, only one continuum source: ``kind`` is "cia1"
    (H2-H2 alone, wavelength-independent k_pair[0]), "cia2" (H2-He alone,
    k_pair[1]) or "rayleigh" (H2 and He Rayleigh scattering, sigma_R =
    ray * (nu/1e4)^4).  The one absorber is present with a negligible cross
    section so that the composition (X_H2, X_He) is that of a pure H2/He gas."""
    n_nu = len(nu)
    wl = constant_sigma_workload(sigma=1e-300, t_iso=t_iso, n_layers=n_layers, n_nu=n_nu, mu=mu)
    wl["nu"] = np.asarray(nu, dtype=np.float64)
    tc = np.linspace(300.0, 3500.0, 3)
    if kind in ("cia1", "cia2"):
        tab = np.full((2, len(tc), n_nu), -300.0)
        j = 0 if kind == "cia1" else 1
        tab[j] = np.log10(k_pair[j])
        wl.update(cia=True, log10_cia=tab, tc_grid=tc, rayleigh=False)
    else:
        wl.update(cia=False, log10_cia=None, rayleigh=True, ray_h2=ray[0], ray_he=ray[1])
    # theta = [T_iso, log10 X]: the absorber's X is negligible, the gas is H2 + He
    wl["theta"] = np.array([t_iso, -12.0])
    wl["params"] = wl["theta"][None, :].copy()
    return wl
