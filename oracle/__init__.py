"""FP64 CPU oracle for the batched atmospheric forward model (test infrastructure).

This package is the plain, slow, obviously-correct definition that the HIP
library is checked against.  It is *test infrastructure*: only the test suite,
the smoke check and the CPU-baseline leg of the benchmark may import it; the
product path never does.  It shares no code with the HIP library: it reads the
same synthetic input arrays (``synth``) and nothing else.

Everything is double precision (complex128 under complex-step
differentiation), cgs units, loops over layers and species, NumPy vectorised
over wavenumber only, with a dense path-matrix product.  Each function cites
the section or equation of the paper it follows; readings of points where the
paper is silent are stated where they are used.
"""
from .model import (  # noqa: F401
    BAR, K_B, M_U, H_PL, C_LIGHT, HE_H2, M_H2, M_HE,
    S_BAD_VMR, S_UNBOUND, S_NONFINITE, S_BAD_T, S_BAD_LAYERS, INVALID_LNL,
    level_pressures, tp_isothermal, tp_guillot3, pchip, tp_profile, chemistry,
    TP_ISOTHERMAL, TP_GUILLOT3, TP_PCHIP, TP_BARSTOW, TP_MILNE, TP_GUILLOT7, KAPPA_AD, Q_HOPF_INF, tp_barstow,
    hopf_stretched, tp_milne, tp_guillot7,
    G_GRAV, M_JUP, toa_flux, brown_dwarf_radius, brown_dwarf_flux,
    altitudes, interp_index, bilinear_log_table, cia_log, cloud_fraction,
    layer_optical_depth, path_matrix, transit_depth, planck, gauss_legendre_01,
    emission_intensity, emission_ratio, bin_means, log_likelihood,
    forward, decode_tables, split_params,
    CLOUD_GREY_DECK, CLOUD_NONGREY, QPROF_UNIFORM, QPROF_SLAB, QPROF_POWER, QEXT_FIT, QEXT_FIT_FEATURE,
    QEXT_GREY, X0_FEATURE, Q_MAX, nongrey_param_count, layer_coverage, condensate_profile,
    feature_efficiency, extinction_efficiency, nongrey_cloud_dtau,
)
from .grad import grad_complex_step, grad_central_fd  # noqa: F401
from . import ck  # noqa: F401
