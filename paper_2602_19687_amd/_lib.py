"""ctypes view of the C ABI declared in include/exofwd.h (marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libexofwd.so")

OK, ERR_ARG, ERR_SHAPE, ERR_CONFIG, ERR_NOMEM, ERR_DEVICE, ERR_UNSUPPORTED = range(7)
TRANSMISSION, EMISSION = 0, 1
PREC_FP64, PREC_MIXED = 0, 1
TP_ISOTHERMAL, TP_GUILLOT3, TP_PCHIP, TP_BARSTOW, TP_MILNE, TP_GUILLOT7 = 0, 1, 2, 3, 4, 5
S_BAD_VMR, S_UNBOUND, S_NONFINITE, S_BAD_T, S_BAD_LAYERS = 1, 2, 4, 8, 16
CK_RORR, CK_PRODUCT = 0, 1

_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int32)
_U8 = C.POINTER(C.c_uint8)


class Config(C.Structure):
    _fields_ = [
        ("mode", C.c_int32), ("precision", C.c_int32), ("tp_kind", C.c_int32), ("n_knots", C.c_int32),
        ("n_species", C.c_int32), ("n_layers_max", C.c_int32), ("batch_max", C.c_int32),
        ("has_cia", C.c_int32), ("has_rayleigh", C.c_int32), ("has_cloud", C.c_int32),
        ("has_scale", C.c_int32), ("has_offset", C.c_int32), ("n_mu", C.c_int32),
        ("cloud_model", C.c_int32), ("cloud_profile", C.c_int32), ("cloud_qext", C.c_int32),
        ("has_fcld", C.c_int32),
        ("mu_fixed", C.c_double), ("p_bot_bar", C.c_double), ("p_top_bar", C.c_double),
        ("p_ref_bar", C.c_double), ("r_p", C.c_double), ("r_s", C.c_double), ("g_ref", C.c_double),
        ("kappa_ir", C.c_double), ("f_hem", C.c_double), ("kappa_cloud", C.c_double),
        ("t_star", C.c_double), ("dilution", C.c_double), ("err_c", C.c_double),
        ("ray_h2", C.c_double), ("ray_he", C.c_double),
        ("n_nu", C.c_int32), ("nu", _D),
        ("n_t", C.c_int32), ("n_p", C.c_int32), ("t_grid", _D), ("logp_grid", _D),
        ("log10_xsec", _D), ("species_mass", _D),
        ("n_tc", C.c_int32), ("tc_grid", _D), ("log10_cia", _D),
        ("n_bins", C.c_int32), ("bin_lo", _I), ("bin_hi", _I), ("y_obs", _D), ("y_err", _D),
        ("offset_mask", _U8),
        ("device", C.c_int32),
        ("has_bd", C.c_int32), ("bd_distance", C.c_double),
        ("ck_g", C.c_int32), ("ck_mix", C.c_int32), ("ck_weights", _D),
    ]


EXPORTS = {
    "exofwd_create": (C.c_int, [C.POINTER(Config), C.POINTER(C.c_void_p)]),
    "exofwd_destroy": (C.c_int, [C.c_void_p]),
    "exofwd_num_params": (C.c_int32, [C.c_void_p]),
    "exofwd_num_nu": (C.c_int32, [C.c_void_p]),
    "exofwd_num_bins": (C.c_int32, [C.c_void_p]),
    "exofwd_precision": (C.c_int32, [C.c_void_p]),
    "exofwd_grad_supported": (C.c_int32, [C.c_void_p]),
    "exofwd_forward": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_void_p]),
    "exofwd_forward_noalloc": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.c_void_p, C.c_void_p]),
    "exofwd_grad": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                              C.c_void_p, C.c_void_p, C.c_void_p]),
    "exofwd_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_char_p]),
    "exofwd_set_tuning": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "exofwd_get_tuning": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "exofwd_set_graphs": (C.c_int, [C.c_void_p, C.c_int32]),
    "exofwd_set_profiling": (C.c_int, [C.c_void_p, C.c_int32]),
    "exofwd_kernel_time": (C.c_int, [C.c_void_p, C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    "exofwd_device_bytes": (C.c_int64, [C.c_void_p]),
    "exofwd_strerror": (C.c_char_p, [C.c_int]),
    "exofwd_last_error": (C.c_char_p, [C.c_void_p]),
}

NOALLOC_SCRATCH_BYTES = 64 << 20   # EXOFWD_NOALLOC_SCRATCH_BYTES

_lib = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load the HIP library; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2602_19687_amd.build` "
                           "(the forward model has no CPU fallback)")
    lib = C.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class ExoError(RuntimeError):
    pass


def check(status: int, ctx=None, what: str = "") -> None:
    if status == OK:
        return
    lib = load()
    detail = lib.exofwd_last_error(ctx).decode() if ctx else ""
    raise ExoError(f"{what}: {lib.exofwd_strerror(status).decode()} ({status}) {detail}".strip())
