"""exofwd: batched atmospheric forward model and adjoint on MI355X (gfx950).

The hot path (profile, opacity, chord product or emission sweep, binning,
likelihood and adjoint) runs in the HIP kernels of libexofwd.so behind the C
ABI of include/exofwd.h; this package only marshals arguments.
"""
from ._lib import LIB_PATH, load, ExoError  # noqa: F401


def __getattr__(name):
    # torch-dependent parts load lazily so that the C-ABI checks run without a device
    if name in ("ForwardModel", "ExoLogLike"):
        from . import model
        return getattr(model, name)
    raise AttributeError(name)
