"""Determinism of the whole gradient step: two contexts, two calls each, give
bitwise-equal spectra, lnL and gradients (no float atomics in any reduction;
every chunked sum is added in a fixed order).  Transmission, emission, the
non-grey cloud and isolated objects, in both precisions."""
import numpy as np
import pytest

import synth
from parity_util import reduced

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _wl(kind):
    if kind == "transmission":
        return reduced(1, n_nu=1280, n_bins=16, batch=8, step=20)
    if kind == "emission":
        return reduced(2, n_nu=640, n_bins=16, batch=8, step=30)
    if kind == "nongrey":
        return reduced(5, n_nu=1280, n_bins=16, batch=8, step=20)
    wl = reduced(2, n_nu=640, n_bins=16, batch=8, step=30)   # isolated objects
    cfg = {**synth.CONFIGS[2], "bd": True}
    bounds = synth.param_bounds(cfg)
    u = np.random.default_rng(77).uniform(size=(8, len(bounds)))
    wl.update(bd=True, param_names=synth.param_names(cfg), param_bounds=bounds,
              params=bounds[:, 0] + u * (bounds[:, 1] - bounds[:, 0]),
              y_obs=np.full(16, 1e-16), y_err=np.full(16, 1e-17))
    return wl


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
@pytest.mark.parametrize("kind", ["transmission", "emission", "nongrey", "isolated"])
def test_gradient_step_is_bitwise_reproducible(kind, prec):
    from paper_2602_19687_amd import ForwardModel
    wl = _wl(kind)
    print(f"[gpu] determinism {kind} {prec}", flush=True)
    th = torch.tensor(wl["params"], device="cuda")
    runs = []
    for _ in range(2):
        fm = ForwardModel(wl, precision=prec, batch_max=len(wl["params"]))
        assert fm.has_grad
        for _ in range(2):
            lnl, g, st, sp = fm.grad(th, want_spectra=True)
            runs.append((lnl.clone(), g.clone(), st.clone(), sp.clone()))
        fm.close()
    assert int(runs[0][2].ne(0).sum()) < len(wl["params"])
    for r in runs[1:]:
        for x, y in zip(runs[0], r):
            # bytes, so that the NaN spectra of invalid samples compare equal too
            assert torch.equal(x.contiguous().view(torch.uint8), y.contiguous().view(torch.uint8))
