"""The allocation-free forward call, exofwd_forward_noalloc, through the C ABI.

Its kernels are exofwd_forward's with the per-call workspace in a static device
array, so its spectra, lnL and status must equal exofwd_forward's bit for bit on
the same inputs.  Each case makes two calls in a row, the second with a smaller
batch (the array keeps the first call's contents), for the reduced-precision and
FP64 transmission models (ragged layer counts, also past 128 layers, where the
samples run in two layer-count classes), reduced-precision emission, the non-grey
cloud, the partly cloudy limb (whose spectra always pass through the array) and
the correlated-k models (both mixings); a batch whose workspace exceeds the array
is refused with EXOFWD_ERR_SHAPE and leaves the context usable.
"""
import ctypes as C

import numpy as np
import pytest

from parity_util import reduced, reduced_ck

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _ptr(t):
    return C.c_void_p(t.data_ptr() if t is not None else None)


def _call(fm, fn, th, nl, want_spectra):
    b = th.shape[0]
    spec = torch.full((b, fm.n_nu), -7.0, dtype=fm.spec_dtype, device="cuda") if want_spectra else None
    lnl = torch.full((b,), -7.0, dtype=torch.float64, device="cuda")
    st = torch.full((b,), -7, dtype=torch.int32, device="cuda")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = fn(fm.ctx, b, _ptr(th), _ptr(nl), _ptr(spec), _ptr(lnl), _ptr(st), stream)
    torch.cuda.synchronize()
    return rc, (spec.cpu().numpy() if spec is not None else None), lnl.cpu().numpy(), st.cpu().numpy()


CASES = [
    # (config, precision, ragged layer counts)
    (1, "mixed", True),
    (1, "fp64", True),
    (2, "mixed", False),
    (4, "mixed", True),
    (5, "mixed", False),
    (6, "mixed", False),
    (7, "mixed", False),
    (8, "mixed", False),
]


@pytest.mark.parametrize("cid,prec,ragged", CASES)
def test_noalloc_forward_equals_forward(cid, prec, ragged):
    from paper_2602_19687_amd import ForwardModel
    from paper_2602_19687_amd import _lib as L
    if cid in (7, 8):
        wl = reduced_ck(cid, n_ck=150, n_bins=15, batch=12, step=13)
    else:
        wl = reduced(cid, n_nu=1000, n_bins=37, batch=12)
    fm = ForwardModel(wl, precision=prec, batch_max=12)
    lib = fm.lib
    rng = np.random.default_rng(100 + cid)
    for b in (12, 5):      # the second call is smaller than the first
        print(f"[gpu] noalloc cid={cid} prec={prec} B={b}", flush=True)
        rows = rng.permutation(len(wl["params"]))[:b]
        th = torch.tensor(wl["params"][rows], dtype=torch.float64, device="cuda")
        nl = (torch.tensor(rng.integers(2, wl["n_layers"] + 1, size=b), dtype=torch.int32, device="cuda")
              if ragged else None)
        for want_spectra in (True, False):
            rc0, s0, l0, t0 = _call(fm, lib.exofwd_forward, th, nl, want_spectra)
            rc1, s1, l1, t1 = _call(fm, lib.exofwd_forward_noalloc, th, nl, want_spectra)
            assert rc0 == L.OK and rc1 == L.OK, (rc0, rc1, lib.exofwd_last_error(fm.ctx))
            assert np.array_equal(t0, t1)
            assert np.array_equal(l0, l1), np.max(np.abs(l0 - l1))
            if want_spectra:
                assert np.array_equal(s0, s1, equal_nan=True)
            assert np.all(t1 >= 0) and np.all(l1 != -7.0)
        assert np.any(t1 == 0)
    fm.close()


def test_noalloc_refuses_batch_beyond_scratch():
    from paper_2602_19687_amd import ForwardModel
    from paper_2602_19687_amd import _lib as L
    # about 77 KB of workspace per sample at 128 padded layers: 1200 samples need more than 64 MiB
    wl = reduced(1, n_nu=1000, n_bins=37, batch=1200)
    fm = ForwardModel(wl, precision="mixed", batch_max=1200)
    th = torch.tensor(wl["params"], dtype=torch.float64, device="cuda")
    print("[gpu] noalloc refusal B=1200", flush=True)
    rc, _, lnl, _ = _call(fm, fm.lib.exofwd_forward_noalloc, th, None, True)
    assert rc == L.ERR_SHAPE
    msg = fm.lib.exofwd_last_error(fm.ctx).decode()
    assert "bytes of scratch" in msg, msg
    assert np.all(lnl == -7.0)            # nothing was enqueued
    # the context still serves both entry points
    rc0, s0, l0, t0 = _call(fm, fm.lib.exofwd_forward, th[:64], None, True)
    rc1, s1, l1, t1 = _call(fm, fm.lib.exofwd_forward_noalloc, th[:64], None, True)
    assert rc0 == rc1 == L.OK
    assert np.array_equal(l0, l1) and np.array_equal(s0, s1, equal_nan=True) and np.array_equal(t0, t1)
    fm.close()
