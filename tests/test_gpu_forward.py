"""GPU parity of the forward model and likelihood against the FP64 oracle.

Reduced workloads span several 64-wavenumber tiles with a ragged tail and are
compared element by element on every sample; full-size workloads (in the
launch shape the benchmark times) are compared on sampled samples.

Tolerances: FP64 path 1e-5 relative (the bar for the plain path); the mixed
path (FP16 tables, FP32 opacity, bf16x3 chord) 1e-3 relative on spectra.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from parity_util import reduced, rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _model(wl, prec, **kw):
    from paper_2602_19687_amd import ForwardModel
    return ForwardModel(wl, precision=prec, **kw)


def _run(wl, prec, params, n_layers=None, **kw):
    print(f"[gpu] cid={wl['cid']} prec={prec} B={len(params)} n_nu={len(wl['nu'])}", flush=True)
    fm = _model(wl, prec, batch_max=len(params), **kw)
    th = torch.tensor(params, dtype=torch.float64, device="cuda")
    spec, lnl, status = fm.forward(th, n_layers=n_layers)
    torch.cuda.synchronize()
    out = spec.double().cpu().numpy(), lnl.cpu().numpy(), status.cpu().numpy()
    fm.close()
    return out


SPEC_TOL = {"fp64": 1e-5, "mixed": 1e-3}
LNL_TOL = {"fp64": 1e-5, "mixed": 1e-3}


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_c0_single_sample(prec):
    wl = synth.workload(0)
    spec, lnl, st = _run(wl, prec, wl["params"])
    ref = oracle.forward(wl, wl["params"][0])
    assert st[0] == 0
    err = rel_err(spec[0], ref["spectrum"])
    print(f"c0 {prec}: spectrum max rel err {err:.3e}, lnL {lnl[0]:.6f} vs {ref['lnL']:.6f}")
    assert err < SPEC_TOL[prec]
    assert abs(lnl[0] - ref["lnL"]) / abs(ref["lnL"]) < LNL_TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("cid", [1, 2])
def test_reduced_every_sample(prec, cid):
    # 1000 wavenumbers = 15 full tiles + a 40-point ragged tail
    wl = reduced(cid, n_nu=1000, n_bins=37, batch=12)
    params = wl["params"]
    spec, lnl, st = _run(wl, prec, params)
    errs = []
    for b in range(len(params)):
        ref = oracle.forward(wl, params[b])
        assert st[b] == ref["status"]
        if ref["status"]:
            assert lnl[b] == -1e300 and np.all(np.isnan(spec[b]))
            continue
        errs.append(rel_err(spec[b], ref["spectrum"]))
        assert abs(lnl[b] - ref["lnL"]) <= LNL_TOL[prec] * abs(ref["lnL"]), (b, lnl[b], ref["lnL"])
    print(f"c{cid} reduced {prec}: spectrum max rel err {max(errs):.3e} median {np.median(errs):.3e}")
    assert max(errs) < SPEC_TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("cid", [1, 2])
def test_full_size_sampled(prec, cid):
    wl = synth.workload(cid)
    params = wl["params"]
    spec, lnl, st = _run(wl, prec, params)
    rng = np.random.default_rng(cid)
    picks = sorted(rng.choice(len(params), 4, replace=False))
    for b in picks:
        ref = oracle.forward(wl, params[b])
        assert st[b] == ref["status"]
        if ref["status"]:
            continue
        err = rel_err(spec[b], ref["spectrum"])
        lerr = abs(lnl[b] - ref["lnL"]) / abs(ref["lnL"])
        print(f"c{cid} full {prec} sample {b}: spectrum rel err {err:.3e} lnL rel err {lerr:.3e}")
        assert err < SPEC_TOL[prec]
        assert lerr < LNL_TOL[prec]
    assert np.all(np.isfinite(spec[st == 0]))


def test_invalid_samples_flagged():
    wl = reduced(1, n_nu=300, n_bins=5, batch=5)
    th = wl["params"].copy()
    th[1, 3] = -0.01           # sum X >= 1 (0.977 + 0.501 + ...)
    th[1, 4] = -0.3
    th[2, 0] = np.nan          # non-finite parameter
    spec, lnl, st = _run(wl, "mixed", th, n_layers=[100, 100, 100, 0, 100])
    assert st[0] == 0 and st[4] == 0
    assert st[1] & synth_bits("BAD_VMR")
    assert st[2] == synth_bits("NONFINITE")
    assert st[3] == synth_bits("BAD_LAYERS")
    for b in (1, 2, 3):
        assert lnl[b] == -1e300 and np.all(np.isnan(spec[b]))


def synth_bits(name):
    return {"BAD_VMR": 1, "UNBOUND": 2, "NONFINITE": 4, "BAD_T": 8, "BAD_LAYERS": 16}[name]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_ragged_layer_counts(prec):
    # per-sample layer counts from 60 to 150 (padded layer dimension 160)
    wl = reduced(1, n_nu=700, n_bins=10, batch=6, n_layers=150)
    nl = np.array([60, 150, 97, 128, 129, 61], dtype=np.int32)
    spec, lnl, st = _run(wl, prec, wl["params"], n_layers=nl)
    for b in range(6):
        ref = oracle.forward(wl, wl["params"][b], n_layers=int(nl[b]))
        assert st[b] == ref["status"] == 0
        err = rel_err(spec[b], ref["spectrum"])
        print(f"ragged {prec} L={nl[b]}: {err:.3e}")
        assert err < SPEC_TOL[prec]


def test_deterministic_bitwise():
    wl = reduced(1, n_nu=640, n_bins=8, batch=16)
    a = _run(wl, "mixed", wl["params"])
    b = _run(wl, "mixed", wl["params"])
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("cid,tol", [(1, 2e-5), (2, 1e-4)])
def test_mixed_matches_oracle_with_decoded_tables(cid, tol):
    """The storage error of the reduced-precision tables (FP16 for transmission, FP32
    for emission) separated from arithmetic error: against the oracle run on the same
    decoded tables the mixed path is much closer."""
    wl = reduced(cid, n_nu=640, n_bins=8, batch=4, start=15000 if cid == 2 else 0)
    spec, _, _ = _run(wl, "mixed", wl["params"])
    tabs = oracle.decode_tables(wl)
    for b in range(4):
        full = oracle.forward(wl, wl["params"][b])["spectrum"]
        dec = oracle.forward(wl, wl["params"][b], tables=tabs)["spectrum"]
        e_full, e_dec = rel_err(spec[b], full), rel_err(spec[b], dec)
        print(f"sample {b}: vs FP64 tables {e_full:.3e}, vs decoded stored tables {e_dec:.3e}")
        assert e_dec < tol


if __name__ == "__main__":
    sys.exit(pytest.main([__file__, "-v", "-s"]))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_c4_reduced_ragged(prec):
    """High-resolution configuration cut to 3000 wavenumbers (23 full tiles + a
    ragged tail), its own per-sample layer counts (60-150), every sample."""
    wl = reduced(4, n_nu=3000, n_bins=20, batch=8, n_layers=150, start=100000)
    nl = synth.workload(4, batch=8)["n_layers_per_sample"]
    spec, lnl, st = _run(wl, prec, wl["params"], n_layers=nl)
    errs = []
    for b in range(8):
        ref = oracle.forward(wl, wl["params"][b], n_layers=int(nl[b]))
        assert st[b] == ref["status"]
        if ref["status"]:
            continue
        errs.append(rel_err(spec[b], ref["spectrum"]))
        assert abs(lnl[b] - ref["lnL"]) <= LNL_TOL[prec] * abs(ref["lnL"])
    print(f"c4 reduced {prec}: spectrum max rel err {max(errs):.3e}")
    assert max(errs) < SPEC_TOL[prec]


@pytest.mark.parametrize("prec", ["mixed"])
def test_c4_full_size_sampled(prec):
    """The full high-resolution batch (B = 64, 400000 wavenumbers, 60-150 layers);
    two samples against the oracle, the rest finite."""
    wl = synth.workload(4)
    nl = wl["n_layers_per_sample"]
    spec, lnl, st = _run(wl, prec, wl["params"], n_layers=nl)
    assert np.all(st == 0) and np.all(np.isfinite(spec))
    for b in (int(np.argmax(nl)), int(np.argmin(nl))):
        ref = oracle.forward(wl, wl["params"][b], n_layers=int(nl[b]))
        err = rel_err(spec[b], ref["spectrum"])
        lerr = abs(lnl[b] - ref["lnL"]) / abs(ref["lnL"])
        print(f"c4 full {prec} sample {b} L={nl[b]}: spectrum rel err {err:.3e} lnL rel err {lerr:.3e}")
        assert err < SPEC_TOL[prec] and lerr < LNL_TOL[prec]


def test_emission_high_wavenumber_end_every_sample():
    """The short-wavelength end of the emission grid, where the flux ratio falls to
    ~1e-9 of its peak and thin hot upper layers can carry the emergent intensity."""
    wl = reduced(2, n_nu=1000, n_bins=25, batch=16, start=19000)
    spec, lnl, st = _run(wl, "mixed", wl["params"])
    errs = []
    for b in range(16):
        ref = oracle.forward(wl, wl["params"][b])
        assert st[b] == ref["status"]
        if ref["status"]:
            continue
        errs.append(rel_err(spec[b], ref["spectrum"]))
    print(f"c2 high-nu mixed: spectrum max rel err {max(errs):.3e}")
    assert max(errs) < 1e-4


def test_emission_full_batch_mixed_vs_fp64():
    """Every sample and wavenumber of the emission batch: the reduced-precision path
    against the FP64 GPU path (itself pinned to the oracle), and the worst sample
    against the oracle."""
    wl = synth.workload(2)
    a, _, sa = _run(wl, "mixed", wl["params"])
    b, _, sb = _run(wl, "fp64", wl["params"])
    ok = (sa == 0) & (sb == 0)
    rel = np.abs(a[ok] - b[ok]) / np.abs(b[ok])
    per = rel.max(axis=1)
    worst = int(np.flatnonzero(ok)[np.argmax(per)])
    print(f"c2 full batch: max rel err mixed vs fp64 {per.max():.3e}, median {np.median(per):.3e}, worst sample {worst}")
    assert per.max() < 1e-4
    ref = oracle.forward(wl, wl["params"][worst])
    assert rel_err(b[worst], ref["spectrum"]) < 1e-10
    assert rel_err(a[worst], ref["spectrum"]) < 1e-4


def test_call_errors_through_the_c_abi():
    """Misuse caught on the host before any launch: B outside [1, batch_max]
    (ERR_SHAPE), NULL params (ERR_ARG), a gradient call without lnL or grad
    buffers (ERR_ARG); the context stays usable and its last error names the cause."""
    import ctypes as C
    from paper_2602_19687_amd import ForwardModel, _lib as L
    wl = reduced(1, n_nu=256, n_bins=4, batch=4)
    fm = ForwardModel(wl, precision="mixed", batch_max=4)
    lib, ctx = fm.lib, fm.ctx
    th = torch.tensor(wl["params"], device="cuda")
    lnl = torch.empty(4, dtype=torch.float64, device="cuda")
    grad = torch.empty_like(th)
    st = torch.empty(4, dtype=torch.int32, device="cuda")
    p = C.c_void_p(th.data_ptr())
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    for B in (0, 5, -1):
        assert lib.exofwd_forward(ctx, B, p, None, None, C.c_void_p(lnl.data_ptr()), C.c_void_p(st.data_ptr()),
                                  stream) == L.ERR_SHAPE
    assert b"batch_max" in lib.exofwd_last_error(ctx)
    assert lib.exofwd_forward(ctx, 4, None, None, None, C.c_void_p(lnl.data_ptr()), C.c_void_p(st.data_ptr()),
                              stream) == L.ERR_ARG
    assert lib.exofwd_grad(ctx, 4, p, None, None, None, C.c_void_p(grad.data_ptr()), C.c_void_p(st.data_ptr()),
                           stream) == L.ERR_ARG
    # still usable
    spec, lnl2, st2 = fm.forward(th)
    torch.cuda.synchronize()
    assert torch.all(st2 == 0) and torch.all(torch.isfinite(lnl2))
    fm.close()
