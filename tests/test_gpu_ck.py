"""GPU parity of the correlated-k path (k-tables mixed by random overlap with
resorting and rebinning, then the transmission chord or the emission sweep per
g-point) against the FP64 oracle: every sample of reduced workloads that span
several mixing waves, chord tiles and emission tiles with a ragged last one,
ragged layer counts, full-size sampled batches, invalid samples, and the refusals
of what the path does not provide.

Tolerance: spectra and lnL 1e-3 relative (reduced precision: FP32 table entries,
FP32 mixing whose sort keys drop the low six bits of each pair sum, bf16x3 chord).
"""
import ctypes as C

import numpy as np
import pytest

import oracle
import synth
from parity_util import reduced_ck, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-3


def _model(wl, batch_max):
    from paper_2602_19687_amd import ForwardModel
    return ForwardModel(wl, precision="mixed", batch_max=batch_max)


def _compare(wl, params, n_layers=None, label=""):
    print(f"[gpu] ck {label}: cid={wl['cid']} B={len(params)} bins={len(wl['nu'])}", flush=True)
    fm = _model(wl, len(params))
    assert not fm.has_grad
    spec, lnl, st = fm.forward(torch.tensor(params, device="cuda"), n_layers=n_layers)
    spec, lnl, st = spec.double().cpu().numpy(), lnl.cpu().numpy(), st.cpu().numpy()
    fm.close()
    errs = []
    for b, th in enumerate(params):
        ref = oracle.forward(wl, th, n_layers=None if n_layers is None else int(n_layers[b]))
        assert st[b] == ref["status"], (b, st[b], ref["status"])
        if ref["status"]:
            assert lnl[b] == -1e300 and np.all(np.isnan(spec[b]))
            continue
        errs.append(rel_err(spec[b], ref["spectrum"]))
        assert abs(lnl[b] - ref["lnL"]) <= TOL * abs(ref["lnL"]), (b, lnl[b], ref["lnL"])
    print(f"ck {label}: spectrum max rel err {max(errs):.3e} median {np.median(errs):.3e}")
    assert max(errs) < TOL
    return errs


CASES = [(7, synth.CK_MIX_RORR), (7, synth.CK_MIX_PRODUCT), (8, synth.CK_MIX_RORR)]
IDS = ["trans-rorr", "trans-product", "emis-rorr"]


@pytest.mark.parametrize("cid,mix", CASES, ids=IDS)
def test_ck_reduced_every_sample(cid, mix):
    # 301 bins: 18 full mixing waves + a partial one, 37 full 8-bin chord or emission
    # tiles + a partial one, 150 two-bin product tiles + a half one
    wl = reduced_ck(cid, n_ck=301, n_bins=25, batch=6, step=7)
    wl["ck_mix"] = mix
    _compare(wl, wl["params"], label=f"reduced mix {mix}")


@pytest.mark.parametrize("cid,mix", CASES, ids=IDS)
def test_ck_ragged_layers(cid, mix):
    wl = reduced_ck(cid, n_ck=130, n_bins=10, batch=5, step=15)
    wl["ck_mix"] = mix
    nl = np.array([100, 2, 37, 64, 99], dtype=np.int32)
    _compare(wl, wl["params"], n_layers=nl, label=f"ragged mix {mix}")


# RORR with one absorber dominating: the pairs of a merge then sort in blocks of
# one g-point of the larger distribution, and the g-interval edges fall exactly on
# block boundaries; the mixing keeps its g bookkeeping in FP64 so that rounding does
# not move part of the next block's (far larger) value across an edge.  Tolerance:
# 2e-5 (the path's other roundings give below 3e-6 on these spectra; running
# weights rounded to FP32 give errors up to 4e-3 in single mixed g-points).
TOL_DOMINANT = 2e-5


@pytest.mark.parametrize("cid", [7, 8], ids=["trans", "emis"])
def test_ck_rorr_dominant_absorber(cid):
    wl = reduced_ck(cid, n_ck=130, n_bins=10, batch=4, step=15)
    wl["ck_mix"] = synth.CK_MIX_RORR
    first = 3 if cid == 7 else 5
    S = wl["log10_xsec"].shape[0]
    th = np.repeat(wl["params"][:1], 4, axis=0)
    th[:, first:first + S] = -12.0
    for b, dom in enumerate((0, S - 1, S // 2)):
        th[b, first + dom] = -2.5
    th[3, first] = th[3, first + 1] = -3.0          # two comparable absorbers, the rest negligible
    print(f"[gpu] ck dominant absorber cid={cid}", flush=True)
    fm = _model(wl, 4)
    spec, lnl, st = fm.forward(torch.tensor(th, device="cuda"))
    spec = spec.double().cpu().numpy()
    fm.close()
    errs = []
    for b in range(4):
        ref = oracle.forward(wl, th[b])
        assert st[b].item() == ref["status"] == 0
        errs.append(rel_err(spec[b], ref["spectrum"]))
    print(f"ck dominant absorber c{cid}: spectrum max rel err {max(errs):.3e}")
    assert max(errs) < TOL_DOMINANT, errs


def test_ck_invalid_samples():
    wl = reduced_ck(8, n_ck=64, n_bins=4, batch=3, step=30)
    th = wl["params"].copy()
    th[1, 5:8] = -0.2            # mixing ratios summing past 1
    th[2, 0] = -50.0             # a negative knot temperature
    _compare(wl, th, label="invalid")


@pytest.mark.parametrize("cid,mix", CASES, ids=IDS)
def test_ck_full_size_sampled(cid, mix):
    wl = dict(synth.workload(cid, batch=64))
    wl["ck_mix"] = mix
    print(f"[gpu] ck full size cid={cid} mix={mix}", flush=True)
    fm = _model(wl, 64)
    spec, lnl, st = fm.forward(torch.tensor(wl["params"], device="cuda"))
    spec, lnl, st = spec.double().cpu().numpy(), lnl.cpu().numpy(), st.cpu().numpy()
    fm.close()
    for b in (0, 41):
        ref = oracle.forward(wl, wl["params"][b])
        assert st[b] == ref["status"] == 0
        err = rel_err(spec[b], ref["spectrum"])
        print(f"ck full c{cid} b={b}: spectrum max rel err {err:.3e}")
        assert err < TOL
        assert abs(lnl[b] - ref["lnL"]) <= TOL * abs(ref["lnL"])


def test_ck_refusals():
    """What the correlated-k path does not provide is refused at create: FP64, the
    cloudy/clear mixing, the product rule in emission; exofwd_grad on a ck context
    returns EXOFWD_ERR_UNSUPPORTED."""
    from paper_2602_19687_amd import _lib as L
    from paper_2602_19687_amd.model import build_config
    lib = L.load()
    wl = reduced_ck(7, n_ck=64, n_bins=4, batch=2, step=30)
    we = reduced_ck(8, n_ck=64, n_bins=4, batch=2, step=30)
    for w_, prec, code in ((dict(wl, fcld=True), L.PREC_MIXED, L.ERR_UNSUPPORTED),
                           (wl, L.PREC_FP64, L.ERR_UNSUPPORTED),
                           (dict(we, ck_mix=synth.CK_MIX_PRODUCT), L.PREC_MIXED, L.ERR_CONFIG)):
        cfg, keep = build_config(w_, prec, 2)
        ctx = C.c_void_p()
        assert lib.exofwd_create(C.byref(cfg), C.byref(ctx)) == code
    fm = _model(dict(wl, ck_mix=synth.CK_MIX_RORR), 2)
    th = torch.tensor(wl["params"], device="cuda")
    with pytest.raises(L.ExoError, match="unsupported"):
        fm.grad(th)
    fm.close()
