"""GPU adjoint (d lnL / d params) against the FP64 oracle's complex-step
gradient and against central differences.

Per-component error is |g - g*| / max(|g*_j|, 1e-3 max_j |g*_j|).
Tolerances: FP64 path 1e-5; reduced-precision path 1e-3.
"""
import numpy as np
import pytest

import oracle
import synth
from parity_util import reduced

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = {"fp64": 1e-5, "mixed": 1e-3}


def grad_err(g, gref):
    scale = np.maximum(np.abs(gref), 1e-3 * np.max(np.abs(gref)))
    return np.max(np.abs(g - gref) / scale)


def _grad(wl, prec, params, n_layers=None):
    from paper_2602_19687_amd import ForwardModel
    print(f"[gpu] grad cid={wl['cid']} prec={prec} B={len(params)} n_nu={len(wl['nu'])}", flush=True)
    fm = ForwardModel(wl, precision=prec, batch_max=len(params))
    th = torch.tensor(params, dtype=torch.float64, device="cuda")
    lnl, g, st, _ = fm.grad(th, n_layers=n_layers)
    _, lnl_f, _ = fm.forward(th, n_layers=n_layers, want_spectra=False)
    torch.cuda.synchronize()
    out = lnl.cpu().numpy(), g.cpu().numpy(), st.cpu().numpy(), lnl_f.cpu().numpy()
    fm.close()
    return out


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_reduced_grad_vs_complex_step(prec):
    wl = reduced(3, n_nu=900, n_bins=30, batch=6)
    lnl, g, st, lnl_f = _grad(wl, prec, wl["params"])
    assert np.array_equal(lnl, lnl_f)
    errs = []
    for b in range(len(wl["params"])):
        gref = oracle.grad_complex_step(wl, wl["params"][b])
        assert st[b] == 0
        e = grad_err(g[b], gref)
        errs.append(e)
        print(f"sample {b}: grad err {e:.3e}\n  gpu {g[b]}\n  ref {gref}")
    print(f"reduced {prec}: max grad err {max(errs):.3e}")
    assert max(errs) < TOL[prec]


def test_isothermal_single_absorber_grad():
    wl = synth.workload(0)
    for prec in ("fp64", "mixed"):
        lnl, g, st, _ = _grad(wl, prec, wl["params"])
        gref = oracle.grad_complex_step(wl, wl["params"][0])
        e = grad_err(g[0], gref)
        print(f"c0 {prec}: {g[0]} vs {gref}: {e:.3e}")
        assert e < TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_full_c3_sampled(prec):
    wl = synth.workload(3)
    lnl, g, st, _ = _grad(wl, prec, wl["params"])
    for b in (5, 77):
        gref = oracle.grad_complex_step(wl, wl["params"][b])
        e = grad_err(g[b], gref)
        print(f"c3 {prec} sample {b}: grad err {e:.3e}")
        assert e < TOL[prec]
    assert np.all(np.isfinite(g[st == 0]))
    assert np.all(g[st != 0] == 0)


def test_fp64_grad_vs_central_differences_of_gpu_forward():
    """Independent of the oracle: the FP64 adjoint against central differences of the
    FP64 GPU forward model (h_j = 1e-6 max(1, |theta_j|))."""
    from paper_2602_19687_amd import ForwardModel
    wl = reduced(3, n_nu=640, n_bins=20, batch=2)
    th0 = wl["params"][:2]
    P = th0.shape[1]
    fm = ForwardModel(wl, precision="fp64", batch_max=2 * P)
    lnl, g, st, _ = fm.grad(torch.tensor(th0, device="cuda"))
    g = g.cpu().numpy()
    for b in range(2):
        h = 1e-6 * np.maximum(1.0, np.abs(th0[b]))
        plus = th0[b][None, :] + np.diag(h)
        minus = th0[b][None, :] - np.diag(h)
        _, lp, _ = fm.forward(torch.tensor(plus, device="cuda"), want_spectra=False)
        _, lm, _ = fm.forward(torch.tensor(minus, device="cuda"), want_spectra=False)
        fd = (lp.cpu().numpy() - lm.cpu().numpy()) / (2 * h)
        e = grad_err(g[b], fd)
        print(f"FD sample {b}: {e:.3e}")
        assert e < 1e-5
    fm.close()


def test_autograd_function_backward():
    from paper_2602_19687_amd import ExoLogLike, ForwardModel
    wl = reduced(1, n_nu=512, n_bins=16, batch=3)
    fm = ForwardModel(wl, precision="mixed", batch_max=3)
    th = torch.tensor(wl["params"], device="cuda", requires_grad=True)
    lnl = ExoLogLike.apply(th, fm, None)
    w = torch.tensor([0.5, -1.0, 2.0], device="cuda", dtype=torch.float64)
    (lnl * w).sum().backward()
    _, g, _, _ = fm.grad(th.detach())
    np.testing.assert_allclose(th.grad.cpu().numpy(), (w[:, None] * g).cpu().numpy(), rtol=1e-14)
    fm.close()


def test_invalid_samples_zero_gradient():
    wl = reduced(1, n_nu=300, n_bins=5, batch=3)
    th = wl["params"].copy()
    th[1, 3] = -0.01
    th[1, 4] = -0.3
    lnl, g, st, _ = _grad(wl, "mixed", th)
    assert st[1] != 0 and lnl[1] == -1e300 and np.all(g[1] == 0)
    assert st[0] == 0 and np.all(np.isfinite(g[0])) and np.any(g[0] != 0)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_ragged_layer_counts_after_full_call(prec):
    """Per-sample layer counts below the maximum, run right after a call in which
    every sample used all layers (nothing from the earlier call may leak in)."""
    from paper_2602_19687_amd import ForwardModel
    wl = reduced(3, n_nu=700, n_bins=14, batch=4, n_layers=110)
    fm = ForwardModel(wl, precision=prec, batch_max=4)
    th = torch.tensor(wl["params"], device="cuda")
    fm.grad(th)
    nl = np.array([110, 37, 64, 2], dtype=np.int32)
    print(f"[gpu] ragged grad prec={prec} n_layers={nl.tolist()}", flush=True)
    lnl, g, st, _ = fm.grad(th, n_layers=torch.tensor(nl, device="cuda"))
    g = g.cpu().numpy()
    st = st.cpu().numpy()
    fm.close()
    for b in range(4):
        gref = oracle.grad_complex_step(wl, wl["params"][b], n_layers=int(nl[b]))
        assert st[b] == 0
        e = grad_err(g[b], gref)
        print(f"ragged {prec} L={nl[b]}: grad err {e:.3e}")
        assert e < TOL[prec]


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_grad_up_to_150_layers(prec):
    """Padded layer count 160 (five 32-row blocks): the reduced-precision reverse
    kernel's 64-wavenumber, five-block shape, and the FP64 reverse kernel's
    32-wavenumber instance (its 64-wavenumber tile stops at 128 layers)."""
    wl = reduced(3, n_nu=700, n_bins=14, batch=4, n_layers=150)
    nl = np.array([150, 129, 97, 33], dtype=np.int32)
    lnl, g, st, lnl_f = _grad(wl, prec, wl["params"], n_layers=torch.tensor(nl, device="cuda"))
    for b in range(4):
        gref = oracle.grad_complex_step(wl, wl["params"][b], n_layers=int(nl[b]))
        assert st[b] == 0
        e = grad_err(g[b], gref)
        print(f"{prec} L={nl[b]} (L_pad 160): grad err {e:.3e}")
        assert e < TOL[prec]


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_c4_reduced_grad(prec):
    """High-resolution configuration (4 absorbers, 8x8 tables, 0.016 cm^-1 grid),
    cut to 1500 wavenumbers, per-sample layer counts of the configuration."""
    wl = reduced(4, n_nu=1500, n_bins=12, batch=3, n_layers=150, start=200000)
    nl = synth.workload(4, batch=3)["n_layers_per_sample"]
    lnl, g, st, _ = _grad(wl, prec, wl["params"], n_layers=torch.tensor(nl, device="cuda"))
    for b in range(3):
        gref = oracle.grad_complex_step(wl, wl["params"][b], n_layers=int(nl[b]))
        assert st[b] == 0
        e = grad_err(g[b], gref)
        print(f"c4 reduced {prec} L={nl[b]}: grad err {e:.3e}")
        assert e < TOL[prec]


# ---------------------------------------------------------------------------
# emission adjoint (reverse linear-in-tau sweep) and the PCHIP knot profile

def test_emission_grad_vs_complex_step():
    """Emission (8 absorbers, CIA, 5 PCHIP knots): every 20th wavenumber of the
    1-12 um grid with a ragged last tile; the reduced-precision adjoint against the
    oracle's complex-step gradient, every sample."""
    wl = reduced(2, n_nu=1000, n_bins=37, batch=6, step=20)
    lnl, g, st, lnl_f = _grad(wl, "mixed", wl["params"])
    assert np.array_equal(lnl, lnl_f)
    errs = []
    for b in range(len(wl["params"])):
        gref = oracle.grad_complex_step(wl, wl["params"][b])
        assert st[b] == 0
        e = grad_err(g[b], gref)
        errs.append(e)
        print(f"emission sample {b}: grad err {e:.3e}\n  gpu {g[b]}\n  ref {gref}")
    print(f"emission reduced: max grad err {max(errs):.3e}")
    assert max(errs) < TOL["mixed"]


def test_emission_grad_ragged_layers():
    from paper_2602_19687_amd import ForwardModel
    wl = reduced(2, n_nu=640, n_bins=16, batch=3, step=31, n_layers=130)
    nl = np.array([130, 71, 12], dtype=np.int32)
    fm = ForwardModel(wl, precision="mixed", batch_max=3)
    th = torch.tensor(wl["params"], device="cuda")
    fm.grad(th)
    print(f"[gpu] emission ragged grad n_layers={nl.tolist()}", flush=True)
    lnl, g, st, _ = fm.grad(th, n_layers=torch.tensor(nl, device="cuda"))
    g, st = g.cpu().numpy(), st.cpu().numpy()
    fm.close()
    for b in range(3):
        gref = oracle.grad_complex_step(wl, wl["params"][b], n_layers=int(nl[b]))
        assert st[b] == 0
        e = grad_err(g[b], gref)
        print(f"emission ragged L={nl[b]}: grad err {e:.3e}")
        assert e < TOL["mixed"]


def test_emission_fp64_grad_vs_complex_step():
    """The plain FP64 emission adjoint against the oracle's complex step at the
    FP64 tolerance: the reverse sweep, Planck sums and chain with no FP32 rounding."""
    wl = reduced(2, n_nu=700, n_bins=25, batch=4, step=28)
    lnl, g, st, lnl_f = _grad(wl, "fp64", wl["params"])
    assert np.array_equal(lnl, lnl_f)
    errs = []
    for b in range(4):
        gref = oracle.grad_complex_step(wl, wl["params"][b])
        assert st[b] == 0
        errs.append(grad_err(g[b], gref))
    print(f"emission fp64: max grad err {max(errs):.3e}")
    assert max(errs) < TOL["fp64"]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_emission_grad_up_to_150_layers(prec):
    """Emission at 160 padded layers: the FP64 forward then keeps only the optical
    depths in LDS (each angle's sweep forms the level intensities), and the FP64 and
    reduced-precision adjoints run past 128 layers; per-sample layer counts on both
    sides of 128."""
    from paper_2602_19687_amd import ForwardModel
    wl = reduced(2, n_nu=300, n_bins=10, batch=4, step=60, n_layers=150)
    nl = np.array([150, 129, 97, 33], dtype=np.int32)
    nl_t = torch.tensor(nl, device="cuda")
    lnl, g, st, lnl_f = _grad(wl, prec, wl["params"], n_layers=nl_t)
    assert np.array_equal(lnl, lnl_f)
    fm = ForwardModel(wl, precision=prec, batch_max=4)
    spec, _, _ = fm.forward(torch.tensor(wl["params"], dtype=torch.float64, device="cuda"), n_layers=nl_t)
    spec = spec.cpu().numpy()
    fm.close()
    stol = {"fp64": 1e-5, "mixed": 1e-4}[prec]
    for b in range(4):
        ref = oracle.forward(wl, wl["params"][b], n_layers=int(nl[b]))
        gref = oracle.grad_complex_step(wl, wl["params"][b], n_layers=int(nl[b]))
        assert st[b] == 0 and ref["status"] == 0
        es = np.max(np.abs(spec[b] - ref["spectrum"]) / np.abs(ref["spectrum"]))
        e = grad_err(g[b], gref)
        print(f"emission {prec} L={nl[b]} (L_pad 160): spectrum err {es:.3e}, grad err {e:.3e}")
        assert es < stol and e < TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_pchip_transmission_grad(prec):
    """Transmission with the 5-knot PCHIP profile: the knot gradient runs through
    the slopes' Jacobian of the shape-preserving rule."""
    wl = reduced(3, n_nu=900, n_bins=30, batch=5)
    cfg = {**synth.CONFIGS[3], "tp": synth.TP_PCHIP, "n_knots": 5}
    bounds = synth.param_bounds(cfg)
    u = np.random.default_rng(31).uniform(size=(5, len(bounds)))
    wl.update(tp=synth.TP_PCHIP, n_knots=5, param_bounds=bounds, param_names=synth.param_names(cfg),
              params=bounds[:, 0] + u * (bounds[:, 1] - bounds[:, 0]))
    lnl, g, st, _ = _grad(wl, prec, wl["params"])
    errs = []
    for b in range(5):
        gref = oracle.grad_complex_step(wl, wl["params"][b])
        assert st[b] == 0
        errs.append(grad_err(g[b], gref))
    print(f"pchip transmission {prec}: max grad err {max(errs):.3e}")
    assert max(errs) < TOL[prec]


def test_emission_grad_eight_angles_isothermal():
    """Emission with 8 Gauss-Legendre angles (the largest count) and an isothermal
    profile: the level and layer temperatures are one parameter."""
    wl = reduced(2, n_nu=500, n_bins=20, batch=3, step=40)
    cfg = {**synth.CONFIGS[2], "tp": synth.TP_ISOTHERMAL}
    bounds = synth.param_bounds(cfg)
    bounds[0] = (900.0, 2200.0)
    u = np.random.default_rng(41).uniform(size=(3, len(bounds)))
    wl.update(tp=synth.TP_ISOTHERMAL, n_mu=8, param_bounds=bounds, param_names=synth.param_names(cfg),
              params=bounds[:, 0] + u * (bounds[:, 1] - bounds[:, 0]))
    lnl, g, st, _ = _grad(wl, "mixed", wl["params"])
    for b in range(3):
        gref = oracle.grad_complex_step(wl, wl["params"][b])
        assert st[b] == 0
        e = grad_err(g[b], gref)
        print(f"emission iso n_mu=8 sample {b}: grad err {e:.3e}")
        assert e < TOL["mixed"]


def test_emission_full_size_grad_sampled():
    """The full emission workload (20000 wavenumbers, 8 absorbers, 100 layers) at
    B = 64, one sample against the oracle's complex-step gradient."""
    wl = synth.workload(2, batch=64)
    lnl, g, st, _ = _grad(wl, "mixed", wl["params"])
    b = 17
    gref = oracle.grad_complex_step(wl, wl["params"][b])
    e = grad_err(g[b], gref)
    print(f"emission full size sample {b}: grad err {e:.3e}")
    assert st[b] == 0 and e < TOL["mixed"]
    assert np.all(np.isfinite(g[st == 0]))


def test_emission_full_batch_grad_vs_fp64():
    """Every sample of the full emission batch (B = 1024, 20000 wavenumbers, 8
    absorbers, 100 layers, PCHIP knots): the reduced-precision gradient against
    the FP64 GPU adjoint (itself held to the oracle at 1e-5 in the tests above)
    at 1e-3 per component.  Samples near the best fit (lnL > 0, residuals at the
    noise level) are the most sensitive to the forward spectrum's rounding."""
    from paper_2602_19687_amd import ForwardModel
    wl = synth.workload(2)
    th = torch.tensor(wl["params"], dtype=torch.float64, device="cuda")
    print("[gpu] emission full batch B=1024, fp64 and mixed gradients", flush=True)
    out = {}
    for prec in ("fp64", "mixed"):
        fm = ForwardModel(wl, precision=prec, batch_max=1024)
        lnl, g, st, _ = fm.grad(th)
        torch.cuda.synchronize()
        out[prec] = (lnl.cpu().numpy(), g.cpu().numpy(), st.cpu().numpy())
        fm.close()
    l64, g64, s64 = out["fp64"]
    lmx, gmx, smx = out["mixed"]
    assert np.array_equal(s64, smx)
    ok = s64 == 0
    assert ok.sum() > 900
    scale = np.maximum(np.abs(g64[ok]), 1e-3 * np.max(np.abs(g64[ok]), axis=1, keepdims=True))
    per = np.max(np.abs(gmx[ok] - g64[ok]) / scale, axis=1)
    worst = int(np.nonzero(ok)[0][np.argmax(per)])
    print(f"emission full batch: max grad err {per.max():.3e} (sample {worst}, lnL {l64[worst]:.1f}), "
          f"median {np.median(per):.2e}, samples with lnL > 0: {int(np.sum(l64[ok] > 0))}")
    assert per.max() < 1e-3
    assert np.max(np.abs(lmx[ok] - l64[ok]) / np.abs(l64[ok])) < 1e-3


def test_ns_full_batch_grad_vs_fp64():
    """Every sample of the NS transmission batch (B = 1024, 30000 wavenumbers, 6
    absorbers, 100 layers): the reduced-precision gradient (FP16 tables) against
    the FP64 GPU adjoint (FP64 tables; held to the oracle at 1e-5 in the tests
    above) at 1e-3 per component, in the bench's launch configuration; and against
    the FP64 adjoint run on the tables as the reduced path stores them (decoded FP16
    entries), which leaves the arithmetic's share alone, at 1e-4.  Samples near the
    best fit carry the storage error: their residuals sit at the noise level."""
    from paper_2602_19687_amd import ForwardModel
    wl = synth.workload(1, batch=1024)
    xs, cia = oracle.decode_tables(wl)
    th = torch.tensor(wl["params"], dtype=torch.float64, device="cuda")
    print("[gpu] NS full batch B=1024, fp64 and mixed gradients", flush=True)
    out = {}
    for name, prec, w_ in (("fp64", "fp64", wl), ("fp64-decoded", "fp64", dict(wl, log10_xsec=xs, log10_cia=cia)),
                           ("mixed", "mixed", wl)):
        fm = ForwardModel(w_, precision=prec, batch_max=1024)
        if prec == "mixed":
            fm.set_tuning([1, 0, 4096, 16])
        lnl, g, st, _ = fm.grad(th)
        torch.cuda.synchronize()
        out[name] = (lnl.cpu().numpy(), g.cpu().numpy(), st.cpu().numpy())
        fm.close()
    ld, gd, sd = out["fp64-decoded"]
    assert np.array_equal(sd, out["mixed"][2])
    okd = sd == 0
    scd = np.maximum(np.abs(gd[okd]), 1e-3 * np.max(np.abs(gd[okd]), axis=1, keepdims=True))
    arith = np.max(np.abs(out["mixed"][1][okd] - gd[okd]) / scd)
    print(f"NS full batch: max grad err against the FP64 adjoint on the stored tables {arith:.3e}")
    assert arith < 1e-4
    l64, g64, s64 = out["fp64"]
    lmx, gmx, smx = out["mixed"]
    assert np.array_equal(s64, smx)
    ok = s64 == 0
    assert ok.sum() > 900
    scale = np.maximum(np.abs(g64[ok]), 1e-3 * np.max(np.abs(g64[ok]), axis=1, keepdims=True))
    rel = np.abs(gmx[ok] - g64[ok]) / scale
    per = np.max(rel, axis=1)
    worst = int(np.nonzero(ok)[0][np.argmax(per)])
    comp = int(np.argmax(rel[np.argmax(per)]))
    print(f"NS full batch: max grad err {per.max():.3e} (sample {worst}, component {comp}, lnL {l64[worst]:.1f}), "
          f"median {np.median(per):.2e}, samples with lnL > 0: {int(np.sum(l64[ok] > 0))}")
    assert per.max() < 1e-3
    assert np.max(np.abs(lmx[ok] - l64[ok]) / np.abs(l64[ok])) < 1e-3


def test_ns_size_grad_sampled():
    """The headline batch as the benchmark times it: the JWST-like transmission
    workload at B = 1024 (30000 wavenumbers, 100 layers, 12 parameters) with the
    launch choices [tiles fastest, 128 x 4 reverse shape, 4096 reverse items,
    16 layer-sum tiles] (4 wavenumber chunks per sample).  Four samples spread
    over the batch against the oracle: spectra, lnL and the gradient within 1e-3."""
    from paper_2602_19687_amd import ForwardModel
    wl = synth.workload(1, batch=1024)
    print("[gpu] NS-size gradient B=1024", flush=True)
    fm = ForwardModel(wl, precision="mixed", batch_max=1024)
    fm.set_tuning([1, 0, 4096, 16])
    th = torch.tensor(wl["params"], dtype=torch.float64, device="cuda")
    lnl, g, st, spec = fm.grad(th, want_spectra=True)
    torch.cuda.synchronize()
    lnl, g, st, spec = lnl.cpu().numpy(), g.cpu().numpy(), st.cpu().numpy(), spec.double().cpu().numpy()
    fm.close()
    worst = [0.0, 0.0, 0.0]
    for b in (0, 341, 682, 1023):
        ref = oracle.forward(wl, wl["params"][b])
        assert st[b] == ref["status"] == 0
        gref = oracle.grad_complex_step(wl, wl["params"][b])
        es = float(np.max(np.abs(spec[b] - ref["spectrum"]) / np.abs(ref["spectrum"])))
        el = abs(lnl[b] - ref["lnL"]) / abs(ref["lnL"])
        eg = grad_err(g[b], gref)
        print(f"NS b={b}: spectrum {es:.2e} lnL {el:.2e} grad {eg:.2e}", flush=True)
        worst = [max(worst[0], es), max(worst[1], el), max(worst[2], eg)]
    assert worst[0] < 1e-3 and worst[1] < 1e-3 and worst[2] < 1e-3, worst
