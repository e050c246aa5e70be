"""Launch choices, autotuning and graph replay on the GPU.

Every launch choice must give the oracle's results within the reduced-precision
tolerance (they differ from each other only in FP32 summation order); graph
replays must reproduce the eager calls bit for bit, replay after replay, with
eager work and synchronisations in between.
"""
import numpy as np
import pytest

import oracle
from parity_util import reduced

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-3


def grad_err(g, gref):
    scale = np.maximum(np.abs(gref), 1e-3 * np.max(np.abs(gref)))
    return np.max(np.abs(g - gref) / scale)


@pytest.fixture(scope="module")
def case():
    wl = reduced(3, n_nu=900, n_bins=30, batch=6)
    refs = [oracle.grad_complex_step(wl, wl["params"][b]) for b in range(6)]
    return wl, refs


def _model(wl, **kw):
    from paper_2602_19687_amd import ForwardModel
    return ForwardModel(wl, precision="mixed", batch_max=len(wl["params"]), **kw)


CHOICES = [
    [0, 0, 1024, 8], [1, 0, 1024, 8], [0, 1, 1024, 8], [0, 2, 1024, 8],
    [0, 0, 512, 4], [0, 0, 4096, 16], [1, 1, 2048, 16], [0, 1, 4096, 4], [1, 0, 4096, 32], [0, 2, 1024, 32],
    [1, 2, 4096, 64], [1, 0, 8192, 16],
]


@pytest.mark.parametrize("choice", CHOICES, ids=[",".join(map(str, c)) for c in CHOICES])
def test_every_launch_choice_matches_oracle(case, choice):
    wl, refs = case
    fm = _model(wl)
    print(f"[gpu] tuning {choice}", flush=True)
    fm.set_tuning(choice)
    assert fm.get_tuning() == choice
    th = torch.tensor(wl["params"], device="cuda")
    lnl, g, st, _ = fm.grad(th)
    g = g.cpu().numpy()
    errs = [grad_err(g[b], refs[b]) for b in range(6)]
    print(f"tuning {choice}: max grad err {max(errs):.3e}")
    assert max(errs) < TOL
    fm.close()


def test_invalid_choices_rejected(case):
    from paper_2602_19687_amd import _lib as L
    wl, _ = case
    fm = _model(wl)
    before = fm.get_tuning()
    for bad in ([2, 0, 1024, 8], [0, 3, 1024, 8], [0, 0, 1000, 8], [0, 0, 1024, 5]):
        with pytest.raises(L.ExoError):
            fm.set_tuning(bad)
        assert fm.get_tuning() == before
    fm.close()


def test_autotune_and_cache(case, tmp_path):
    wl, refs = case
    cache = str(tmp_path / "tune.txt")
    fm = _model(wl)
    print("[gpu] autotune", flush=True)
    t1 = fm.autotune(6, cache_path=cache)
    text = open(cache).read().split()
    assert len(text) == 5 and [int(x) for x in text[1:]] == t1
    lnl, g, st, _ = fm.grad(torch.tensor(wl["params"], device="cuda"))
    g = g.cpu().numpy()
    assert max(grad_err(g[b], refs[b]) for b in range(6)) < TOL
    fm.close()
    # a second context takes the cached choice without timing
    fm2 = _model(wl)
    fm2.set_tuning([1 - t1[0], t1[1], t1[2], t1[3]])
    assert fm2.autotune(6, cache_path=cache) == t1
    fm2.close()


@pytest.mark.parametrize("ragged", [False, True], ids=["uniform", "ragged"])
@pytest.mark.parametrize("kind", ["forward", "grad"])
def test_graph_replays_match_eager(case, kind, ragged):
    """Replays equal eager calls bit for bit; with ragged layer counts each replay
    reads new per-sample counts (2-100) from the same buffer, so the captured
    launches serve any mix of layer grids."""
    wl, _ = case
    rng = np.random.default_rng(7)
    thetas = [wl["params"] * (1.0 + 1e-3 * rng.standard_normal(wl["params"].shape)) for _ in range(3)]
    thetas = [np.where(np.abs(t) > 0, t, 0.0) for t in thetas]
    layers = [rng.integers(2, wl["n_layers"] + 1, size=len(wl["params"])).astype(np.int32) if ragged else None
              for _ in range(3)]
    eager = _model(wl)
    graph = _model(wl)
    graph.set_graphs(True)
    print(f"[gpu] graph replay {kind} ragged={ragged}", flush=True)
    for rep in range(3):
        for th_np, nl in zip(thetas, layers):
            th = torch.tensor(th_np, device="cuda")
            if kind == "forward":
                a = eager.forward(th, n_layers=nl)
                b = graph.forward(th, n_layers=nl)
            else:
                a = eager.grad(th, n_layers=nl, want_spectra=True)
                b = graph.grad(th, n_layers=nl, want_spectra=True)
            # eager work and a synchronisation between replays
            junk = torch.randn(1 << 20, device="cuda").sum()
            torch.cuda.synchronize()
            for x, y in zip(a, b):
                assert torch.equal(x, y), (rep, kind)
            assert torch.isfinite(junk)
    assert len(graph._gbuf) == 1
    eager.close()
    graph.close()


def test_graph_mode_rejects_null_stream(case):
    from paper_2602_19687_amd import _lib as L
    import ctypes as C
    wl, _ = case
    fm = _model(wl)
    L.check(fm.lib.exofwd_set_graphs(fm.ctx, 1), fm.ctx, "set_graphs")
    th = torch.tensor(wl["params"], device="cuda")
    lnl = torch.empty(6, dtype=torch.float64, device="cuda")
    st = fm.lib.exofwd_forward(fm.ctx, 6, C.c_void_p(th.data_ptr()), None, None,
                               C.c_void_p(lnl.data_ptr()), None, None)
    assert st == 1   # EXOFWD_ERR_ARG
    fm.close()


@pytest.fixture(scope="module")
def ragged_case():
    # padded to 160 layers, layer counts on both sides of 128 (the two classes), with
    # invalid-free prior draws of the grey-deck transmission setup
    wl = reduced(3, n_nu=700, n_bins=20, batch=6, n_layers=150)
    nl = np.array([150, 64, 129, 128, 97, 140], dtype=np.int32)
    refs = [oracle.grad_complex_step(wl, wl["params"][b], n_layers=int(nl[b])) for b in range(6)]
    specs = [oracle.forward(wl, wl["params"][b], n_layers=int(nl[b]))["spectrum"] for b in range(6)]
    return wl, nl, refs, specs


@pytest.mark.parametrize("choice", [[1, 1, 4096, 16], [1, 2, 4096, 16], [0, 1, 1024, 64], [1, 1, 8192, 8],
                                    [1, 0, 4096, 16], [0, 0, 512, 64], [0, 0, 2048, 64]],
                         ids=["split", "unsplit", "split-samples-fastest", "split-8192", "split-128",
                              "split-128-512", "split-128-2048"])
def test_layer_classes_match_oracle(ragged_case, choice):
    """A ragged batch of more than 128 padded layers: the forward kernel runs the
    samples of at most 128 layers and the rest as two classes, and reverse shapes 0
    and 1 do the same (128 x 4 or 64 x 4, then 64 x 5, with equal chunk counts);
    every choice agrees with the oracle."""
    wl, nl, refs, specs = ragged_case
    fm = _model(wl)
    print(f"[gpu] layer classes {choice}", flush=True)
    fm.set_tuning(choice)
    th = torch.tensor(wl["params"], device="cuda")
    lnl, g, st, sp = fm.grad(th, n_layers=nl, want_spectra=True)
    g, st, sp = g.cpu().numpy(), st.cpu().numpy(), sp.double().cpu().numpy()
    fm.close()
    assert np.all(st == 0)
    serr = max(float(np.max(np.abs(sp[b] - specs[b]) / np.abs(specs[b]))) for b in range(6))
    gerr = max(grad_err(g[b], refs[b]) for b in range(6))
    print(f"layer classes {choice}: spectrum {serr:.2e}, gradient {gerr:.2e}")
    assert serr < TOL and gerr < TOL
