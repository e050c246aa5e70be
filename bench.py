"""Benchmark: batched transmission forward model + adjoint on one MI355X.

Workload: JWST-like transmission (6 absorbers x 20 T x 20 log p x 30000
wavenumbers, 100 layers, reduced Guillot profile, CIA, Rayleigh, grey cloud,
400 bins, 12 parameters) at B = 1024 parameter samples per step.  A step is
one call of the whole hot path (profile, fused opacity + chord + transit depth,
likelihood, and the adjoint to d lnL / d params) on inputs already resident in
HBM.  The reduced-precision path (FP16 tables, FP32 opacity, bf16x3 MFMA chord,
FP64 profile and likelihood) is the measured value; the plain FP64 path is
timed beside it, and the FP64 oracle on the host cores gives the CPU baseline.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# published MI355X FP32 vector peak (256 CU x 4 SIMD x 16 lanes x 2.4 GHz x 2 (FMA) x 2 (packed));
# this build disables packed FP32, so its attainable ceiling is half of it
FP32_VECTOR_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0   # dense


def algorithmic_bytes_per_sample(L, S, n_nu, b_tab, b_out):
    """Table entries the method must gather per sample (4 bilinear corners per
    layer, species and wavenumber; 2 T corners for each of 2 CIA pairs), the
    Rayleigh axis and the output spectrum."""
    return (4 * L * S * n_nu + 4 * L * n_nu) * b_tab + 2 * n_nu * 4 + n_nu * b_out


def kernel_model(kernel, Ls, S, n_nu, n_mu=4, ck_mix=0):
    """Roofline model of one launch of a hot kernel over samples with layer
    counts Ls, S sources and n_nu wavenumbers: (bound, algorithmic amount, peak, unit).

    trans_fwd, layer_sums: vector FP32 operations per (sample, layer, wavenumber),
    counting an FMA as 2 and an exp2 as 1, against the FP32 vector peak:
      trans_fwd  : line source bilinear (4 FMA) + offset add + exp2 + accumulate = 11 per
                   source, CIA pair T lerp (2 FMA) + add + exp2 + accumulate = 7 per pair,
                   Rayleigh + deck 1 FMA = 2, transit exp2 + FMA = 3   -> 11 S + 19
      layer_sums : line source 20 (forward 11, T-weight derivative 2 sub + 2 FMA,
                   2 FMA into the sums), CIA pair 11, Rayleigh + deck sums 4 -> 20 S + 26
    trans_adj: the three triangular products tau = P dtau, Pbar = tau_bar dtau^T and
    dtau_bar = P^T tau_bar, L(L+1)/2 FMA each per wavenumber, each done as three bf16
    MFMA products (bf16x3), against the dense bf16 MFMA peak."""
    import numpy as np
    Ls = np.asarray(Ls, dtype=np.int64)
    elems = int(Ls.sum()) * n_nu
    if kernel == "trans_fwd":
        return "alu", (11 * S + 19) * elems, FP32_VECTOR_PEAK_TFLOPS, "TFLOP/s"
    if kernel == "layer_sums":
        return "alu", (20 * S + 26) * elems, FP32_VECTOR_PEAK_TFLOPS, "TFLOP/s"
    if kernel == "emis_fwd":
        # opacity as in trans_fwd without Rayleigh and deck (11 S + 14), Planck at the levels (5), and per
        # Gauss angle the sweep step x = dtau/mu, exp, linear-source update (12)
        return "alu", (11 * S + 14 + 5 + 12 * n_mu) * elems, FP32_VECTOR_PEAK_TFLOPS, "TFLOP/s"
    if kernel == "trans_adj":
        return "mfma", 3 * 3 * int((Ls * (Ls + 1) // 2).sum()) * 2 * n_nu, BF16_MFMA_PEAK_TFLOPS, "TFLOP/s"
    if kernel == "ck_mix":
        # per (sample, layer, bin): S x 8 interpolations (4 FMA + add + exp2 = 10), then S - 1
        # random-overlap merges of 64 pairs: pair sum (1), the merge of the eight sorted
        # rows of the pair matrix (three bitonic merge levels, 15 steps of 32
        # compare-exchanges, min + max), two 64-long running sums (128) and the rebinning
        # (7 edges x FMA + 8 differences x multiply = 22), and the continuum (11)
        per_merge = 64 + 15 * 32 * 2 + 128 + 22
        return "alu", int(Ls.sum()) * n_nu * (S * 8 * 10 + (S - 1) * per_merge + 11), FP32_VECTOR_PEAK_TFLOPS, "TFLOP/s"
    if kernel == "ck_spectrum":
        # the chord over the (bin, g-point) columns: L(L+1)/2 FMA per column as three bf16 MFMA products
        # (RORR: 8 columns per bin; product of transmissions: 64, one per absorber slot and g-point)
        cols = n_nu * (8 if ck_mix == 0 else 64)
        return "mfma", 3 * int((Ls * (Ls + 1) // 2).sum()) * 2 * cols, BF16_MFMA_PEAK_TFLOPS, "TFLOP/s"
    if kernel == "ck_spectrum_emis":
        # per (layer, bin, g-point): Planck at the level (10) and per angle the sweep step (12)
        return "alu", int(Ls.sum()) * n_nu * 8 * (10 + 12 * n_mu), FP32_VECTOR_PEAK_TFLOPS, "TFLOP/s"
    raise ValueError(kernel)


def source_digest(hip_name):
    """SHA-256 over one kernel source file and the csrc headers it includes
    (transitively); a counter summary records it per kernel, so a change to one
    kernel's sources voids only that kernel's figures."""
    import hashlib
    import re
    csrc = os.path.join(ROOT, "paper_2602_19687_amd", "csrc")
    seen, todo = set(), [hip_name]
    while todo:
        name = todo.pop()
        if name in seen or not os.path.exists(os.path.join(csrc, name)):
            continue
        seen.add(name)
        with open(os.path.join(csrc, name)) as f:
            todo += re.findall(r'^#include "([^"]+)"', f.read(), flags=re.M)
    d = hashlib.sha256()
    for name in sorted(seen):
        with open(os.path.join(csrc, name), "rb") as f:
            d.update(name.encode() + b"\0" + f.read())
    return d.hexdigest()


def measured_traffic(kernel, workload_tag="transmission_ns_b1024"):
    """HBM bytes per launch of `kernel` from the committed PMC summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by a copy-kernel calibration), or
    None when the summary is missing or the kernel's sources have changed since
    (each line names the source file and its digest)."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload_tag}.md")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        for line in f:
            if line.startswith("traffic_bytes_per_launch:"):
                parts = line.split(":", 1)[1].split()
                if len(parts) == 4 and parts[0] == kernel:
                    return float(parts[1]) if source_digest(parts[2]) == parts[3] else None
    return None


def measured_sq(kernel, workload_tag="transmission_ns_b1024"):
    """(VALU instructions per SIMD and cycle, MFMA busy fraction) of `kernel` from the
    committed SQ counter summary, or None when it is missing or the kernel's sources
    have changed since."""
    path = os.path.join(ROOT, "profiles", f"sq_counters_{workload_tag}.md")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        for line in f:
            if line.startswith("sq_per_launch:"):
                parts = line.split(":", 1)[1].split()
                if len(parts) == 5 and parts[0] == kernel:
                    return (float(parts[1]), float(parts[2])) if source_digest(parts[3]) == parts[4] else None
    return None


_WL = {}


def spec_err(a, ref):
    """Largest relative spectrum error, each point relative to max(|ref|, 1e-12 x the
    sample's peak |ref|): points far below that carry nothing at any observational
    precision, and the fluxes of cold isolated objects can fall below FP32's normal
    range (1.2e-38) there."""
    import numpy as np
    a, ref = np.atleast_2d(a), np.atleast_2d(ref)
    floor = 1e-12 * np.max(np.abs(ref), axis=1, keepdims=True)
    return float(np.max(np.abs(a - ref) / np.maximum(np.abs(ref), floor)))

TP_KINDS = {"barstow": 3, "milne": 4, "guillot7": 5}


def with_tp(wl, cid, tp_name):
    """The workload with its T-p profile replaced (Barstow, modified Milne or the
    seven-parameter modified Guillot form): the T-p parameters are drawn from that
    profile's prior bounds, every other parameter keeps the workload's own draw."""
    if not tp_name:
        return wl
    import numpy as np
    import synth
    tp = TP_KINDS[tp_name]
    cfg = {**synth.CONFIGS[cid], "tp": tp}
    names, bounds = synth.param_names(cfg), synth.param_bounds(cfg)
    n_new = next(i for i, n in enumerate(names) if n.startswith("log10_X_"))
    n_old = next(i for i, n in enumerate(wl["param_names"]) if n.startswith("log10_X_"))
    B = wl["params"].shape[0]
    u = np.random.default_rng([19687, cid, 7, tp]).uniform(size=(B, n_new))
    tp_par = bounds[:n_new, 0] + u * (bounds[:n_new, 1] - bounds[:n_new, 0])
    out = dict(wl)
    out.update(tp=tp, param_names=names, param_bounds=bounds,
               params=np.concatenate([tp_par, wl["params"][:, n_old:]], axis=1))
    return out


def with_bd(wl, cid, on):
    """The emission workload as an isolated object (Eqs. 46-47): log10 g and M_bd are
    drawn from their prior bounds and placed where the parameter layout puts them;
    the observations are a flat flux of the objects' order (timing only)."""
    if not on:
        return wl
    import numpy as np
    import synth
    cfg = {**synth.CONFIGS[cid], "tp": wl["tp"], "bd": True}
    names, bounds = synth.param_names(cfg), synth.param_bounds(cfg)
    B = wl["params"].shape[0]
    u = np.random.default_rng([19687, cid, 8]).uniform(size=(B, 2))
    extra = bounds[-2:, 0] + u * (bounds[-2:, 1] - bounds[-2:, 0])
    out = dict(wl)
    k = len(wl["bin_lo"])
    col = {n: wl["params"][:, i] for i, n in enumerate(wl["param_names"])}
    col.update(log10_g_cgs=extra[:, 0], M_bd_MJup=extra[:, 1])
    out.update(bd=True, param_names=names, param_bounds=bounds, params=np.stack([col[n] for n in names], axis=1),
               y_obs=np.full(k, 1.0e-16), y_err=np.full(k, 1.0e-17))
    return out


def _oracle_init(cid, batch, tp_name=None, bd=False, ck_mix=None):
    os.environ["OMP_NUM_THREADS"] = "1"
    import synth
    _WL["wl"] = with_bd(with_tp(synth.workload(cid, batch=batch), cid, tp_name), cid, bd)
    if ck_mix is not None:
        _WL["wl"] = dict(_WL["wl"], ck_mix=ck_mix)


def _oracle_worker(args):
    idx, do_grad = args
    import oracle
    wl = _WL["wl"]
    th = wl["params"][idx]
    t0 = time.perf_counter()
    out = oracle.forward(wl, th)
    t_fwd = time.perf_counter() - t0
    g = oracle.grad_complex_step(wl, th) if do_grad else None
    return idx, out["spectrum"], out["lnL"], g, time.perf_counter() - t0, t_fwd


def cpu_baseline(cid, batch, n_samples, do_grad, tp_name=None, bd=False, ck_mix=None):
    """Time the FP64 oracle, as it stands, on a bounded sample of the workload on
    the host cores: one sample per task, one BLAS thread per worker process;
    throughput = samples / (summed per-sample seconds / workers)."""
    cores = min(16, os.cpu_count() or 1)
    idx = list(range(0, batch, max(1, batch // n_samples)))[:n_samples]
    workers = min(cores, len(idx))
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers, initializer=_oracle_init, initargs=(cid, batch, tp_name, bd, ck_mix)) as pool:
        res = pool.map(_oracle_worker, [(i, do_grad) for i in idx], chunksize=1)
    busy = sum(r[4] for r in res)
    busy_fwd = sum(r[5] for r in res)
    return [r[:4] for r in res], busy / workers, workers, busy, busy_fwd


def cpu_model():
    """The host CPU's model name (Linux), or the platform's processor string."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=1, choices=(1, 2, 4, 5, 6, 7, 8),
                    help="1: the JWST-like transmission batch (default); 2: the emission batch (forward); "
                         "4: the high-resolution ragged batch; 5: the transmission batch with a non-grey cloud; "
                         "6: as 5 with a partly cloudy limb (two spectra per sample); 7: correlated-k transmission "
                         "(forward); 8: correlated-k emission (forward)")
    ap.add_argument("--batch", type=int, default=None,
                    help="default 1024 (configs 1, 2, 5, 6), 64 (config 4) or 256 (configs 7, 8)")
    ap.add_argument("--ck-mix", type=int, default=None, choices=(0, 1),
                    help="correlated-k transmission mixing: 0 random overlap with resorting and rebinning, "
                         "1 product of transmission functions (config 7's default)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tuning", type=str, default=None,
                    help="launch choices a,b,c,d to use instead of autotuning (see exofwd_set_tuning)")
    ap.add_argument("--no-graphs", action="store_true")
    ap.add_argument("--tp", choices=sorted(TP_KINDS), default=None,
                    help="replace the workload's T-p profile (Barstow, modified Milne, 7-parameter modified Guillot)")
    ap.add_argument("--bd", action="store_true",
                    help="emission batch (--config 2) as isolated objects: retrieved gravity and mass, flux at 10 pc")
    ap.add_argument("--cpu-samples", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy 5 times (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the path shards by samples with no exchange, "
              "and multi-GPU runs are not part of this build", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4, "launches": 5}))
        return

    import synth
    from paper_2602_19687_amd import ForwardModel

    cid = args.config
    B = args.batch or (64 if cid == 4 else 256 if cid in (7, 8) else 1024)
    ck = cid in (7, 8)
    t_setup = time.perf_counter()
    if args.bd and cid != 2:
        print("--bd applies to the emission batch (--config 2)", file=sys.stderr)
        sys.exit(2)
    wl = with_bd(with_tp(synth.workload(cid, batch=B), cid, args.tp), cid, args.bd)
    if ck and args.ck_mix is not None:
        wl = dict(wl, ck_mix=args.ck_mix)
    L_, S, n_nu = wl["n_layers"], wl["n_species"], len(wl["nu"])
    th = torch.tensor(wl["params"], dtype=torch.float64, device="cuda")
    nl_np = wl["n_layers_per_sample"]
    nl = torch.tensor(nl_np, dtype=torch.int32, device="cuda") if nl_np is not None else None
    Ls = nl_np if nl_np is not None else np.full(B, L_)
    print(f"[bench] workload ready in {time.perf_counter() - t_setup:.1f}s", file=sys.stderr, flush=True)

    # measured HBM copy peak: a 1 GiB device-to-device copy (read + write) timed with events
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(5):
        dst.copy_(src)
    c1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * src.numel() * 4 / (c0.elapsed_time(c1) / 5 / 1e3) / 1e9
    del src, dst
    torch.cuda.empty_cache()

    def run(prec, steps, warmup, want_grad=True):
        fm = ForwardModel(wl, precision=prec, batch_max=B)
        has_grad = fm.has_grad and want_grad
        tuning = None
        if prec == "mixed" and args.tuning:
            fm.set_tuning([int(x) for x in args.tuning.split(",")])
            tuning = fm.get_tuning()
        elif prec == "mixed" and not args.no_autotune:
            t0 = time.perf_counter()
            tuning = fm.autotune(B, th, nl)
            print(f"[bench] autotune {tuning} in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
        step = (lambda: fm.grad(th, n_layers=nl)) if has_grad else (lambda: fm.forward(th, n_layers=nl, want_spectra=False))
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        fm.set_profiling(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            out = step()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        kern = {k: fm.kernel_time(k) for k in ("profile", "trans_fwd", "emis_fwd", "ck_mix", "ck_spectrum", "loglike",
                                               "trans_adj", "emis_adj", "layer_sums", "chain")}
        fm.set_profiling(False)
        graph_ms = graph_pct = None
        if not args.no_graphs:
            # the same step captured once into a hipGraph and replayed; the replays run
            # on a side stream ordered with torch's current stream, so events recorded
            # on the current stream bracket each replay
            fm.set_graphs(True)
            step()
            torch.cuda.synchronize()
            evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
            t0 = time.perf_counter()
            for e0, e1 in evs:
                e0.record()
                step()
                e1.record()
            torch.cuda.synchronize()
            graph_ms = (time.perf_counter() - t0) / steps * 1e3
            per_step = np.array([e0.elapsed_time(e1) for e0, e1 in evs])
            graph_pct = [float(np.percentile(per_step, q)) for q in (50, 10, 90)]
            fm.set_graphs(False)
        spec, lnl, status = fm.forward(th, n_layers=nl)
        torch.cuda.synchronize()
        res = dict(ms_per_step=dt / steps * 1e3, has_grad=has_grad, kernels=kern, graph_ms=graph_ms, graph_pct=graph_pct,
                   tuning=tuning,
                   spec=spec.double().cpu().numpy(), lnl=lnl.cpu().numpy(), status=status.cpu().numpy(),
                   grad=out[1].cpu().numpy() if has_grad else None, bytes=fm.device_bytes())
        fm.close()
        return res

    # the emission batch is quoted as a forward rate (its FP64 path has no adjoint); its
    # reduced-precision forward+gradient step is timed beside it
    mixed = run("mixed", args.steps, args.warmup, want_grad=cid not in (2, 7, 8))
    print(f"[bench] mixed {mixed['ms_per_step']:.2f} ms/step", file=sys.stderr, flush=True)
    emis_grad = emis_grad64 = fwd_only = None
    if cid in (1, 4, 5, 6):
        # the forward model alone beside the forward+gradient step
        fwd_only = run("mixed", max(2, args.steps // 2), 1, want_grad=False)
        print(f"[bench] mixed forward {fwd_only['ms_per_step']:.2f} ms/step", file=sys.stderr, flush=True)
    if cid == 2:
        emis_grad = run("mixed", max(2, args.steps // 2), 1, want_grad=True)
        print(f"[bench] mixed forward+grad {emis_grad['ms_per_step']:.2f} ms/step", file=sys.stderr, flush=True)
        if not args.no_fp64:
            emis_grad64 = run("fp64", 2, 1, want_grad=True)
            print(f"[bench] fp64 forward+grad {emis_grad64['ms_per_step']:.2f} ms/step", file=sys.stderr, flush=True)
    fp64 = fp64_fwd = None
    if not args.no_fp64 and cid in (1, 2, 4):
        fp64 = run("fp64", max(2, args.steps // 4), 1, want_grad=cid != 2)
        print(f"[bench] fp64 {fp64['ms_per_step']:.2f} ms/step", file=sys.stderr, flush=True)
    if not args.no_fp64 and cid in (1, 4):
        # the plain FP64 forward model alone, beside the reduced-precision forward alone
        fp64_fwd = run("fp64", 2, 1, want_grad=False)
        print(f"[bench] fp64 forward {fp64_fwd['ms_per_step']:.2f} ms/step", file=sys.stderr, flush=True)
    ck_other = None
    if cid == 7:
        # the other mixing of the absorbers, timed beside the configured one
        other = 1 - int(wl["ck_mix"])
        wl_main = wl
        wl = dict(wl, ck_mix=other)
        ck_other = run("mixed", max(2, args.steps // 2), 1, want_grad=False)
        ck_other["ck_mix"] = other
        wl = wl_main
        print(f"[bench] ck mix {other}: {ck_other['ms_per_step']:.2f} ms/step", file=sys.stderr, flush=True)

    value = B / (mixed["ms_per_step"] / 1e3)
    # dominant kernel of the step by time
    per = {k: v[0] / max(1, v[1]) for k, v in mixed["kernels"].items() if v[1]}
    hot = ("emis_fwd",) if cid == 2 else ("ck_mix", "ck_spectrum") if ck else ("trans_fwd", "trans_adj", "layer_sums")
    dom = max(hot, key=lambda k: per.get(k, 0.0))
    dom_ms = per[dom]
    tag = ("transmission_ns_b1024" if (cid == 1 and B == 1024) else
           f"emission_c2_b{B}" if cid == 2 else f"ck_c{cid}_b{B}" if ck else f"transmission_c{cid}_b{B}")
    ck_mix = int(wl.get("ck_mix", 0))

    def model_of(k):
        if k == "ck_spectrum" and wl["mode"] == 1:
            return kernel_model("ck_spectrum_emis", Ls, S, n_nu)
        return kernel_model(k, Ls, S, n_nu, ck_mix=ck_mix)
    bound, amount, peak, unit = model_of(dom)
    achieved = amount / (dom_ms / 1e3) / 1e12
    traffic = measured_traffic(dom, tag)
    alg_bytes = sum(algorithmic_bytes_per_sample(int(l), S, n_nu, 2, 4) for l in Ls)
    roofline = {"bound": bound, "achieved": round(achieved, 2), "peak": peak, "unit": unit,
                "frac": round(achieved / peak, 4), "traffic": traffic,
                "kernel": dom, "kernel_ms": round(dom_ms, 4), "flops_per_launch": amount}
    for k in hot:
        if k in per:
            bk, ak, pk, _ = model_of(k)
            a = ak / (per[k] / 1e3) / 1e12
            tr = measured_traffic(k, tag)
            sq = measured_sq(k, tag)
            roofline.setdefault("kernels", {})[k] = {"bound": bk, "ms": round(per[k], 4), "achieved": round(a, 2),
                                                     "peak": pk, "frac": round(a / pk, 4), "traffic": tr,
                                                     "traffic_gbs": round(tr / (per[k] / 1e3) / 1e9, 1) if tr else None,
                                                     "valu_ipc": sq[0] if sq else None,
                                                     "mfma_busy": sq[1] if sq else None}
    # table-gather bytes the method needs (the forward pass) per launch time: an algorithmic
    # rate, not HBM traffic (the tables stay in the 256 MB MALL across samples; rocprof's
    # counters give the HBM bytes, `traffic` above)
    fwd_kernel = "emis_fwd" if cid == 2 else ("ck_mix" if ck_mix == 0 else "ck_spectrum") if ck else "trans_fwd"
    if cid == 2:   # FP32 table entries
        alg_bytes = sum((4 * int(l) * S * n_nu + 4 * int(l) * n_nu) * 4 + n_nu * 4 for l in Ls)
    elif ck:       # FP32 k-table entries at 8 g-points, CIA at the bin centres
        alg_bytes = sum((4 * int(l) * S * n_nu * 8 + 4 * int(l) * n_nu) * 4 + n_nu * 4 for l in Ls)
    gather_gbs = alg_bytes / (per[fwd_kernel] / 1e3) / 1e9
    roofline["table_gather"] = {"bytes_per_launch": alg_bytes, "kernel": fwd_kernel,
                                "algorithmic_gbs": round(gather_gbs, 1),
                                "algorithmic_over_hbm_peak": round(gather_gbs / HBM_PEAK_GBS, 4),
                                "copy_peak_gbs": round(copy_gbs, 1),
                                "note": "table reuse across samples is served from the MALL and L2, so a ratio "
                                        "above 1 is no HBM figure; the opacity kernels are bound by the VALU"}

    if cid == 1:
        workload = ("jwst-like transmission, 6 absorbers, 20x20x30000 FP16 tables, 100 layers, 400 bins, 12 params")
    elif cid == 2:
        workload = ("emission, 8 absorbers, 20x20x20000 FP32 tables, 100 layers, 4 Gauss-Legendre angles, "
                    "5-knot PCHIP profile, 400 bins")
    elif cid == 5:
        workload = ("jwst-like transmission with a non-grey cloud (power-law condensate profile, fitted Q_ext with "
                    f"a mid-IR feature), 6 absorbers, 20x20x30000 FP16 tables, 100 layers, 400 bins, {th.shape[1]} params")
    elif cid == 6:
        workload = ("jwst-like transmission with a partly cloudy limb (cloudy and clear spectra mixed by f_cld; "
                    "non-grey slab cloud, fitted Q_ext), 6 absorbers, 20x20x30000 FP16 tables, 100 layers, 400 bins, "
                    f"{th.shape[1]} params")
    elif cid == 7:
        workload = (f"correlated-k transmission, 6 absorbers, 20x20 k-tables on {n_nu} R=1000 bins x 8 g-points, "
                    f"100 layers, 400 bins, {th.shape[1]} params, "
                    + ("random overlap with resorting and rebinning" if ck_mix == 0 else
                       "product of the absorbers' transmission functions"))
    elif cid == 8:
        workload = (f"correlated-k emission, 8 absorbers, 20x20 k-tables on {n_nu} R=1000 bins x 8 g-points, "
                    f"100 layers, 4 Gauss-Legendre angles, 5-knot PCHIP profile, 400 bins, random overlap with "
                    f"resorting and rebinning")
    else:
        workload = (f"high-resolution transmission, 4 absorbers, 8x8x400000 FP16 tables, {int(Ls.min())}-{int(Ls.max())} "
                    f"layers per sample, 400 bins, {th.shape[1]} params")
    if args.tp:
        names = {"barstow": "Barstow 2020", "milne": "modified Milne", "guillot7": "7-parameter modified Guillot"}
        workload += f"; T-p profile replaced by the {names[args.tp]} profile ({th.shape[1]} params)"
    if args.bd:
        workload += f"; isolated objects at 10 pc, log10 g and mass retrieved ({th.shape[1]} params)"
    out = {
        "metric": ("forward+grad spectra/sec at B=1024 (FP32/FP16 vs FP64 plain), max rel err"
                   if mixed["has_grad"] else "forward spectra/sec at B=1024 (FP32/FP16 vs FP64 plain), max rel err")
        if cid == 1 else (f"emission forward spectra/sec at B={B} (FP32 vs FP64 plain)" if cid == 2 else
                          f"correlated-k forward spectra/sec at B={B} (FP32)" if ck else
                          f"forward+grad spectra/sec, non-grey cloud transmission batch B={B} (FP32/FP16)" if cid == 5
                          else f"forward+grad spectra/sec, partly cloudy transmission batch B={B} (FP32/FP16)"
                          if cid == 6 else f"forward+grad spectra/sec, high-resolution ragged batch B={B} (FP32/FP16)"),
        "value": round(value, 1), "unit": "spectra/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(mixed["ms_per_step"], 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": workload, "batch": B, "n_nu": n_nu, "n_layers": L_ if nl_np is None else
                   f"{int(Ls.min())}-{int(Ls.max())} (mean {float(Ls.mean()):.1f})", "n_species": S,
                   "precision": ("fp32 tables / fp32 opacity / fp32 sweep, fp64 intensities / fp64 profile+lnL"
                                 if cid == 2 else
                                 "fp32 k-tables / fp32 mixing / " + ("fp32 sweep, fp64 intensities" if cid == 8 else
                                                                     "bf16x3 mfma chord") + " / fp64 profile+lnL"
                                 if ck else "fp16 tables / fp32 opacity / bf16x3 mfma chord / fp64 profile+lnL"),
                   "launch_choices": mixed["tuning"]},
        "roofline": roofline,
        "kernel_ms_per_step": {k: round(v[0] / max(1, v[1]), 4) for k, v in mixed["kernels"].items() if v[1]},
    }
    if fwd_only is not None:
        out["forward_only"] = {"spectra_per_s": round(B / (fwd_only["ms_per_step"] / 1e3), 1),
                               "ms_per_step": round(fwd_only["ms_per_step"], 4),
                               "launch_choices": fwd_only["tuning"],
                               "kernel_ms_per_step": {k: round(v[0] / max(1, v[1]), 4)
                                                      for k, v in fwd_only["kernels"].items() if v[1]}}
    if emis_grad is not None and emis_grad["has_grad"]:
        out["forward_grad"] = {"spectra_per_s": round(B / (emis_grad["ms_per_step"] / 1e3), 1),
                               "ms_per_step": round(emis_grad["ms_per_step"], 4),
                               "kernel_ms_per_step": {k: round(v[0] / max(1, v[1]), 4)
                                                      for k, v in emis_grad["kernels"].items() if v[1]}}
        if emis_grad64 is not None and emis_grad64["has_grad"]:
            out["forward_grad"]["fp64_ms_per_step"] = round(emis_grad64["ms_per_step"], 3)
            out["forward_grad"]["speedup_vs_fp64"] = round(emis_grad64["ms_per_step"] / emis_grad["ms_per_step"], 3)
            ok = (emis_grad["status"] == 0) & (emis_grad64["status"] == 0)
            gm, g64 = emis_grad["grad"][ok], emis_grad64["grad"][ok]
            scale = np.maximum(np.abs(g64), 1e-3 * np.max(np.abs(g64), axis=1, keepdims=True))
            out["forward_grad"]["max_grad_err_vs_fp64_gpu"] = float(np.max(np.abs(gm - g64) / scale))
    if mixed["graph_ms"] is not None:
        out["graph_replay"] = {"ms_per_step": round(mixed["graph_ms"], 4),
                               "spectra_per_s": round(B / (mixed["graph_ms"] / 1e3), 1),
                               "event_ms_median_p10_p90": [round(x, 4) for x in mixed["graph_pct"]]}
    if ck_other is not None:
        out["ck_other_mixing"] = {"ck_mix": ck_other["ck_mix"],
                                  "spectra_per_s": round(B / (ck_other["ms_per_step"] / 1e3), 1),
                                  "ms_per_step": round(ck_other["ms_per_step"], 4),
                                  "kernel_ms_per_step": {k: round(v[0] / max(1, v[1]), 4)
                                                         for k, v in ck_other["kernels"].items() if v[1]}}
    if fp64 is not None:
        out["fp64_plain"] = {"spectra_per_s": round(B / (fp64["ms_per_step"] / 1e3), 1),
                             "ms_per_step": round(fp64["ms_per_step"], 3),
                             "kernel_ms_per_step": {k: round(v[0] / max(1, v[1]), 4)
                                                    for k, v in fp64["kernels"].items() if v[1]}}
        if fp64["has_grad"] == mixed["has_grad"]:
            out["speedup_vs_fp64"] = round(fp64["ms_per_step"] / mixed["ms_per_step"], 3)
            if mixed["has_grad"]:
                # every sample's reduced-precision gradient against the FP64 GPU adjoint, per
                # component relative to max(|g*|, 1e-3 max|g*|) of its sample
                okg = (mixed["status"] == 0) & (fp64["status"] == 0)
                gm, g64 = mixed["grad"][okg], fp64["grad"][okg]
                scale = np.maximum(np.abs(g64), 1e-3 * np.max(np.abs(g64), axis=1, keepdims=True))
                out["max_grad_err_vs_fp64_gpu"] = float(np.max(np.abs(gm - g64) / scale))
        else:
            out["fp64_plain"]["step"] = "forward only (the FP64 path has no adjoint for this workload)"
        ok = (mixed["status"] == 0) & (fp64["status"] == 0)
        out["max_rel_err_vs_fp64_gpu"] = spec_err(mixed["spec"][ok], fp64["spec"][ok])
    if fp64_fwd is not None and fwd_only is not None:
        out["fp64_plain"]["forward_only"] = {"spectra_per_s": round(B / (fp64_fwd["ms_per_step"] / 1e3), 1),
                                             "ms_per_step": round(fp64_fwd["ms_per_step"], 3)}
        out["speedup_vs_fp64_forward_only"] = round(fp64_fwd["ms_per_step"] / fwd_only["ms_per_step"], 3)
    if not args.no_cpu_baseline and cid in (1, 7, 8):
        res, dt, cores, busy, busy_fwd = cpu_baseline(cid, B, args.cpu_samples, mixed["has_grad"], args.tp, args.bd,
                                                      int(wl["ck_mix"]) if ck else None)
        n = len(res)
        errs, lerrs, gerrs = [], [], []
        for idx, spec, lnl, g in res:
            if not np.all(np.isfinite(spec)):
                continue
            errs.append(spec_err(mixed["spec"][idx][None], spec[None]))
            lerrs.append(abs(mixed["lnl"][idx] - lnl) / abs(lnl))
            if g is not None and mixed["grad"] is not None:
                gm = mixed["grad"][idx]
                scale = np.maximum(np.abs(g), 1e-3 * np.max(np.abs(g)))
                gerrs.append(float(np.max(np.abs(gm - g) / scale)))
        out["cpu_baseline"] = {"value": round(n / dt, 4), "unit": "spectra/s", "cores": cores, "kind": "oracle",
                               "sample": f"{n} of the {B} samples (every {B // n}th), FP64 oracle forward"
                                         + (" + complex-step gradient" if mixed["has_grad"] else "")
                                         + f", {cores} worker processes, {dt:.1f} s per worker",
                               "cpu": cpu_model(), "per_core_value": round(n / busy, 4),
                               "forward_only_value": round(n / (busy_fwd / cores), 4)}
        out["max_rel_err"] = {"spectrum": max(errs) if errs else None, "lnL": float(max(lerrs)) if lerrs else None,
                              "grad": max(gerrs) if gerrs else None, "samples": len(errs)}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
