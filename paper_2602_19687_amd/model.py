"""Python face of the library: a context per workload, forward and gradient
calls on torch device tensors, and a torch.autograd.Function.

Torch only supplies device memory and the stream; every step of the forward
model and its adjoint runs in the HIP kernels of libexofwd.so.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L


def _dptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def build_config(wl, precision: int, batch_max: int, device: int = 0, n_layers_max: int | None = None):
    """The exofwd_config of a workload; returns (config, arrays it points into).

    The arrays must stay alive until exofwd_create has returned."""
    keep = []

    def arr(x, dt):
        a = np.ascontiguousarray(np.asarray(x, dtype=dt))
        keep.append(a)
        return a

    nu = arr(wl["nu"], np.float64)
    cfg = L.Config()
    cfg.mode = int(wl["mode"])
    cfg.precision = precision
    cfg.tp_kind = int(wl["tp"])
    cfg.n_knots = int(wl.get("n_knots", 0) or 0)
    cfg.n_species = int(wl["n_species"])
    cfg.n_layers_max = int(n_layers_max or wl["n_layers"])
    cfg.batch_max = batch_max
    cfg.has_cia = int(bool(wl["cia"]))
    cfg.has_rayleigh = int(bool(wl["rayleigh"]))
    cfg.has_cloud = int(bool(wl["cloud"]))
    cfg.has_scale = int(bool(wl["scale"]))
    cfg.has_offset = int(bool(wl["offset"]))
    cfg.n_mu = int(wl["n_mu"])
    cfg.cloud_model = int(wl.get("cloud_model", 0))
    cfg.cloud_profile = int(wl.get("cloud_profile", 0))
    cfg.cloud_qext = int(wl.get("cloud_qext", 0))
    cfg.has_fcld = int(bool(wl.get("fcld", False)))
    cfg.has_bd = int(bool(wl.get("bd", False)))
    cfg.bd_distance = float(wl.get("bd_distance", 0.0))
    for k in ("mu_fixed", "r_p", "r_s", "g_ref", "kappa_ir", "f_hem", "kappa_cloud", "t_star", "dilution",
              "err_c", "ray_h2", "ray_he"):
        setattr(cfg, k, float(wl[k]))
    cfg.p_bot_bar, cfg.p_top_bar, cfg.p_ref_bar = float(wl["p_bot"]), float(wl["p_top"]), float(wl["p_ref_bar"])
    cfg.n_nu = len(nu)
    cfg.nu = _dptr(nu, C.c_double)
    tg, pg = arr(wl["t_grid"], np.float64), arr(wl["logp_grid"], np.float64)
    cfg.n_t, cfg.n_p = len(tg), len(pg)
    cfg.t_grid, cfg.logp_grid = _dptr(tg, C.c_double), _dptr(pg, C.c_double)
    cfg.log10_xsec = _dptr(arr(wl["log10_xsec"], np.float64), C.c_double)
    cfg.species_mass = _dptr(arr(wl["species_mass"], np.float64), C.c_double)
    if wl["cia"]:
        tc = arr(wl["tc_grid"], np.float64)
        cfg.n_tc = len(tc)
        cfg.tc_grid = _dptr(tc, C.c_double)
        cfg.log10_cia = _dptr(arr(wl["log10_cia"], np.float64), C.c_double)
    cfg.n_bins = len(wl["bin_lo"])
    cfg.bin_lo = _dptr(arr(wl["bin_lo"], np.int32), C.c_int32)
    cfg.bin_hi = _dptr(arr(wl["bin_hi"], np.int32), C.c_int32)
    cfg.y_obs = _dptr(arr(wl["y_obs"], np.float64), C.c_double)
    cfg.y_err = _dptr(arr(wl["y_err"], np.float64), C.c_double)
    cfg.offset_mask = _dptr(arr(wl["offset_mask"], np.uint8), C.c_uint8)
    if wl.get("ck", False):
        cw = arr(wl["ck_w"], np.float64)
        cfg.ck_g = len(cw)
        cfg.ck_mix = int(wl.get("ck_mix", 0))
        cfg.ck_weights = _dptr(cw, C.c_double)
    cfg.device = device
    return cfg, keep


class ForwardModel:
    """One library context built from a workload description.

    ``wl`` is a mapping with the keys produced by ``synth.workload`` (grids,
    tables, bins, observed data and scalar settings).  ``precision`` is
    "mixed" (FP16 tables in transmission, FP32 in emission; FP32 opacity; bf16x3
    MFMA chord) or "fp64".
    """

    def __init__(self, wl, precision: str = "mixed", batch_max: int | None = None, device: int = 0,
                 n_layers_max: int | None = None):
        self.lib = L.load()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the forward model runs only on the GPU")
        self.device = torch.device("cuda", device)
        self.precision = {"mixed": L.PREC_MIXED, "fp64": L.PREC_FP64}[precision]
        self.batch_max = int(batch_max or wl["batch"])
        cfg, self._keep = build_config(wl, self.precision, self.batch_max, device, n_layers_max)
        ctx = C.c_void_p()
        with torch.cuda.device(self.device):
            L.check(self.lib.exofwd_create(C.byref(cfg), C.byref(ctx)), None, "exofwd_create")
        self.ctx = ctx
        self.n_params = self.lib.exofwd_num_params(ctx)
        self.n_nu = self.lib.exofwd_num_nu(ctx)
        self.n_bins = self.lib.exofwd_num_bins(ctx)
        self.has_grad = self.lib.exofwd_grad_supported(ctx) == 1
        self._graphs = False
        self._gstream = None
        self._gbuf = {}
        self.spec_dtype = torch.float64 if self.precision == L.PREC_FP64 else torch.float32

    # ------------------------------------------------------------------ helpers
    def _check_params(self, params: torch.Tensor) -> torch.Tensor:
        if params.device != self.device or params.dtype != torch.float64 or params.dim() != 2:
            raise ValueError(f"params must be a float64 [B, {self.n_params}] tensor on {self.device}")
        if params.shape[1] != self.n_params:
            raise ValueError(f"params has {params.shape[1]} columns, the model takes {self.n_params}")
        return params.contiguous()

    def _nl(self, n_layers, b):
        if n_layers is None:
            return None, None
        t = torch.as_tensor(n_layers, dtype=torch.int32, device=self.device).contiguous()
        if t.shape != (b,):
            raise ValueError("n_layers must have one entry per sample")
        return t, t.data_ptr()

    def _stream(self):
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    # ------------------------------------------------------------- graph mode
    def set_graphs(self, enable: bool):
        """Capture each distinct call into a hipGraph once and replay it after.

        Inputs are copied into buffers kept per (call kind, B), the library runs
        on a side stream ordered after the caller's current stream (and the
        caller's stream after it), and the results are returned as fresh tensors."""
        L.check(self.lib.exofwd_set_graphs(self.ctx, int(enable)), self.ctx, "set_graphs")
        self._graphs = bool(enable)
        self._gbuf = {}
        self._gstream = torch.cuda.Stream(self.device) if enable else None

    def _graph_call(self, kind, params, nl_t, want_spectra, call):
        b = params.shape[0]
        key = (kind, b, nl_t is not None, want_spectra)
        buf = self._gbuf.get(key)
        if buf is None:
            dev = self.device
            buf = dict(params=torch.empty_like(params),
                       nl=torch.empty(b, dtype=torch.int32, device=dev) if nl_t is not None else None,
                       spec=torch.empty((b, self.n_nu), dtype=self.spec_dtype, device=dev) if want_spectra else None,
                       lnl=torch.empty(b, dtype=torch.float64, device=dev),
                       grad=torch.empty((b, self.n_params), dtype=torch.float64, device=dev) if kind == "g" else None,
                       status=torch.empty(b, dtype=torch.int32, device=dev))
            self._gbuf[key] = buf
        buf["params"].copy_(params)
        if nl_t is not None:
            buf["nl"].copy_(nl_t)
        cur = torch.cuda.current_stream(self.device)
        self._gstream.wait_stream(cur)
        call(buf, C.c_void_p(self._gstream.cuda_stream))
        cur.wait_stream(self._gstream)
        return {k: (v.clone() if v is not None and k not in ("params", "nl") else None) for k, v in buf.items()}

    @staticmethod
    def _ptr(t):
        return C.c_void_p(t.data_ptr() if t is not None else None)

    # ------------------------------------------------------------------ calls
    def forward(self, params: torch.Tensor, n_layers=None, want_spectra: bool = True, out=None):
        """Spectra [B, n_nu] (or None), lnL [B] float64, status [B] int32."""
        params = self._check_params(params)
        b = params.shape[0]
        nl_t, nl_p = self._nl(n_layers, b)
        if self._graphs:
            def call(buf, st):
                L.check(self.lib.exofwd_forward(self.ctx, b, self._ptr(buf["params"]), self._ptr(buf["nl"]),
                                                self._ptr(buf["spec"]), self._ptr(buf["lnl"]),
                                                self._ptr(buf["status"]), st), self.ctx, "exofwd_forward")
            o = self._graph_call("f", params, nl_t, want_spectra, call)
            if out is not None and o["spec"] is not None:
                out.copy_(o["spec"])
                o["spec"] = out
            return o["spec"], o["lnl"], o["status"]
        spec = None
        if want_spectra:
            spec = out if out is not None else torch.empty((b, self.n_nu), dtype=self.spec_dtype, device=self.device)
        lnl = torch.empty(b, dtype=torch.float64, device=self.device)
        status = torch.empty(b, dtype=torch.int32, device=self.device)
        L.check(self.lib.exofwd_forward(self.ctx, b, C.c_void_p(params.data_ptr()), C.c_void_p(nl_p),
                                        C.c_void_p(spec.data_ptr() if spec is not None else None),
                                        C.c_void_p(lnl.data_ptr()), C.c_void_p(status.data_ptr()), self._stream()),
                self.ctx, "exofwd_forward")
        return spec, lnl, status

    def grad(self, params: torch.Tensor, n_layers=None, want_spectra: bool = False):
        """lnL [B], d lnL / d params [B, P], status [B], spectra or None."""
        params = self._check_params(params)
        b = params.shape[0]
        nl_t, nl_p = self._nl(n_layers, b)
        if self._graphs:
            def call(buf, st):
                L.check(self.lib.exofwd_grad(self.ctx, b, self._ptr(buf["params"]), self._ptr(buf["nl"]),
                                             self._ptr(buf["spec"]), self._ptr(buf["lnl"]), self._ptr(buf["grad"]),
                                             self._ptr(buf["status"]), st), self.ctx, "exofwd_grad")
            o = self._graph_call("g", params, nl_t, want_spectra, call)
            return o["lnl"], o["grad"], o["status"], o["spec"]
        spec = torch.empty((b, self.n_nu), dtype=self.spec_dtype, device=self.device) if want_spectra else None
        lnl = torch.empty(b, dtype=torch.float64, device=self.device)
        g = torch.empty((b, self.n_params), dtype=torch.float64, device=self.device)
        status = torch.empty(b, dtype=torch.int32, device=self.device)
        L.check(self.lib.exofwd_grad(self.ctx, b, C.c_void_p(params.data_ptr()), C.c_void_p(nl_p),
                                     C.c_void_p(spec.data_ptr() if spec is not None else None),
                                     C.c_void_p(lnl.data_ptr()), C.c_void_p(g.data_ptr()),
                                     C.c_void_p(status.data_ptr()), self._stream()),
                self.ctx, "exofwd_grad")
        return lnl, g, status, spec

    # ------------------------------------------------------------- launch choices
    def get_tuning(self):
        """[forward order, reverse shape, reverse work items, layer-sum tiles]."""
        t = (C.c_int32 * 4)()
        L.check(self.lib.exofwd_get_tuning(self.ctx, t), self.ctx, "get_tuning")
        return list(t)

    def set_tuning(self, tuning):
        t = (C.c_int32 * 4)(*[int(x) for x in tuning])
        L.check(self.lib.exofwd_set_tuning(self.ctx, t), self.ctx, "set_tuning")

    def autotune(self, batch: int, params: torch.Tensor | None = None, n_layers=None, cache_path: str | None = None):
        """Time the launch choices at this batch size and keep the fastest; returns them."""
        p = self._check_params(params) if params is not None else None
        nl_t, nl_p = self._nl(n_layers, batch)
        L.check(self.lib.exofwd_autotune(self.ctx, int(batch), self._ptr(p), C.c_void_p(nl_p),
                                         cache_path.encode() if cache_path else None), self.ctx, "autotune")
        return self.get_tuning()

    def set_profiling(self, enable: bool):
        L.check(self.lib.exofwd_set_profiling(self.ctx, int(enable)), self.ctx, "set_profiling")

    def kernel_time(self, name: str):
        ms = C.c_double()
        n = C.c_int32()
        L.check(self.lib.exofwd_kernel_time(self.ctx, name.encode(), C.byref(ms), C.byref(n)), self.ctx,
                "kernel_time")
        return ms.value, n.value

    def device_bytes(self) -> int:
        return int(self.lib.exofwd_device_bytes(self.ctx))

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.exofwd_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ExoLogLike(torch.autograd.Function):
    """lnL(params) with the hand-written adjoint as its backward.

    apply(params [B, P] float64 cuda, model, n_layers or None) -> lnL [B].
    """

    @staticmethod
    def forward(ctx, params, model: ForwardModel, n_layers=None):
        if params.requires_grad:
            lnl, g, _, _ = model.grad(params.detach(), n_layers)
            ctx.save_for_backward(g)
        else:
            _, lnl, _ = model.forward(params, n_layers, want_spectra=False)
            ctx.save_for_backward(None)
        return lnl

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return grad_out[:, None] * g, None, None
