"""PyTorch-facing binding of liblipfit.so.

Tensors supply device memory and the current HIP stream; every computation
runs in the library's kernels.  Functions mirror the C entry points:

    fit_eval / bounds   -> lip_fit_eval / lip_bounds      (Eq. 2-3)
    backward            -> lip_fit_backward
    consistency         -> lip_consistency                (Sec. 1, 4.1, Eqs. 5-6)
    estimate_M          -> lip_estimate_M                 (Sec. 5, Sec. 4.3)
    local_knots         -> lip_local_knots                (Sec. 4.3, step-function M_k(t))
    local_steps         -> lip_local_steps
    fit_eval_steps      -> lip_fit_eval_steps
    StepModel           -> the three above in sequence
    fit_eval_k          -> lip_fit_eval_k                 (Sec. 5, k > 1 weighted bounds)
    smooth_objective    -> lip_smooth_objective           (Sec. 4.4, Eq. 7)
    smooth_lipschitz    -> L-BFGS over smooth_objective   (Sec. 5, smooth_lipschitz)
    Plan                -> lip_plan_create / execute / destroy
    LipFitFn            -> torch.autograd.Function over fit_eval + backward
"""
from __future__ import annotations

import ctypes
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import _lib as L

NORMS = {"l1": L.LIP_L1, "l2": L.LIP_L2, "linf": L.LIP_LINF, 1: L.LIP_L1, 2: L.LIP_L2,
         3: L.LIP_LINF}


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Metric:
    """Distance definition: dimension, norm, weights and monotonicity (host).

    mon per coordinate: 0 free, +1 / -1 increasing / decreasing (Sec. 4.1),
    or 2..5 for cases I..IV of Sec. 4.2 on [a_i, b_i] (a, b given then)."""

    def __init__(self, d: int, norm="l2", mon: Optional[Sequence[int]] = None,
                 w: Optional[Sequence[float]] = None, a: Optional[Sequence[float]] = None,
                 b: Optional[Sequence[float]] = None):
        self.d = int(d)
        self.norm = NORMS[norm]
        self.mon = None if mon is None else np.ascontiguousarray(np.asarray(mon, np.int8))
        self.w = None if w is None else np.ascontiguousarray(np.asarray(w, np.float32))
        self.a = None if a is None else np.ascontiguousarray(np.asarray(a, np.float32))
        self.b = None if b is None else np.ascontiguousarray(np.asarray(b, np.float32))
        for nm in ("mon", "w", "a", "b"):
            v = getattr(self, nm)
            if v is not None and v.shape != (self.d,):
                raise ValueError(f"{nm} must have d entries")
        ptr = lambda v: None if v is None else v.ctypes.data_as(ctypes.c_void_p)
        self._c = L.LipMetric(self.d, self.norm, ptr(self.w), ptr(self.mon), ptr(self.a),
                              ptr(self.b))

    @property
    def n_mon(self) -> int:
        return 0 if self.mon is None else int(np.count_nonzero(self.mon))

    def ref(self):
        return ctypes.byref(self._c)


# ---- workspace cache: one growing byte buffer per (device, stream) ----------
#
# Calls are asynchronous on the current stream, so two streams must not share
# scratch: each (device, stream) pair keeps its own buffer, allocated through
# the caching allocator while that stream is current (a replaced buffer is
# returned to the allocator in that stream's order).

_WS: Dict[tuple, torch.Tensor] = {}


def workspace(device: torch.device, nbytes: int) -> torch.Tensor:
    idx = device.index if device.index is not None else torch.cuda.current_device()
    key = (idx, torch.cuda.current_stream(device).cuda_stream)
    t = _WS.get(key)
    if t is None or t.numel() < nbytes:
        t = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
        _WS[key] = t
    return t


def _f32(t: torch.Tensor, name: str, device=None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32:
        raise TypeError(f"{name} must be a float32 tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on a GPU device")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    return t.contiguous()


def _prep(x, y, M, Mk):
    x = _f32(x, "x")
    dev = x.device
    y = _f32(y, "y", dev)
    if Mk is not None:
        Mk = _f32(Mk, "Mk", dev)
        M = 0.0
    elif M is None:
        raise ValueError("give M or Mk")
    return x, y, float(M), Mk, dev


def fit_eval(x: torch.Tensor, y: torch.Tensor, xq: torch.Tensor, metric: Metric,
             M: Optional[float] = None, Mk: Optional[torch.Tensor] = None,
             want=("g", "h_up", "h_lo", "arg_up", "arg_lo"), bf16: bool = False,
             check_finite: bool = False) -> Dict[str, torch.Tensor]:
    """Eq. (2)-(3) at the queries: returns the requested outputs."""
    x, y, M, Mk, dev = _prep(x, y, M, Mk)
    xq = _f32(xq, "xq", dev)
    n, q = x.shape[0], xq.shape[0]
    out = {}
    for k in want:
        if k in ("g", "h_up", "h_lo"):
            out[k] = torch.empty(q, dtype=torch.float32, device=dev)
        elif k in ("arg_up", "arg_lo"):
            out[k] = torch.empty(q, dtype=torch.int32, device=dev)
        else:
            raise ValueError(k)
    flags = (L.LIP_FLAG_BF16 if bf16 else 0) | (L.LIP_FLAG_CHECK_FINITE if check_finite else 0)
    lib = L.load()
    nbytes = lib.lip_workspace_size(n, q, metric.d, flags)
    ws = workspace(dev, nbytes)
    st = lib.lip_fit_eval(metric.ref(), _ptr(x), _ptr(y), n, M, _ptr(Mk), _ptr(xq), q,
                          _ptr(out.get("g")), _ptr(out.get("h_up")), _ptr(out.get("h_lo")),
                          _ptr(out.get("arg_up")), _ptr(out.get("arg_lo")), _ptr(ws), ws.numel(),
                          flags, _stream(dev))
    L.check("lip_fit_eval", st)
    return out


def fit_eval_k(x, y, xq, metric: Metric, wk, M=None, Mk=None,
               want=("g", "h_up", "h_lo"), check_finite: bool = False) -> Dict[str, torch.Tensor]:
    """Weighted k-best bounds (k = len(wk)) and their midpoint."""
    x, y, M, Mk, dev = _prep(x, y, M, Mk)
    xq = _f32(xq, "xq", dev)
    n, q = x.shape[0], xq.shape[0]
    w = np.ascontiguousarray(np.asarray(wk, np.float32).reshape(-1))
    out = {k: torch.empty(q, dtype=torch.float32, device=dev) for k in want}
    lib = L.load()
    ws = workspace(dev, lib.lip_workspace_size(n, q, metric.d, 0))
    st = lib.lip_fit_eval_k(metric.ref(), _ptr(x), _ptr(y), n, M, _ptr(Mk), w.shape[0],
                            w.ctypes.data_as(ctypes.c_void_p), _ptr(xq), q, _ptr(out.get("g")),
                            _ptr(out.get("h_up")), _ptr(out.get("h_lo")), _ptr(ws), ws.numel(),
                            L.LIP_FLAG_CHECK_FINITE if check_finite else 0, _stream(dev))
    L.check("lip_fit_eval_k", st)
    return out


def bounds(x, y, xq, metric: Metric, M=None, Mk=None, **kw):
    return fit_eval(x, y, xq, metric, M=M, Mk=Mk, want=("h_up", "h_lo", "arg_up", "arg_lo"), **kw)


def backward(x, y, xq, metric: Metric, arg_up, arg_lo, dg=None, dh_up=None, dh_lo=None,
             M=None, Mk=None, want_dxq=True, want_dy=True, want_dM=True,
             deterministic: bool = False, check_finite: bool = False):
    """Subgradients through the saved indices: returns (dxq, dy, dM)."""
    x, y, M, Mk, dev = _prep(x, y, M, Mk)
    xq = _f32(xq, "xq", dev)
    n, q = x.shape[0], xq.shape[0]
    au = arg_up.to(torch.int32).contiguous()
    al = arg_lo.to(torch.int32).contiguous()
    opt = lambda t, nm: None if t is None else _f32(t, nm, dev)
    dg, dh_up, dh_lo = opt(dg, "dg"), opt(dh_up, "dh_up"), opt(dh_lo, "dh_lo")
    dxq = torch.empty((q, metric.d), dtype=torch.float32, device=dev) if want_dxq else None
    dy = torch.zeros(n, dtype=torch.float32, device=dev) if want_dy else None
    dM = (torch.zeros(n if Mk is not None else 1, dtype=torch.float32, device=dev)
          if want_dM else None)
    flags = (L.LIP_FLAG_DETERMINISTIC if deterministic else 0) | \
        (L.LIP_FLAG_CHECK_FINITE if check_finite else 0)
    lib = L.load()
    ws = workspace(dev, lib.lip_workspace_size(n, q, metric.d, flags))
    st = lib.lip_fit_backward(metric.ref(), _ptr(x), _ptr(y), n, M, _ptr(Mk), _ptr(xq), q,
                              _ptr(au), _ptr(al), _ptr(dg), _ptr(dh_up), _ptr(dh_lo), _ptr(dxq),
                              _ptr(dy), _ptr(dM), _ptr(ws), ws.numel(), flags, _stream(dev))
    L.check("lip_fit_backward", st)
    return dxq, dy, dM


def consistency(x, y, metric: Metric, M=None, Mk=None, tol: float = 0.0,
                per_row: bool = True, worst: bool = True,
                check_finite: bool = False) -> Dict[str, torch.Tensor]:
    """FP64 pairwise consistency check; counts[0] / counts[1] = violations up / lo,
    worst_slack[1] and worst_pair[2] the smallest slack and its (i, k)."""
    x, y, M, Mk, dev = _prep(x, y, M, Mk)
    n = x.shape[0]
    counts = torch.zeros(2, dtype=torch.int64, device=dev)
    out = {"counts": counts}
    if worst:
        out["worst_slack"] = torch.empty(1, dtype=torch.float64, device=dev)
        out["worst_pair"] = torch.empty(2, dtype=torch.int64, device=dev)
    if per_row:
        out["slack_up"] = torch.empty(n, dtype=torch.float64, device=dev)
        out["slack_lo"] = torch.empty(n, dtype=torch.float64, device=dev)
        out["partner_up"] = torch.empty(n, dtype=torch.int32, device=dev)
        out["partner_lo"] = torch.empty(n, dtype=torch.int32, device=dev)
    lib = L.load()
    ws = workspace(dev, lib.lip_workspace_size(n, 0, metric.d, 0))
    flags = L.LIP_FLAG_CHECK_FINITE if check_finite else 0
    st = lib.lip_consistency(metric.ref(), _ptr(x), _ptr(y), n, M, _ptr(Mk), float(tol),
                             _ptr(counts), _ptr(out.get("worst_slack")), _ptr(out.get("worst_pair")),
                             _ptr(out.get("slack_up")), _ptr(out.get("slack_lo")),
                             _ptr(out.get("partner_up")), _ptr(out.get("partner_lo")), _ptr(ws),
                             ws.numel(), flags, _stream(dev))
    L.check("lip_consistency", st)
    return out


def estimate_M(x, y, metric: Metric, mode: str = "global", knn: int = 16,
               check_finite: bool = False):
    """Global: (M64[1], M32[1], pair[2]); local kNN: (M64[n], M32[n], None).
    check_finite: scan the inputs first and raise on an infinite estimate."""
    x = _f32(x, "x")
    dev = x.device
    y = _f32(y, "y", dev)
    n = x.shape[0]
    m = L.LIP_M_GLOBAL if mode == "global" else L.LIP_M_LOCAL_KNN
    cnt = 1 if m == L.LIP_M_GLOBAL else n
    M64 = torch.empty(cnt, dtype=torch.float64, device=dev)
    M32 = torch.empty(cnt, dtype=torch.float32, device=dev)
    pair = torch.empty(2, dtype=torch.int64, device=dev) if m == L.LIP_M_GLOBAL else None
    lib = L.load()
    ws = workspace(dev, lib.lip_workspace_size(n, 0, metric.d, 0))
    flags = L.LIP_FLAG_CHECK_FINITE if check_finite else 0
    st = lib.lip_estimate_M(metric.ref(), _ptr(x), _ptr(y), n, m, int(knn), _ptr(M64), _ptr(M32),
                            _ptr(pair), _ptr(ws), ws.numel(), flags, _stream(dev))
    L.check("lip_estimate_M", st)
    return M64, M32, pair


# ---- step-function local constants (Sec. 4.3) ------------------------------------


def _host_f64(a) -> np.ndarray:
    if isinstance(a, torch.Tensor):
        a = a.detach().cpu().numpy()
    return np.ascontiguousarray(np.asarray(a, np.float64).reshape(-1))


def local_knots(x: torch.Tensor, metric: Metric, pairs, probs) -> torch.Tensor:
    """Quantile knots (float64 [K], on x's device) of the distances of the
    sampled pairs (host int array [m, 2]) at the probabilities probs."""
    x = _f32(x, "x")
    dev = x.device
    pr = np.ascontiguousarray(np.asarray(pairs, np.int64).reshape(-1, 2))
    pb = _host_f64(probs)
    K = pb.shape[0]
    out = torch.empty(K, dtype=torch.float64, device=dev)
    lib = L.load()
    ws = workspace(dev, lib.lip_workspace_size(max(pr.shape[0], x.shape[0]), 0, metric.d, 0))
    st = lib.lip_local_knots(metric.ref(), _ptr(x), x.shape[0],
                             pr.ctypes.data_as(ctypes.c_void_p), pr.shape[0],
                             pb.ctypes.data_as(ctypes.c_void_p), K, _ptr(out) if K else None,
                             _ptr(ws), ws.numel(), 0, _stream(dev))
    L.check("lip_local_knots", st)
    return out


def local_steps(x: torch.Tensor, y: torch.Tensor, metric: Metric, knots,
                check_finite: bool = False):
    """Step tables: (d1 float64 [n], V64 float64 [n, K+2], V32 float32 [n, K+2]).
    knots: host array-like or tensor (copied to the host)."""
    x = _f32(x, "x")
    dev = x.device
    y = _f32(y, "y", dev)
    n = x.shape[0]
    kn = _host_f64(knots)
    K = kn.shape[0]
    d1 = torch.empty(n, dtype=torch.float64, device=dev)
    V64 = torch.empty((n, K + 2), dtype=torch.float64, device=dev)
    V32 = torch.empty((n, K + 2), dtype=torch.float32, device=dev)
    lib = L.load()
    ws = workspace(dev, lib.lip_workspace_size(n, 0, metric.d, 0))
    st = lib.lip_local_steps(metric.ref(), _ptr(x), _ptr(y), n,
                             kn.ctypes.data_as(ctypes.c_void_p) if K else None, K, _ptr(d1),
                             _ptr(V64), _ptr(V32), _ptr(ws), ws.numel(),
                             L.LIP_FLAG_CHECK_FINITE if check_finite else 0, _stream(dev))
    L.check("lip_local_steps", st)
    return d1, V64, V32


def fit_eval_steps(x, y, xq, metric: Metric, knots, d1: torch.Tensor, V: torch.Tensor,
                   want=("g", "h_up", "h_lo", "arg_up", "arg_lo"),
                   check_finite: bool = False) -> Dict[str, torch.Tensor]:
    """Eq. (2)-(3) with the step-function constants M_k(dist)."""
    x = _f32(x, "x")
    dev = x.device
    y = _f32(y, "y", dev)
    xq = _f32(xq, "xq", dev)
    V = _f32(V, "V", dev)
    if d1.dtype != torch.float64 or d1.device != dev:
        raise ValueError("d1 must be a float64 tensor on the data's device")
    d1 = d1.contiguous()
    kn = _host_f64(knots)
    K = kn.shape[0]
    n, q = x.shape[0], xq.shape[0]
    if tuple(V.shape) != (n, K + 2) or tuple(d1.shape) != (n,):
        raise ValueError("table shapes must be d1 [n] and V [n, K+2]")
    out = {}
    for k in want:
        if k in ("g", "h_up", "h_lo"):
            out[k] = torch.empty(q, dtype=torch.float32, device=dev)
        elif k in ("arg_up", "arg_lo"):
            out[k] = torch.empty(q, dtype=torch.int32, device=dev)
        else:
            raise ValueError(k)
    steps = L.LipSteps(K, kn.ctypes.data_as(ctypes.c_void_p) if K else None, d1.data_ptr(),
                       V.data_ptr())
    flags = L.LIP_FLAG_CHECK_FINITE if check_finite else 0
    lib = L.load()
    ws = workspace(dev, lib.lip_workspace_size(n, q, metric.d, flags))
    st = lib.lip_fit_eval_steps(metric.ref(), _ptr(x), _ptr(y), n, ctypes.byref(steps), _ptr(xq),
                                q, _ptr(out.get("g")), _ptr(out.get("h_up")),
                                _ptr(out.get("h_lo")), _ptr(out.get("arg_up")),
                                _ptr(out.get("arg_lo")), _ptr(ws), ws.numel(), flags,
                                _stream(dev))
    L.check("lip_fit_eval_steps", st)
    return out


class StepModel:
    """compute_local_lipschitz / values_local of Sec. 5 with the step-function
    constants of Sec. 4.3: knots from m sampled pairs (drawn here with a seeded
    numpy generator: the random sample is an input of the method), the tables,
    then evaluation at any queries."""

    def __init__(self, x, y, metric: Metric, K: int = 4, m: int = 65536, seed: int = 0,
                 probs=None):
        self.x, self.y, self.metric = _f32(x, "x"), _f32(y, "y"), metric
        n = self.x.shape[0]
        rng = np.random.default_rng(seed)
        self.pairs = rng.integers(0, n, size=(m, 2))
        self.probs = (np.arange(1, K + 1, dtype=np.float64) / (K + 1) if probs is None
                      else _host_f64(probs))
        self.knots = local_knots(self.x, metric, self.pairs, self.probs).cpu().numpy()
        self.d1, self.V64, self.V32 = local_steps(self.x, self.y, metric, self.knots)

    def __call__(self, xq, want=("g", "h_up", "h_lo", "arg_up", "arg_lo")):
        return fit_eval_steps(self.x, self.y, xq, self.metric, self.knots, self.d1, self.V32,
                              want=want)


# ---- smoothing (Sec. 4.4) ---------------------------------------------------------


def smooth_objective(x, y, eps, metric: Metric, M=None, Mk=None, p: float = 1.0,
                     prune: float = 0.0, want_F: bool = True, want_grad: bool = True,
                     check_finite: bool = False):
    """Eq. (7) at the corrections eps: (F float64 [1] tensor or None,
    grad float32 [n] tensor or None).  prune = c > 0 leaves out the pairs of
    the Sec. 5 pre-screening (data within c times their Lipschitz allowance;
    the paper's c is 1/3)."""
    x, y, M, Mk, dev = _prep(x, y, M, Mk)
    eps = _f32(eps, "eps", dev)
    n = x.shape[0]
    F = torch.empty(1, dtype=torch.float64, device=dev) if want_F else None
    g = torch.empty(n, dtype=torch.float32, device=dev) if want_grad else None
    lib = L.load()
    ws = workspace(dev, lib.lip_workspace_size(n, 0, metric.d, 0))
    st = lib.lip_smooth_objective(metric.ref(), _ptr(x), _ptr(y), n, M, _ptr(Mk), _ptr(eps),
                                  float(p), float(prune), _ptr(F), _ptr(g), _ptr(ws),
                                  ws.numel(), L.LIP_FLAG_CHECK_FINITE if check_finite else 0,
                                  _stream(dev))
    L.check("lip_smooth_objective", st)
    return F, g


def smooth_lipschitz(x, y, metric: Metric, M=None, Mk=None, p: float = 1.0, prune: float = 0.0,
                     max_iter: int = 200, tolerance_grad: float = 1e-7, history_size: int = 20):
    """Smoothed data y + eps minimising Eq. (7) with torch's L-BFGS as the
    unconstrained minimiser (the paper's choice); every objective and
    gradient evaluation is one lip_smooth_objective call.  Returns
    (y + eps, eps, final objective)."""
    x = _f32(x, "x")
    y = _f32(y, "y", x.device)
    eps = torch.zeros_like(y, requires_grad=True)
    opt = torch.optim.LBFGS([eps], max_iter=max_iter, tolerance_grad=tolerance_grad,
                            tolerance_change=0.0, history_size=history_size,
                            line_search_fn="strong_wolfe")

    def closure():
        # the objective stays FP64 (the fixed-order sums of the kernel): the
        # optimiser compares its values in the line search
        F, g = smooth_objective(x, y, eps.detach(), metric, M=M, Mk=Mk, p=p, prune=prune)
        eps.grad = g
        return F.reshape(())

    opt.step(closure)
    F, _ = smooth_objective(x, y, eps.detach(), metric, M=M, Mk=Mk, p=p, prune=prune,
                            want_grad=False)
    e = eps.detach()
    return y + e, e, F


class LipFitFn(torch.autograd.Function):
    """g(xq) (and H_up, H_lo) with subgradients w.r.t. xq, y and M / Mk.

    forward(xq, x, y, M_or_Mk, metric, return_bounds=False)
    M_or_Mk is a 0-d / 1-element tensor (global M) or an [n] tensor (M_k).
    The attaining indices are saved for the backward pass.
    """

    @staticmethod
    def forward(ctx, xq, x, y, M_or_Mk, metric: Metric, return_bounds: bool = False):
        local = M_or_Mk.numel() == x.shape[0] and M_or_Mk.dim() == 1 and x.shape[0] > 1
        Mk = M_or_Mk.detach().float().contiguous() if local else None
        M = None if local else float(M_or_Mk.detach().reshape(-1)[0].item())
        out = fit_eval(x.detach(), y.detach(), xq.detach(), metric, M=M, Mk=Mk)
        ctx.save_for_backward(xq, x, y, M_or_Mk, out["arg_up"], out["arg_lo"])
        ctx.metric, ctx.local, ctx.return_bounds = metric, local, return_bounds
        ctx.mark_non_differentiable(out["arg_up"], out["arg_lo"])
        if return_bounds:
            return out["g"], out["h_up"], out["h_lo"]
        return out["g"]

    @staticmethod
    def backward(ctx, *grads):
        xq, x, y, M_or_Mk, au, al = ctx.saved_tensors
        dg = grads[0]
        dh_up = grads[1] if ctx.return_bounds else None
        dh_lo = grads[2] if ctx.return_bounds else None
        c = lambda t: None if t is None else t.float().contiguous()
        Mk = M_or_Mk.detach().float().contiguous() if ctx.local else None
        M = None if ctx.local else float(M_or_Mk.detach().reshape(-1)[0].item())
        dxq, dy, dM = backward(x.detach(), y.detach(), xq.detach(), ctx.metric, au, al,
                               dg=c(dg), dh_up=c(dh_up), dh_lo=c(dh_lo), M=M, Mk=Mk,
                               want_dxq=ctx.needs_input_grad[0], want_dy=ctx.needs_input_grad[2],
                               want_dM=ctx.needs_input_grad[3])
        if dM is not None:
            dM = dM.reshape(M_or_Mk.shape).to(M_or_Mk.dtype)
        return dxq, None, dy, dM, None, None


def lipfit(xq, x, y, M_or_Mk, metric: Metric, return_bounds: bool = False):
    return LipFitFn.apply(xq, x, y, M_or_Mk, metric, return_bounds)


# ---- batched plans -------------------------------------------------------------


class Plan:
    """Many independent fits executed by one graph launch (lip_plan_*).

    sets: list of dicts with keys x, y, xq, metric, and M or Mk.  Outputs are
    allocated here (g, h_up, h_lo, arg_up, arg_lo per set).
    """

    def __init__(self, sets: List[dict]):
        lib = L.load()
        self.sets = []
        descs = (L.LipBatchDesc * len(sets))()
        self._keep = []
        for i, s in enumerate(sets):
            x, y, M, Mk, dev = _prep(s["x"], s["y"], s.get("M"), s.get("Mk"))
            xq = _f32(s["xq"], "xq", dev)
            q = xq.shape[0]
            o = dict(g=torch.empty(q, dtype=torch.float32, device=dev),
                     h_up=torch.empty(q, dtype=torch.float32, device=dev),
                     h_lo=torch.empty(q, dtype=torch.float32, device=dev),
                     arg_up=torch.empty(q, dtype=torch.int32, device=dev),
                     arg_lo=torch.empty(q, dtype=torch.int32, device=dev))
            met: Metric = s["metric"]
            self._keep += [x, y, Mk, xq, met]
            descs[i] = L.LipBatchDesc(met._c, x.data_ptr(), y.data_ptr(), x.shape[0], M,
                                      None if Mk is None else Mk.data_ptr(), xq.data_ptr(), q,
                                      o["g"].data_ptr(), o["h_up"].data_ptr(),
                                      o["h_lo"].data_ptr(), o["arg_up"].data_ptr(),
                                      o["arg_lo"].data_ptr())
            self.sets.append(o)
            self.device = dev
        self._descs = descs
        self._plan = ctypes.c_void_p()
        st = lib.lip_plan_create(ctypes.byref(self._plan), descs, len(sets), 0, _stream(self.device))
        L.check("lip_plan_create", st)

    def execute(self):
        L.check("lip_plan_execute", L.load().lip_plan_execute(self._plan, _stream(self.device)))
        return self.sets

    def tiles(self, i: int) -> dict:
        """Tile parameters set i runs with (argmin tile, data chunks, waves)."""
        cfg = L.LipTileCfg()
        L.check("lip_plan_tiles", L.load().lip_plan_tiles(self._plan, i, ctypes.byref(cfg)))
        return dict(tile=cfg.tile, split=cfg.split, waves=cfg.waves, flags=cfg.flags)

    def close(self):
        if self._plan:
            L.load().lip_plan_destroy(self._plan)
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tune_get(d, n_mon, norm, n, q):
    cfg = L.LipTileCfg()
    L.check("lip_tune_get", L.load().lip_tune_get(d, n_mon, NORMS[norm], n, q, ctypes.byref(cfg)))
    return dict(tile=cfg.tile, split=cfg.split, waves=cfg.waves, flags=cfg.flags)


def tune_set(d, n_mon, norm, tile=None, split=None, waves=None, clear=False, n=0, q=0,
             flags=0):
    """Tile parameters for the size class of (n, q), or every size (n = q = 0);
    flags: LIP_TILE_* bits (1: the root-free l2 filter, 2: queries in Morton order)."""
    lib = L.load()
    if clear:
        L.check("lip_tune_set", lib.lip_tune_set(d, n_mon, NORMS[norm], n, q, None))
        return
    cfg = L.LipTileCfg(tile, split, waves, flags)
    L.check("lip_tune_set", lib.lip_tune_set(d, n_mon, NORMS[norm], n, q, ctypes.byref(cfg)))


def tune_save(path: str, arch: Optional[str] = None):
    L.check("lip_tune_save", L.load().lip_tune_save(path.encode(), None if arch is None
                                                    else arch.encode()))


def tune_load(path: str, arch: Optional[str] = None):
    L.check("lip_tune_load", L.load().lip_tune_load(path.encode(), None if arch is None
                                                    else arch.encode()))


def tune_clear():
    L.check("lip_tune_clear", L.load().lip_tune_clear())


def autotune(d, n_mon, norm, n, q, device=None):
    device = device or torch.device("cuda", torch.cuda.current_device())
    cfg = L.LipTileCfg()
    L.check("lip_autotune", L.load().lip_autotune(d, n_mon, NORMS[norm], n, q, _stream(device),
                                                   ctypes.byref(cfg)))
    return dict(tile=cfg.tile, split=cfg.split, waves=cfg.waves, flags=cfg.flags)
