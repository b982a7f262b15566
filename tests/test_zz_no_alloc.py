"""lip_fit_eval_noalloc (no workspace, no allocation) against lip_fit_eval.

Both run the same kernels; the variant takes its scratch memory from the
library's static device array and may use a smaller data split, which does
not change any result.  So every output must equal lip_fit_eval's bit for bit
(values compared with ==), on two calls in a row (the second smaller, so it
runs on scratch the first one filled), and sizes beyond the array's limit
are refused before any work.
"""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
KEYS = ("g", "h_up", "h_lo", "arg_up", "arg_lo")


@pytest.fixture(scope="module")
def lf():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2606_04670_amd as lf
    lf.load()
    return lf


def _noalloc(lf, p, x, y, xq, mk):
    from paper_2606_04670_amd import _lib as L
    q = xq.shape[0]
    out = {k: torch.empty(q, dtype=torch.float32 if k in ("g", "h_up", "h_lo") else torch.int32,
                          device=DEV) for k in KEYS}
    met = lf.Metric(p.d, p.norm, mon=p.mon, w=p.w)
    ptr = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())
    st = L.load().lip_fit_eval_noalloc(
        met.ref(), ptr(x), ptr(y), x.shape[0], 0.0 if mk is not None else p.M, ptr(mk), ptr(xq), q,
        ptr(out["g"]), ptr(out["h_up"]), ptr(out["h_lo"]), ptr(out["arg_up"]),
        ptr(out["arg_lo"]), 0, ctypes.c_void_p(torch.cuda.current_stream(DEV).cuda_stream))
    return st, out


def _check(lf, p, label):
    t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    x, y, xq, mk = t(p.x), t(p.y), t(p.xq), t(p.Mk)
    met = lf.Metric(p.d, p.norm, mon=p.mon, w=p.w)
    ref = lf.fit_eval(x, y, xq, met, M=None if mk is not None else p.M, Mk=mk)
    st, got = _noalloc(lf, p, x, y, xq, mk)
    torch.cuda.synchronize()
    assert st == 0, f"{label}: status {st}"
    for k in KEYS:
        a, b = got[k].cpu().numpy(), ref[k].cpu().numpy()
        bad = np.nonzero(a != b)[0]
        assert bad.size == 0, f"{label}: {k} differs at {bad.size} queries, first {bad[:5]}"


def test_two_calls_second_smaller(lf):
    # the benchmark workload (d = 4, N = 1e5, Q = 1e6, l1, two increasing
    # coordinates, per-datum M_k), then a small weighted l2 problem
    _check(lf, W.monotone_local(norm=1), "monotone_local l1")
    _check(lf, W.random_problem(5, n=3001, q=777, d=3, norm=2, mon=np.array([0, -1, 1], np.int8),
                                weighted=True), "small l2")
    _check(lf, W.random_problem(6, n=20, q=5, d=16, norm=3, local=True), "tiny linf")


def test_limits_and_refusals(lf):
    from paper_2606_04670_amd import _lib as L
    # staged data beyond 64 MiB: refused with LIP_E_SHAPE before any work
    n, d = 900_000, 16
    p = W.Problem("big", np.zeros((1, d), np.float32), np.zeros(1, np.float32), 1.0, None,
                  np.zeros((1, d), np.float32), 2, np.zeros(d, np.int8), np.ones(d, np.float32))
    x = torch.zeros((n, d), device=DEV)
    y = torch.zeros(n, device=DEV)
    xq = torch.zeros((10, d), device=DEV)
    st, _ = _noalloc(lf, p, x, y, xq, None)
    assert st == L.LIP_E_SHAPE
    # just below the limit it runs (n = 880,000 at d = 16)
    x2 = torch.rand((880_000, d), device=DEV, generator=torch.Generator(DEV).manual_seed(1))
    y2 = torch.rand(880_000, device=DEV, generator=torch.Generator(DEV).manual_seed(2))
    xq2 = torch.rand((300, d), device=DEV, generator=torch.Generator(DEV).manual_seed(3))
    st, got = _noalloc(lf, p, x2, y2, xq2, None)
    ref = lf.fit_eval(x2, y2, xq2, lf.Metric(d, "l2"), M=1.0)
    torch.cuda.synchronize()
    assert st == 0
    for k in KEYS:
        assert torch.equal(got[k], ref[k]), k
    # flags are not accepted
    st = L.load().lip_fit_eval_noalloc(lf.Metric(d, "l2").ref(), ctypes.c_void_p(x2.data_ptr()),
                                       ctypes.c_void_p(y2.data_ptr()), 10, 1.0, None,
                                       ctypes.c_void_p(xq2.data_ptr()), 1, None, None, None, None,
                                       None, L.LIP_FLAG_BF16, None)
    assert st == L.LIP_E_UNSUPPORTED
