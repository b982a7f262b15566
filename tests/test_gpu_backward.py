"""GPU subgradients (lip_fit_backward, LipFitFn) against the FP64 oracle.

The oracle's gradient is evaluated at the oracle's own attaining indices and
compared on the queries where the GPU selected the same indices (queries
with FP32 near-ties elsewhere are excluded; their count is bounded).  The
oracle gradient itself is pinned to finite differences on the CPU (see
test_oracle_pins.py); here finite differences of the oracle forward are also
taken on tie-free queries of the differentiable workload.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def lf():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2606_04670_amd as lf
    lf.load()
    return lf


def _t(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _gpu_fwd_bwd(lf, p, deterministic=False, with_bounds=False, gen=None):
    met = lf.Metric(p.d, p.norm, mon=p.mon, w=p.w)
    x, y, xq, mk = _t(p.x), _t(p.y), _t(p.xq), _t(p.Mk)
    out = lf.fit_eval(x, y, xq, met, M=None if mk is not None else p.M, Mk=mk)
    dg = _t(p.dg)
    dh_up = dh_lo = None
    if with_bounds:
        g = np.random.default_rng(gen)
        dh_up = _t(g.standard_normal(p.q).astype(np.float32))
        dh_lo = _t(g.standard_normal(p.q).astype(np.float32))
    dxq, dy, dM = lf.backward(x, y, xq, met, out["arg_up"], out["arg_lo"], dg=dg, dh_up=dh_up,
                              dh_lo=dh_lo, M=None if mk is not None else p.M, Mk=mk,
                              deterministic=deterministic)
    torch.cuda.synchronize()
    cpu = lambda t: None if t is None else t.cpu().numpy()
    return ({k: cpu(v) for k, v in out.items()}, cpu(dxq), cpu(dy), cpu(dM), cpu(dh_up),
            cpu(dh_lo))


def _compare(p, out, dxq, dy, dM, dh_up=None, dh_lo=None, label=""):
    hu, hl, g, au, al = oracle.bounds(p.x, p.y, p.xq, p.norm, M=p.M, Mk=p.Mk, mon=p.mon, w=p.w)
    same = (out["arg_up"] == au) & (out["arg_lo"] == al)
    assert same.mean() > 0.995, f"{label}: too many index mismatches {(~same).sum()}"
    odx, ody, odM = oracle.grad(p.x, p.y, p.xq[same], p.norm, au[same], al[same],
                                dg=p.dg[same], dh_up=None if dh_up is None else dh_up[same],
                                dh_lo=None if dh_lo is None else dh_lo[same], M=p.M, Mk=p.Mk,
                                mon=p.mon, w=p.w)
    scale = max(1.0, float(np.abs(odx).max()))
    err = np.abs(dxq[same] - odx)
    assert err.max() <= 2e-5 * scale * max(1.0, float(np.max(p.Mk) if p.Mk is not None else p.M)), \
        f"{label}: dxq err {err.max()}"
    if same.all():
        np.testing.assert_allclose(dy, ody, rtol=1e-5, atol=1e-5 * max(1.0, np.abs(ody).max()))
        np.testing.assert_allclose(dM, odM, rtol=1e-4, atol=1e-4 * max(1.0, np.abs(odM).max()))
    return int((~same).sum())


@pytest.mark.parametrize("norm", [1, 2, 3])
@pytest.mark.parametrize("mon,local", [([0, 0, 0], False), ([1, 0, -1], True), ([1, 1, 0], False)])
def test_backward_matches_oracle(lf, norm, mon, local):
    p = W.random_problem(200 + norm, n=1500, q=2000, d=3, norm=norm, mon=np.array(mon, np.int8),
                         local=local, weighted=True)
    out, dxq, dy, dM, _, _ = _gpu_fwd_bwd(lf, p)
    _compare(p, out, dxq, dy, dM, label=f"norm={norm} mon={mon}")


def test_backward_with_bound_gradients(lf):
    p = W.random_problem(300, n=2000, q=1500, d=4, norm=2, mon=np.array([1, 0, 0, 0], np.int8),
                         local=True)
    out, dxq, dy, dM, dhu, dhl = _gpu_fwd_bwd(lf, p, with_bounds=True, gen=1)
    _compare(p, out, dxq, dy, dM, dh_up=dhu, dh_lo=dhl, label="bounds grads")


def test_deterministic_accumulation(lf):
    """LIP_FLAG_DETERMINISTIC: bitwise identical dy / dM over repeated calls and
    within FP32 accuracy of the atomic path."""
    p = W.random_problem(301, n=500, q=20000, d=3, norm=1, mon=np.array([1, 0, 0], np.int8),
                         local=True)
    r1 = _gpu_fwd_bwd(lf, p, deterministic=True)
    r2 = _gpu_fwd_bwd(lf, p, deterministic=True)
    np.testing.assert_array_equal(r1[2], r2[2])
    np.testing.assert_array_equal(r1[3], r2[3])
    ra = _gpu_fwd_bwd(lf, p, deterministic=False)
    np.testing.assert_allclose(r1[2], ra[2], rtol=1e-4, atol=1e-3)
    np.testing.assert_allclose(r1[3], ra[3], rtol=1e-4, atol=1e-3)
    _compare(p, r1[0], r1[1], r1[2], r1[3], label="deterministic")


def test_autograd_function(lf):
    """LipFitFn: torch.autograd gradients equal the explicit backward call."""
    p = W.random_problem(302, n=800, q=600, d=2, norm=2, local=False)
    met = lf.Metric(p.d, "l2")
    xq = _t(p.xq).requires_grad_(True)
    y = _t(p.y).requires_grad_(True)
    M = torch.tensor([p.M], device=DEV, requires_grad=True)
    g, hu, hl = lf.lipfit(xq, _t(p.x), y, M, met, return_bounds=True)
    w1, w2, w3 = (torch.randn(p.q, device=DEV) for _ in range(3))
    (g * w1 + hu * w2 + hl * w3).sum().backward()
    out = lf.fit_eval(_t(p.x), _t(p.y), _t(p.xq), met, M=p.M)
    dxq, dy, dM = lf.backward(_t(p.x), _t(p.y), _t(p.xq), met, out["arg_up"], out["arg_lo"],
                              dg=w1, dh_up=w2, dh_lo=w3, M=p.M)
    torch.testing.assert_close(xq.grad, dxq)
    torch.testing.assert_close(y.grad, dy)
    torch.testing.assert_close(M.grad, dM)


def test_diff_l2_workload_gradients_and_fd(lf):
    """d=8, N=200,000, Q=262,144, l2, M=2, upstream grads ~ N(0,1): GPU
    gradient vs oracle on 1,024 tie-free queries, whose oracle gradient is
    also checked against FP64 central differences of the oracle forward."""
    p = W.diff_l2()
    met = lf.Metric(p.d, "l2")
    x, y, xq = _t(p.x), _t(p.y), _t(p.xq)
    out = lf.fit_eval(x, y, xq, met, M=p.M)
    dxq, dy, dM = lf.backward(x, y, xq, met, out["arg_up"], out["arg_lo"], dg=_t(p.dg), M=p.M)
    au_g, al_g = out["arg_up"].cpu().numpy(), out["arg_lo"].cpu().numpy()
    dxq = dxq.cpu().numpy()
    sel = np.arange(1024)
    sub = W.Problem("fd", p.x, p.y, p.M, None, p.xq[sel], 2, p.mon, p.w, p.dg[sel])
    hu, hl, g, au, al = oracle.bounds(sub.x, sub.y, sub.xq, 2, M=p.M)
    ok = (au == au_g[sel]) & (al == al_g[sel])
    odx, _, _ = oracle.grad(sub.x, sub.y, sub.xq[ok], 2, au[ok], al[ok], dg=sub.dg[ok], M=p.M)
    np.testing.assert_allclose(dxq[sel][ok], odx, rtol=1e-4, atol=1e-4)
    # finite differences of the oracle forward on the first 64 agreeing queries
    h = 2.0 ** -12
    idx = np.nonzero(ok)[0][:64]
    checked = 0
    for j in idx:
        num = np.zeros(p.d)
        for i in range(p.d):
            xp = sub.xq[j:j + 1].copy()
            xm = sub.xq[j:j + 1].copy()
            xp[0, i] += np.float32(h)
            xm[0, i] -= np.float32(h)
            rp = oracle.bounds(sub.x, sub.y, xp, 2, M=p.M)
            rm = oracle.bounds(sub.x, sub.y, xm, 2, M=p.M)
            if not (rp[3][0] == rm[3][0] == au[j] and rp[4][0] == rm[4][0] == al[j]):
                num = None  # a selection change within h: not a smooth piece
                break
            num[i] = (rp[2][0] - rm[2][0]) / (float(xp[0, i]) - float(xm[0, i]))
        if num is None:
            continue
        checked += 1
        np.testing.assert_allclose(num * sub.dg[j], dxq[sel][j], rtol=2e-3, atol=2e-3)
    assert checked >= 48
