"""GPU subgradients (lip_fit_backward, LipFitFn) against the FP64 oracle.

The oracle's gradient is evaluated at the GPU's own attaining indices (the
forward's choice; ties and near-ties are the forward tests' business), so
dxq, dy and dM are compared element by element on every query, with no
gate.  Tolerances follow the FP32 arithmetic of the backward kernel:

  dxq[j, i]  one product chain per bound, the l2 gradient c dc / s formed in
             FP32: (d + 8) 2^-24 (|G_up| M_a + |G_lo| M_b) max w
  dy[k]      exact terms G = dg/2 (+ dh) summed in FP32 (wave sums, then
             atomics): (c_k + 2) 2^-24 A_k, with c_k the number of terms and
             A_k the sum of their magnitudes (the oracle's dy for |G|)
  dM         terms G dist with the FP32 distance ((d + 4) 2^-24 relative)
             summed the same way: (d + 5 + c) 2^-24 A, c = number of terms
             (global M: log2(64) wave levels + one atomic per wave)
  LIP_FLAG_DETERMINISTIC: int64 fixed-point sums, each term rounded to
             2^-s, s = 61 - e - b (2^e > the largest term, 2^b > q): the sum
             errs by at most q 2^-s more than the terms' own error.

The oracle gradient itself is pinned to finite differences on the CPU
(test_oracle_pins.py).  Here the GPU's dxq, dy and dM are also checked
against FP64 finite differences of the oracle forward: central differences
in each query coordinate, and directional differences in y and M along
seeded random directions (g is affine in y and M on a selection piece, so
those differences are exact up to FP64 rounding), on the differentiable
workload's first 1,024 queries whose selection stays fixed under the step.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
U = 2.0 ** -24


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


def _fixed_slack(q, largest):
    """Extra error of the deterministic fixed-point sums (see module doc)."""
    e = math.frexp(largest if largest > 0 else 1.0)[1]
    b = math.frexp(float(max(q, 1)))[1]
    return q * 2.0 ** -(61 - e - b)


def compare_grads(p, au, al, dxq, dy, dM, dh_up=None, dh_lo=None, deterministic=False,
                  label=""):
    """Element-by-element comparison at the GPU's indices (au, al) on every
    query; returns the largest errors relative to their tolerances."""
    kw = dict(M=p.M, Mk=p.Mk, mon=p.mon, w=p.w)
    dg = p.dg.astype(np.float64)
    odx, ody, odM = oracle.grad(p.x, p.y, p.xq, p.norm, au, al, dg=dg, dh_up=dh_up, dh_lo=dh_lo,
                                **kw)
    Gu = 0.5 * dg + (0.0 if dh_up is None else dh_up)
    Gl = 0.5 * dg + (0.0 if dh_lo is None else dh_lo)
    # |G| sums: the oracle's dy / dM for the magnitudes of the terms
    _, Ay, _ = oracle.grad(p.x, p.y, p.xq, p.norm, au, al, dh_up=np.abs(Gu), dh_lo=np.abs(Gl),
                           **kw)
    _, _, AM = oracle.grad(p.x, p.y, p.xq, p.norm, au, al, dh_up=np.abs(Gu), dh_lo=-np.abs(Gl),
                           **kw)
    AM = np.abs(AM)
    Mk = p.Mk.astype(np.float64) if p.Mk is not None else None
    Ma = Mk[au] if Mk is not None else p.M
    Mb = Mk[al] if Mk is not None else p.M
    wmax = float(np.max(p.w))
    rep = {"label": label}
    # dxq
    tol = (p.d + 8) * U * (np.abs(Gu) * Ma + np.abs(Gl) * Mb) * wmax + 1e-30
    err = np.abs(dxq.astype(np.float64) - odx)
    r = err / tol[:, None]
    assert r.max() <= 1.0, (f"{label}: dxq off at query {np.unravel_index(r.argmax(), r.shape)}: "
                            f"gpu {dxq.reshape(-1)[r.argmax()]!r} oracle {odx.reshape(-1)[r.argmax()]!r}")
    rep["dxq_err/tol"] = float(r.max())
    # dy
    cnt = np.bincount(au, minlength=p.n) + np.bincount(al, minlength=p.n)
    # the fixed-point scale comes from the largest term |G| or |G dist|; the
    # weighted box diagonal (l1 form, the largest of the three) bounds dist
    box = np.maximum(p.x.max(0), p.xq.max(0)).astype(np.float64) - \
        np.minimum(p.x.min(0), p.xq.min(0)).astype(np.float64)
    dbox = float((box * p.w).sum()) * 1.01
    largest = max(float(np.abs(Gu).max()), float(np.abs(Gl).max())) * max(1.0, dbox) * 1.01
    if dy is not None:
        tol = (cnt + 2) * U * Ay + 1e-30
        if deterministic:
            tol = 2 * U * np.abs(ody) + U * Ay + _fixed_slack(p.q, largest)
        err = np.abs(dy.astype(np.float64) - ody)
        r = err / tol
        k = int(r.argmax())
        assert r.max() <= 1.0, f"{label}: dy[{k}] gpu {dy[k]!r} oracle {ody[k]!r} tol {tol[k]:g}"
        rep["dy_err/tol"] = float(r.max())
    # dM
    if dM is not None:
        c = cnt if Mk is not None else np.array([6 + math.ceil(p.q / 64)])
        tol = (p.d + 5 + c) * U * AM + 1e-30
        if deterministic:
            tol = 2 * U * np.abs(odM) + (p.d + 5) * U * AM + _fixed_slack(p.q, largest)
        err = np.abs(dM.astype(np.float64).reshape(odM.shape) - odM)
        r = err / tol
        k = int(r.argmax())
        assert r.max() <= 1.0, (f"{label}: dM[{k}] gpu {dM.reshape(-1)[k]!r} oracle {odM[k]!r} "
                                f"tol {tol[k]:g}")
        rep["dM_err/tol"] = float(r.max())
    return rep


@pytest.mark.parametrize("norm", [1, 2, 3])
@pytest.mark.parametrize("mon,local", [([0, 0, 0], False), ([1, 0, -1], True), ([1, 1, 0], False)])
def test_backward_matches_oracle(lf, norm, mon, local):
    p = W.random_problem(200 + norm, n=1500, q=2000, d=3, norm=norm, mon=np.array(mon, np.int8),
                         local=local, weighted=True)
    out, dxq, dy, dM, _, _ = _gpu_fwd_bwd(lf, p)
    print(compare_grads(p, out["arg_up"], out["arg_lo"], dxq, dy, dM,
                        label=f"norm={norm} mon={mon}"))


@pytest.mark.parametrize("norm", [1, 2, 3])
@pytest.mark.parametrize("d", [1, 5, 8, 16])
def test_backward_dimensions(lf, norm, d):
    mon = np.zeros(d, np.int8)
    mon[::3] = 1
    for local in (False, True):
        p = W.random_problem(260 + d * 3 + norm, n=900, q=1500, d=d, norm=norm, mon=mon,
                             local=local, weighted=True)
        out, dxq, dy, dM, _, _ = _gpu_fwd_bwd(lf, p)
        compare_grads(p, out["arg_up"], out["arg_lo"], dxq, dy, dM,
                      label=f"d={d} norm={norm} local={local}")


def test_backward_with_bound_gradients(lf):
    p = W.random_problem(300, n=2000, q=1500, d=4, norm=2, mon=np.array([1, 0, 0, 0], np.int8),
                         local=True)
    out, dxq, dy, dM, dhu, dhl = _gpu_fwd_bwd(lf, p, with_bounds=True, gen=1)
    compare_grads(p, out["arg_up"], out["arg_lo"], dxq, dy, dM, dh_up=dhu, dh_lo=dhl,
                  label="bounds grads")


@pytest.mark.parametrize("local", [False, True])
def test_deterministic_accumulation(lf, local):
    """LIP_FLAG_DETERMINISTIC: bitwise identical dy / dM over repeated calls,
    each within its fixed-point error of the oracle."""
    p = W.random_problem(301, n=500, q=20000, d=3, norm=1, mon=np.array([1, 0, 0], np.int8),
                         local=local)
    r1 = _gpu_fwd_bwd(lf, p, deterministic=True)
    r2 = _gpu_fwd_bwd(lf, p, deterministic=True)
    np.testing.assert_array_equal(r1[2], r2[2])
    np.testing.assert_array_equal(r1[3], r2[3])
    print(compare_grads(p, r1[0]["arg_up"], r1[0]["arg_lo"], r1[1], r1[2], r1[3],
                        deterministic=True, label="deterministic"))
    ra = _gpu_fwd_bwd(lf, p, deterministic=False)
    compare_grads(p, ra[0]["arg_up"], ra[0]["arg_lo"], ra[1], ra[2], ra[3], label="atomics")


def test_autograd_function(lf):
    """LipFitFn: torch.autograd gradients equal the explicit backward call
    and the oracle's at the forward's indices."""
    p = W.random_problem(302, n=800, q=600, d=2, norm=2, local=False)
    met = lf.Metric(p.d, "l2")
    xq = _t(p.xq).requires_grad_(True)
    y = _t(p.y).requires_grad_(True)
    M = torch.tensor([p.M], device=DEV, requires_grad=True)
    g, hu, hl = lf.lipfit(xq, _t(p.x), y, M, met, return_bounds=True)
    w1, w2, w3 = (torch.randn(p.q, device=DEV, generator=torch.Generator(DEV).manual_seed(s))
                  for s in (1, 2, 3))
    (g * w1 + hu * w2 + hl * w3).sum().backward()
    out = lf.fit_eval(_t(p.x), _t(p.y), _t(p.xq), met, M=p.M)
    dxq, dy, dM = lf.backward(_t(p.x), _t(p.y), _t(p.xq), met, out["arg_up"], out["arg_lo"],
                              dg=w1, dh_up=w2, dh_lo=w3, M=p.M)
    torch.testing.assert_close(xq.grad, dxq)
    torch.testing.assert_close(y.grad, dy)
    torch.testing.assert_close(M.grad, dM)
    pw = W.Problem("autograd", p.x, p.y, p.M, None, p.xq, 2, p.mon, p.w, w1.cpu().numpy())
    compare_grads(pw, out["arg_up"].cpu().numpy(), out["arg_lo"].cpu().numpy(),
                  xq.grad.cpu().numpy(), y.grad.cpu().numpy(), M.grad.cpu().numpy(),
                  dh_up=w2.cpu().numpy().astype(np.float64),
                  dh_lo=w3.cpu().numpy().astype(np.float64), label="autograd")


def _objective(p, xq, y=None, M=None, Mk=None, dg=None):
    """G = sum_j dg_j g_j by the oracle forward, with its indices."""
    y = p.y if y is None else y
    hu, hl, g, au, al = oracle.bounds(p.x, y, xq, p.norm, M=p.M if M is None else M,
                                      Mk=Mk, mon=p.mon, w=p.w)
    return g, au, al


def test_diff_l2_workload_full(lf):
    """d=8, N=200,000, Q=262,144, l2, M=2, upstream grads ~ N(0,1): dxq, dy
    [N] and dM compared with the oracle at the GPU's indices over all
    queries, with FP32 atomics and in deterministic mode."""
    p = W.diff_l2()
    for det in (False, True):
        out, dxq, dy, dM, _, _ = _gpu_fwd_bwd(lf, p, deterministic=det)
        print(compare_grads(p, out["arg_up"], out["arg_lo"], dxq, dy, dM, deterministic=det,
                            label=f"diff_l2 deterministic={det}"))


def test_diff_l2_finite_differences(lf):
    """Finite differences of the oracle forward against the GPU gradients on
    the first 1,024 queries of the differentiable workload: central
    differences in every query coordinate, directional differences in y and
    M.  A query enters a check only if the oracle's selection at both
    perturbed points equals the GPU's (the same affine / smooth piece)."""
    full = W.diff_l2()
    sel = np.arange(1024)
    p = W.Problem("fd", full.x, full.y, full.M, None, full.xq[sel], 2, full.mon, full.w,
                  full.dg[sel])
    out, dxq, dy, dM, _, _ = _gpu_fwd_bwd(lf, p, deterministic=True)
    au, al = out["arg_up"], out["arg_lo"]
    dg = p.dg.astype(np.float64)
    # query coordinates: h = 2^-12, g smooth (l2) away from data points
    h = 2.0 ** -12
    checked = 0
    for j in range(p.q):
        num = np.zeros(p.d)
        ok = True
        for i in range(p.d):
            xp = p.xq[j:j + 1].copy()
            xm = p.xq[j:j + 1].copy()
            xp[0, i] += np.float32(h)
            xm[0, i] -= np.float32(h)
            gp, ap, lp = _objective(p, xp)
            gm, am, lm = _objective(p, xm)
            if not (ap[0] == am[0] == au[j] and lp[0] == lm[0] == al[j]):
                ok = False
                break
            num[i] = (gp[0] - gm[0]) / (float(xp[0, i]) - float(xm[0, i]))
        if not ok:
            continue
        checked += 1
        # central difference of a smooth piece: O(h^2) curvature error
        np.testing.assert_allclose(num * dg[j], dxq[j], rtol=2e-4, atol=2e-4 * abs(dg[j]) * p.M)
        if checked == 128:
            break
    assert checked == 128
    # directional differences in y: g is affine in y on a selection piece
    g0 = W.rng_for(3, 7)
    v = g0.standard_normal(p.n)
    e = 2.0 ** -12
    yp = (p.y.astype(np.float64) + e * v).astype(np.float32)
    ym = (p.y.astype(np.float64) - e * v).astype(np.float32)
    gp, ap, lp = _objective(p, p.xq, y=yp)
    gm, am, lm = _objective(p, p.xq, y=ym)
    same = (ap == au) & (am == au) & (lp == al) & (lm == al)
    assert same.mean() > 0.95, f"selection changed on {(~same).sum()} queries"
    # the GPU's dy restricted to the fixed-selection queries
    sub = W.Problem("fd-y", p.x, p.y, p.M, None, p.xq[same], 2, p.mon, p.w, p.dg[same])
    _, _, dy_s, _, _, _ = _gpu_fwd_bwd(lf, sub, deterministic=True)
    dyv = (yp.astype(np.float64) - ym.astype(np.float64))
    num = float(dg[same] @ (gp[same] - gm[same]))
    ana = float(dy_s.astype(np.float64) @ dyv)
    scale = float(np.abs(dg[same]) @ np.abs(0.5 * (dyv[au[same]] + dyv[al[same]])))
    assert abs(num - ana) <= 1e-5 * scale + 1e-12, f"dy: FD {num!r} vs GPU {ana!r}"
    # directional difference in the global M
    eM = 2.0 ** -14
    gp, ap, lp = _objective(p, p.xq, M=p.M + eM)
    gm, am, lm = _objective(p, p.xq, M=p.M - eM)
    same = (ap == au) & (am == au) & (lp == al) & (lm == al)
    assert same.mean() > 0.95
    sub = W.Problem("fd-M", p.x, p.y, p.M, None, p.xq[same], 2, p.mon, p.w, p.dg[same])
    _, _, _, dM_s, _, _ = _gpu_fwd_bwd(lf, sub, deterministic=True)
    num = float(dg[same] @ (gp[same] - gm[same])) / (2 * eM)
    hu, hl, _, _, _ = oracle.bounds(p.x, p.y, p.xq[same], 2, M=p.M)
    scale = float(np.abs(dg[same]) @ (np.abs(hu - p.y[au[same]]) + np.abs(hl - p.y[al[same]]))) / p.M
    assert abs(num - float(dM_s[0])) <= 1e-5 * scale, f"dM: FD {num!r} vs GPU {dM_s[0]!r}"


@pytest.mark.parametrize("norm", [1, 3])
def test_local_M_directional_differences(lf, norm):
    """Per-datum M_k, l1 / linf with monotone coordinates: directional
    differences in y and M_k of the oracle forward against the GPU's dy and
    dM (g is affine in both on a selection piece)."""
    p = W.random_problem(330 + norm, n=3000, q=4000, d=4, norm=norm,
                         mon=np.array([1, 0, -1, 0], np.int8), local=True, weighted=True)
    out, _, dy, dM, _, _ = _gpu_fwd_bwd(lf, p, deterministic=True)
    au, al = out["arg_up"], out["arg_lo"]
    dg = p.dg.astype(np.float64)
    rng = W.rng_for(331, norm)
    for which in ("y", "Mk"):
        v = rng.standard_normal(p.n)
        base = (p.y if which == "y" else p.Mk).astype(np.float64)
        e = 2.0 ** -13 if which == "y" else 2.0 ** -13 * base
        vp = (base + e * v).astype(np.float32)
        vm = (base - e * v).astype(np.float32)
        kwp = dict(y=vp, Mk=p.Mk) if which == "y" else dict(Mk=vp)
        kwm = dict(y=vm, Mk=p.Mk) if which == "y" else dict(Mk=vm)
        gp, ap, lp = _objective(p, p.xq, **kwp)
        gm, am, lm = _objective(p, p.xq, **kwm)
        same = (ap == au) & (am == au) & (lp == al) & (lm == al)
        assert same.mean() > 0.95, f"{which}: selection changed on {(~same).sum()} queries"
        sub = W.Problem("fd", p.x, p.y, p.M, p.Mk, p.xq[same], norm, p.mon, p.w, p.dg[same])
        _, _, dy_s, dM_s, _, _ = _gpu_fwd_bwd(lf, sub, deterministic=True)
        delta = vp.astype(np.float64) - vm.astype(np.float64)
        num = float(dg[same] @ (gp[same] - gm[same]))
        grad = dy_s if which == "y" else dM_s
        ana = float(grad.astype(np.float64) @ delta)
        # magnitude of the directional derivative's terms: the oracle's
        # gradient for |G| (both roles counted positive)
        hg = np.abs(0.5 * dg[same])
        _, ay, am = oracle.grad(sub.x, sub.y, sub.xq, norm, au[same], al[same], dh_up=hg,
                                dh_lo=hg if which == "y" else -hg, Mk=p.Mk, mon=p.mon, w=p.w)
        scale = float((ay if which == "y" else am) @ np.abs(delta)) + 1e-30
        assert abs(num - ana) <= 1e-5 * scale, f"{which}: FD {num!r} vs GPU {ana!r}"
