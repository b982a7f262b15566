"""GPU parity of the smoothing objective (Sec. 4.4, Eq. 7) and its gradient.

The pair terms are FP32 on the GPU and FP64 in the oracle.  With
S = max|z| + max M_k * D_max (z = y + eps, D_max the weighted bounding-box
diagonal) one FP32 term (a few differences, one fused multiply-add, the
distance within (d + 6) 2^-24 relative) errs by at most delta = (d + 12) 2^-24 S,
so the tolerances are
    |F_gpu - F_orc|         <= 2 delta A + c delta^2 + 2^-17 F       (A = sum of
                               positive parts, c = number of terms above -delta;
                               2^-17 covers the FP32 sums over 64-column tiles)
    |grad_gpu_i - grad_orc_i| <= 2 delta c_i + 2^-17 (|grad_i| + row_abs_i)
with c_i the terms moving eps_i that are above -delta and row_abs_i the sum
of their gradient magnitudes (oracle.smooth_scale).

With the pre-screening of Sec. 5 the dropped pairs are a yes / no answer and
must be the oracle's exactly: a wrong one moves F by a whole pair term.  The
cases use corrections large enough that many dropped pairs would be active,
and data on a grid where many pairs sit exactly on the threshold.
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
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _check(p, eps, F_gpu, g_gpu, M, Mk, pen, label, prune=0.0):
    F, g = oracle.smooth(p.x, p.y, eps, p.norm, M=M, Mk=Mk, p=pen, mon=p.mon, w=p.w, prune=prune)
    z = np.abs(p.y.astype(np.float64) + eps).max()
    span = (p.x.max(0) - p.x.min(0)).astype(np.float64) * p.w
    dmax = {1: span.sum(), 2: np.sqrt((span ** 2).sum()), 3: span.max()}[p.norm]
    mmax = float(np.max(Mk)) if Mk is not None else float(M)
    S = z + mmax * dmax
    delta = (p.d + 12) * 2.0 ** -24 * S
    A, row_abs, row_cnt = oracle.smooth_scale(p.x, p.y, eps, p.norm, delta, M=M, Mk=Mk,
                                              mon=p.mon, w=p.w, prune=prune)
    tolF = 2 * delta * A + row_cnt.sum() / 2 * delta ** 2 + 2.0 ** -17 * F
    assert abs(F_gpu - F) <= tolF, f"{label}: F gpu={F_gpu!r} oracle={F!r} tol={tolF:g}"
    tolg = 2 * delta * row_cnt + 2.0 ** -17 * (np.abs(g) + row_abs)
    bad = np.nonzero(np.abs(g_gpu - g) > tolg)[0]
    assert bad.size == 0, (f"{label}: grad off at {bad.size} rows, e.g. {bad[0]}: "
                           f"gpu={g_gpu[bad[0]]!r} oracle={g[bad[0]]!r} tol={tolg[bad[0]]:g}")
    return F


CASES = [
    # (seed, n, d, mon, local, weighted)
    (1, 1, 3, [0, 0, 0], False, False),
    (2, 2, 1, [0], False, False),
    (3, 130, 2, [1, 0], False, False),
    (4, 777, 4, [1, 0, 1, 0], False, False),
    (5, 1537, 4, [1, 0, 1, 0], True, False),
    (6, 1000, 7, [0, -1, 0, 1, 0, 0, 1], False, True),
    (7, 640, 16, [0, 1] * 8, True, True),
    (8, 2100, 3, [0, 0, 0], True, False),
]


@pytest.mark.parametrize("norm", [1, 2, 3])
@pytest.mark.parametrize("seed,n,d,mon,local,weighted", CASES)
def test_smooth_objective_parity(lf, norm, seed, n, d, mon, local, weighted):
    p = W.random_problem(600 + seed, n=n, q=1, d=d, norm=norm, mon=np.array(mon, np.int8),
                         local=local, weighted=weighted, M=0.8)
    rng = W.rng_for(601, seed)
    eps = (0.05 * rng.standard_normal(n)).astype(np.float32).astype(np.float64)
    pen = 0.7
    met = lf.Metric(d, norm, mon=p.mon, w=p.w)
    mk = None if p.Mk is None else _t(p.Mk)
    F, g = lf.smooth_objective(_t(p.x), _t(p.y), _t(eps.astype(np.float32)), met,
                               M=None if mk is not None else p.M, Mk=mk, p=pen)
    torch.cuda.synchronize()
    Fo = _check(p, eps, F.item(), g.cpu().numpy().astype(np.float64), p.M, p.Mk, pen,
                f"smooth n={n} d={d} norm={norm}")
    if n > 2:
        assert Fo > 0  # the cases do violate constraints


def test_smooth_objective_repeatable(lf):
    p = W.random_problem(650, n=3000, q=1, d=4, norm=2, mon=np.array([1, 0, 1, 0], np.int8),
                         M=0.5)
    met = lf.Metric(4, 2, mon=p.mon)
    eps = torch.zeros(3000, device=DEV)
    F1, g1 = lf.smooth_objective(_t(p.x), _t(p.y), eps, met, M=p.M, p=1.0)
    F2, g2 = lf.smooth_objective(_t(p.x), _t(p.y), eps, met, M=p.M, p=1.0)
    assert F1.item() == F2.item() and torch.equal(g1, g2)


@pytest.mark.parametrize("norm", [1, 2, 3])
def test_smoothing_removes_violations(lf, norm):
    """L-BFGS on Eq. (7): the objective falls, the gradient at the result is
    near zero, and the smoothed data violate far fewer constraints."""
    p = W.random_problem(660 + norm, n=600, q=1, d=2, norm=norm, M=0.6)
    x, y = _t(p.x), _t(p.y)
    met = lf.Metric(2, norm)
    z, eps, F = lf.smooth_lipschitz(x, y, met, M=p.M, p=10.0, max_iter=300)
    torch.cuda.synchronize()
    F0, _ = oracle.smooth(p.x, p.y, np.zeros(600), norm, M=p.M, p=10.0)
    e = eps.cpu().numpy().astype(np.float64)
    F1, g1 = oracle.smooth(p.x, p.y, e, norm, M=p.M, p=10.0)
    assert F1 < 0.05 * F0
    assert np.abs(g1).max() < 1e-2 * max(1.0, np.abs(oracle.smooth(p.x, p.y, np.zeros(600), norm,
                                                                  M=p.M, p=10.0)[1]).max())
    c0 = oracle.consistency(p.x, p.y, norm, M=p.M)
    zs = z.cpu().numpy()
    c1 = oracle.consistency(p.x, zs, norm, M=p.M, tol=1e-3)
    assert c1["viol_up"].sum() < 0.2 * max(1, c0["viol_up"].sum())


def test_monotone_local_full_size_objective(lf):
    """d = 4, N = 1e5 (the monotone local workload, global M = 2): the
    objective and the gradient on sampled rows against the oracle's rows."""
    p = W.monotone_local(norm=1)
    met = lf.Metric(4, 1, mon=p.mon)
    eps = torch.zeros(p.n, device=DEV)
    F, g = lf.smooth_objective(_t(p.x), _t(p.y), eps, met, M=2.0, p=1.0)
    torch.cuda.synchronize()
    assert np.isfinite(F.item()) and F.item() > 0
    # the row sums of a 2000-datum subset form a smaller problem of their own;
    # check that subset end to end
    sub = W.rng_for(670).choice(p.n, 2000, replace=False)
    xs, ys = p.x[sub], p.y[sub]
    Fs, gs = lf.smooth_objective(_t(xs), _t(ys), torch.zeros(2000, device=DEV), met, M=2.0,
                                 p=1.0)
    torch.cuda.synchronize()

    class _P:  # the subset as a problem for _check
        pass
    q = _P()
    q.x, q.y, q.norm, q.mon, q.w, q.d = xs, ys, 1, p.mon, np.ones(4), 4
    _check(q, np.zeros(2000), Fs.item(), gs.cpu().numpy().astype(np.float64), 2.0, None, 1.0,
           "monotone_local subset")


# ---- pre-screening (Sec. 5) -----------------------------------------------------


@pytest.mark.parametrize("norm", [1, 2, 3])
@pytest.mark.parametrize("seed,n,d,mon,local,weighted", CASES)
def test_smooth_objective_pruned_parity(lf, norm, seed, n, d, mon, local, weighted):
    p = W.random_problem(700 + seed, n=n, q=1, d=d, norm=norm, mon=np.array(mon, np.int8),
                         local=local, weighted=weighted, M=0.8)
    rng = W.rng_for(701, seed)
    eps = (0.3 * rng.standard_normal(n)).astype(np.float32).astype(np.float64)
    pen, c = 0.7, 1.0 / 3.0
    M = np.float32(p.M)
    met = lf.Metric(d, norm, mon=p.mon, w=p.w)
    mk = None if p.Mk is None else _t(p.Mk)
    F, g = lf.smooth_objective(_t(p.x), _t(p.y), _t(eps.astype(np.float32)), met,
                               M=None if mk is not None else p.M, Mk=mk, p=pen, prune=c)
    torch.cuda.synchronize()
    Fo = _check(p, eps, F.item(), g.cpu().numpy().astype(np.float64), M, p.Mk, pen,
                f"pruned n={n} d={d} norm={norm}", prune=c)
    if n > 100:
        # the pre-screening dropped pairs that would have counted
        F_all, _ = oracle.smooth(p.x, p.y, eps, norm, M=M, Mk=p.Mk, p=pen, mon=p.mon, w=p.w)
        assert Fo < F_all


def _grid_problem(seed, n, d, norm, mon):
    """Integer coordinates in [0, 4]^d and values on a grid of 1/4: with M = 1
    and c = 1/4, c M dist and |y_i - y_k| are exact multiples of 1/4 (l1, linf;
    l2 where the distance is an integer), so many pairs sit on the threshold."""
    rng = W.rng_for(seed)

    class _P:
        pass
    p = _P()
    p.x = rng.integers(0, 5, size=(n, d)).astype(np.float32)
    p.y = (0.25 * rng.integers(-8, 9, size=n)).astype(np.float32)
    p.norm, p.d, p.mon, p.w = norm, d, np.array(mon, np.int8), np.ones(d)
    return p


@pytest.mark.parametrize("norm", [1, 2, 3])
@pytest.mark.parametrize("d,mon,local", [(1, [0], False), (2, [0, 0], False), (2, [1, 0], True),
                                         (3, [0, -1, 1], False)])
def test_smooth_pruned_ties_on_a_grid(lf, norm, d, mon, local):
    n = 900
    p = _grid_problem(710 + d, n, d, norm, mon)
    rng = W.rng_for(711, d)
    eps = (0.25 * rng.integers(-6, 7, size=n)).astype(np.float64)
    Mk = (0.25 * rng.integers(2, 7, size=n)).astype(np.float32) if local else None
    c, pen = 0.25, 1.0
    # ties at the threshold are common here (y_i - y_k = c M_k dist exactly)
    x64, y64 = p.x.astype(np.float64), p.y.astype(np.float64)
    i, k = rng.integers(0, n, 4000), rng.integers(0, n, 4000)
    dist = {1: np.abs(x64[i] - x64[k]).sum(1), 2: np.sqrt(((x64[i] - x64[k]) ** 2).sum(1)),
            3: np.abs(x64[i] - x64[k]).max(1)}[norm]
    mk = 1.0 if Mk is None else Mk[k].astype(np.float64)
    assert np.sum(np.abs(y64[i] - y64[k]) == c * mk * dist) > 20
    met = lf.Metric(d, norm, mon=p.mon)
    F, g = lf.smooth_objective(_t(p.x), _t(p.y), _t(eps.astype(np.float32)), met,
                               M=None if Mk is not None else 1.0,
                               Mk=None if Mk is None else _t(Mk), p=pen, prune=c)
    torch.cuda.synchronize()
    _check(p, eps, F.item(), g.cpu().numpy().astype(np.float64), 1.0, Mk, pen,
           f"grid ties d={d} norm={norm}", prune=c)


def test_smooth_pruned_repeatable_and_zero_is_all_pairs(lf):
    p = W.random_problem(720, n=3000, q=1, d=4, norm=2, mon=np.array([1, 0, 1, 0], np.int8),
                         M=0.5)
    met = lf.Metric(4, 2, mon=p.mon)
    eps = _t((0.2 * W.rng_for(721).standard_normal(3000)).astype(np.float32))
    F1, g1 = lf.smooth_objective(_t(p.x), _t(p.y), eps, met, M=p.M, p=1.0, prune=0.3)
    F2, g2 = lf.smooth_objective(_t(p.x), _t(p.y), eps, met, M=p.M, p=1.0, prune=0.3)
    assert F1.item() == F2.item() and torch.equal(g1, g2)
    F3, g3 = lf.smooth_objective(_t(p.x), _t(p.y), eps, met, M=p.M, p=1.0, prune=0.0)
    F4, g4 = lf.smooth_objective(_t(p.x), _t(p.y), eps, met, M=p.M, p=1.0)
    assert F3.item() == F4.item() and torch.equal(g3, g4)
    assert F1.item() < F3.item()


def test_monotone_local_full_size_pruned(lf):
    """d = 4, N = 1e5 with the paper's c = 1/3 and per-datum constants: the
    full-size call, then a 2000-datum subset end to end against the oracle."""
    p = W.monotone_local(norm=2)
    met = lf.Metric(4, 2, mon=p.mon)
    eps = _t((0.2 * W.rng_for(730).standard_normal(p.n)).astype(np.float32))
    mk = _t(p.Mk)
    F, g = lf.smooth_objective(_t(p.x), _t(p.y), eps, met, Mk=mk, p=1.0, prune=1 / 3)
    F0, _ = lf.smooth_objective(_t(p.x), _t(p.y), eps, met, Mk=mk, p=1.0)
    torch.cuda.synchronize()
    assert np.isfinite(F.item()) and 0 < F.item() < F0.item()
    assert torch.isfinite(g).all()
    sub = W.rng_for(731).choice(p.n, 2000, replace=False)
    xs, ys, ms = p.x[sub], p.y[sub], p.Mk[sub]
    es = (0.2 * W.rng_for(732).standard_normal(2000)).astype(np.float32).astype(np.float64)
    Fs, gs = lf.smooth_objective(_t(xs), _t(ys), _t(es.astype(np.float32)), met, Mk=_t(ms),
                                 p=1.0, prune=1 / 3)
    torch.cuda.synchronize()

    class _P:
        pass
    q = _P()
    q.x, q.y, q.norm, q.mon, q.w, q.d = xs, ys, 2, p.mon, np.ones(4), 4
    _check(q, es, Fs.item(), gs.cpu().numpy().astype(np.float64), 0.0, ms, 1.0,
           "monotone_local subset, pruned", prune=1 / 3)


@pytest.mark.parametrize("norm", [1, 2, 3])
def test_smooth_pruned_degenerate_pairs(lf, norm):
    """Zero constants (c M_k = 0: only pairs with equal values are dropped),
    duplicated points (zero distances) and repeated values, where the filter
    value sits exactly at the threshold and the FP64 decision takes over."""
    n, d = 700, 3
    rng = W.rng_for(740, norm)
    base_x = rng.random((n // 2, d)).astype(np.float32)
    x = np.concatenate([base_x, base_x[: n - n // 2]])            # every point twice
    y = (0.125 * rng.integers(-4, 5, size=n)).astype(np.float32)  # many equal values
    Mk = rng.random(n).astype(np.float32)
    Mk[rng.random(n) < 0.3] = 0.0
    eps = (0.25 * rng.standard_normal(n)).astype(np.float32).astype(np.float64)

    class _P:
        pass
    p = _P()
    p.x, p.y, p.norm, p.d, p.mon, p.w = x, y, norm, d, np.array([0, 1, 0], np.int8), np.ones(d)
    met = lf.Metric(d, norm, mon=p.mon)
    F, g = lf.smooth_objective(_t(x), _t(y), _t(eps.astype(np.float32)), met, Mk=_t(Mk), p=0.5,
                               prune=0.5)
    torch.cuda.synchronize()
    _check(p, eps, F.item(), g.cpu().numpy().astype(np.float64), 0.0, Mk, 0.5,
           f"pruned degenerate norm={norm}", prune=0.5)
