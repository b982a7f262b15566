"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

None of these tests re-types the oracle's formulas: each compares it with a
library routine (scipy cdist / pdist / cKDTree), a closed form derived from
Eq. (2) (1-D envelopes, N = 1, M = 0, constant data), the invariants of the
optimal interpolant (Sec. 3 and 4.1: containment of every admissible f,
interpolation, Lipschitz continuity, monotonicity), exact rational brute force
on tiny dyadic inputs, hand-worked examples (tests/golden) or finite
differences of the oracle's own forward.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.spatial import cKDTree
from scipy.spatial.distance import cdist, pdist

import oracle
import workloads as W

L1, L2, LINF = oracle.L1, oracle.L2, oracle.LINF
NORMS = [L1, L2, LINF]
SCIPY_METRIC = {L1: "cityblock", L2: "euclidean", LINF: "chebyshev"}
KD_P = {L1: 1, L2: 2, LINF: np.inf}
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")


def _rng(seed):
    return np.random.default_rng(seed)


def _lipschitz_ok(h_a, h_b, dist_ab, M, rel=1e-12):
    return np.all(np.abs(h_a - h_b) <= M * dist_ab * (1 + rel) + 1e-12)


# ---------------------------------------------------------------- hand examples

def test_hand_worked_examples():
    with open(GOLDEN) as f:
        cases = json.load(f)
    for c in cases:
        norm = {"l1": L1, "l2": L2, "linf": LINF}[c["norm"]]
        x = np.array([[float(Fraction(v)) for v in row] for row in c["x"]], np.float32)
        y = np.array([float(Fraction(v)) for v in c["y"]], np.float32)
        Mk = None if "Mk" not in c else np.array([float(Fraction(v)) for v in c["Mk"]], np.float32)
        mon = np.array(c["mon"], np.int8)
        xq = np.array([[float(Fraction(v)) for v in qq["xq"]] for qq in c["queries"]], np.float32)
        hu, hl, g, au, al = oracle.bounds(x, y, xq, norm, M=float(Fraction(c["M"])), Mk=Mk, mon=mon)
        for j, qq in enumerate(c["queries"]):
            assert hu[j] == float(Fraction(qq["h_up"])), (c["name"], j)
            assert hl[j] == float(Fraction(qq["h_lo"])), (c["name"], j)
            assert g[j] == float(Fraction(qq["g"])), (c["name"], j)
            assert au[j] == qq["arg_up"] and al[j] == qq["arg_lo"], (c["name"], j)


# ---------------------------------------------------------------- library reductions

@pytest.mark.parametrize("norm", NORMS)
@pytest.mark.parametrize("local", [False, True])
def test_unconstrained_equals_scipy_cdist(norm, local):
    """Without monotone coordinates Eq. (2) is min/max over y + M * cdist."""
    p = W.random_problem(1, n=300, q=400, d=3, norm=norm, local=local, weighted=True)
    w64 = p.w.astype(np.float64)
    D = cdist(p.xq.astype(np.float64) * w64, p.x.astype(np.float64) * w64, SCIPY_METRIC[norm])
    Mv = p.Mk.astype(np.float64) if local else np.full(p.n, p.M)
    U = p.y.astype(np.float64)[None, :] + Mv[None, :] * D
    L = p.y.astype(np.float64)[None, :] - Mv[None, :] * D
    hu, hl, g, au, al = oracle.bounds(p.x, p.y, p.xq, norm, M=p.M, Mk=p.Mk, w=p.w)
    np.testing.assert_allclose(hu, U.min(1), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(hl, L.max(1), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(g, 0.5 * (U.min(1) + L.max(1)), rtol=1e-12, atol=1e-12)
    # indices where the winner is clear of the runner-up
    su, sl = np.sort(U, 1), np.sort(L, 1)
    clear_u = (su[:, 1] - su[:, 0]) > 1e-9
    clear_l = (sl[:, -1] - sl[:, -2]) > 1e-9
    assert clear_u.mean() > 0.95 and clear_l.mean() > 0.95
    np.testing.assert_array_equal(au[clear_u], U.argmin(1)[clear_u])
    np.testing.assert_array_equal(al[clear_l], L.argmax(1)[clear_l])


@pytest.mark.parametrize("norm", NORMS)
def test_constant_data_selects_nearest_neighbour(norm):
    """y = c: both bounds pick the nearest datum (cKDTree), H_up - c = M * NN distance."""
    g0 = _rng(7)
    x = g0.random((500, 4)).astype(np.float32)
    y = np.full(500, 0.75, np.float32)
    xq = g0.random((300, 4)).astype(np.float32)
    tree = cKDTree(x.astype(np.float64))
    dnn, inn = tree.query(xq.astype(np.float64), k=1, p=KD_P[norm])
    hu, hl, g, au, al = oracle.bounds(x, y, xq, norm, M=3.0)
    np.testing.assert_array_equal(au, inn)
    np.testing.assert_array_equal(al, inn)
    np.testing.assert_allclose(hu - 0.75, 3.0 * dnn, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(0.75 - hl, 3.0 * dnn, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(g, 0.75, atol=1e-15)


@pytest.mark.parametrize("norm", NORMS)
def test_error_bound_uses_nearest_distance(norm):
    """Sec. 3: (H_up - H_lo)/2 <= M * min_k dist(x, x^k) (nearest datum from cKDTree)."""
    p = W.random_problem(2, n=400, q=500, d=3, norm=norm)
    hu, hl, g, au, al = oracle.bounds(p.x, p.y, p.xq, norm, M=p.M)
    dnn, _ = cKDTree(p.x.astype(np.float64)).query(p.xq.astype(np.float64), k=1, p=KD_P[norm])
    assert np.all(0.5 * (hu - hl) <= p.M * dnn * (1 + 1e-12) + 1e-15)


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("norm", NORMS)
def test_1d_envelope_closed_form(norm):
    """Consistent sorted 1-D data: only the two bracketing points matter, and
    g is the constant end value outside the hull."""
    g0 = _rng(3)
    n, M = 60, 2.0
    xs = np.sort(g0.random(n)).astype(np.float32)
    steps = np.diff(xs.astype(np.float64)) * g0.uniform(-0.9, 0.9, n - 1) * M
    ys = np.concatenate([[0.3], 0.3 + np.cumsum(steps)]).astype(np.float32)
    # re-check consistency in float64 on the float32 values
    assert np.all(np.abs(np.diff(ys.astype(np.float64))) <= M * np.diff(xs.astype(np.float64)))
    xq = np.concatenate([g0.uniform(-0.3, 1.3, 400), xs[:5]]).astype(np.float32)
    hu, hl, g, au, al = oracle.bounds(xs[:, None], ys, xq[:, None], norm, M=M)
    X, Y, XQ = xs.astype(np.float64), ys.astype(np.float64), xq.astype(np.float64)
    for j, t in enumerate(XQ):
        if t <= X[0]:
            eu, el = Y[0] + M * (X[0] - t), Y[0] - M * (X[0] - t)
        elif t >= X[-1]:
            eu, el = Y[-1] + M * (t - X[-1]), Y[-1] - M * (t - X[-1])
        else:
            b = np.searchsorted(X, t)
            a = b - 1
            eu = min(Y[a] + M * (t - X[a]), Y[b] + M * (X[b] - t))
            el = max(Y[a] - M * (t - X[a]), Y[b] - M * (X[b] - t))
        assert abs(hu[j] - eu) <= 1e-12 and abs(hl[j] - el) <= 1e-12, j
    out = (XQ < X[0]) | (XQ > X[-1])
    ends = np.where(XQ[out] < X[0], Y[0], Y[-1])
    np.testing.assert_allclose(g[out], ends, atol=1e-12)
    # at the data the interpolant reproduces y
    np.testing.assert_allclose(g[-5:], Y[:5], atol=1e-12)


def test_1d_monotone_closed_form():
    """Eq. (4), increasing 1-D data with slopes in [0, M]:
    H_up = min(y_b, y_a + M (x - x_a)), H_lo = max(y_a, y_b - M (x_b - x))."""
    g0 = _rng(4)
    n, M = 50, 1.5
    xs = np.sort(g0.random(n)).astype(np.float32)
    steps = np.diff(xs.astype(np.float64)) * g0.uniform(0.0, 0.95, n - 1) * M
    ys = np.concatenate([[0.0], np.cumsum(steps)]).astype(np.float32)
    X, Y = xs.astype(np.float64), ys.astype(np.float64)
    assert np.all(np.diff(Y) >= 0) and np.all(np.diff(Y) <= M * np.diff(X))
    xq = g0.uniform(X[0], X[-1], 300).astype(np.float32)
    for norm in NORMS:
        hu, hl, g, au, al = oracle.bounds(xs[:, None], ys, xq[:, None], norm, M=M,
                                          mon=np.array([1], np.int8))
        for j, t in enumerate(xq.astype(np.float64)):
            b = np.searchsorted(X, t)
            a = max(b - 1, 0)
            eu = min(Y[b], Y[a] + M * (t - X[a]))
            el = max(Y[a], Y[b] - M * (X[b] - t))
            assert abs(hu[j] - eu) <= 1e-12 and abs(hl[j] - el) <= 1e-12


@pytest.mark.parametrize("norm", NORMS)
def test_decreasing_is_mirror_of_increasing(norm):
    """mon = -1 on x equals mon = +1 on -x (Sec. 4.1: 'w.l.o.g. increasing')."""
    p = W.random_problem(5, n=200, q=150, d=3, norm=norm, local=True)
    mon_dec = np.array([-1, 0, 1], np.int8)
    mon_inc = np.array([1, 0, 1], np.int8)
    flip = np.array([-1.0, 1.0, 1.0], np.float32)
    a = oracle.bounds(p.x, p.y, p.xq, norm, Mk=p.Mk, mon=mon_dec)
    b = oracle.bounds(p.x * flip, p.y, p.xq * flip, norm, Mk=p.Mk, mon=mon_inc)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)


@pytest.mark.parametrize("norm", NORMS)
def test_single_datum_and_zero_constant(norm):
    g0 = _rng(6)
    x = g0.random((1, 3)).astype(np.float32)
    y = np.array([0.4], np.float32)
    xq = g0.random((50, 3)).astype(np.float32)
    D = cdist(xq.astype(np.float64), x.astype(np.float64), SCIPY_METRIC[norm])[:, 0]
    hu, hl, g, au, al = oracle.bounds(x, y, xq, norm, M=2.5)
    np.testing.assert_allclose(hu, float(np.float32(0.4)) + 2.5 * D, rtol=1e-12)
    np.testing.assert_allclose(hl, float(np.float32(0.4)) - 2.5 * D, rtol=1e-12)
    np.testing.assert_allclose(g, np.float32(0.4), rtol=1e-15)
    assert np.all(au == 0) and np.all(al == 0)
    # M = 0: the bounds are the extreme values of y, first occurrence
    p = W.random_problem(6, n=100, q=20, d=3, norm=norm)
    y2 = np.round(p.y, 1).astype(np.float32)  # create exact ties
    hu, hl, g, au, al = oracle.bounds(p.x, y2, p.xq, norm, M=0.0)
    assert np.all(hu == y2.min()) and np.all(hl == y2.max())
    assert np.all(au == np.argmin(y2)) and np.all(al == np.argmax(y2))


# ---------------------------------------------------------------- invariants

def _monotone_lipschitz_data(seed, n, d, norm, mon):
    """f(x) = a.x + b.clip(x) ramps: increasing along mon=+1 axes, decreasing
    along mon=-1 axes; M = dual norm of the slope bound (so f in Lip(M))."""
    g0 = _rng(seed)
    a = g0.uniform(-1, 1, d)
    a[mon > 0] = np.abs(a[mon > 0])
    a[mon < 0] = -np.abs(a[mon < 0])
    dual = {L1: lambda v: np.abs(v).max(), L2: lambda v: np.sqrt((v ** 2).sum()),
            LINF: lambda v: np.abs(v).sum()}[norm]
    M = float(dual(a)) * 1.0000001
    f = lambda X: X.astype(np.float64) @ a
    x = g0.random((n, d)).astype(np.float32)
    return x, f, M


@pytest.mark.parametrize("norm", NORMS)
def test_envelopes_are_the_tight_bounds(norm):
    """Sec. 3 / 4.1: every admissible f lies in [H_lo, H_up]; H_up and H_lo are
    themselves admissible (interpolating, M-Lipschitz, monotone) -> tight."""
    d = 3
    mon = np.array([1, 0, -1], np.int8)
    x, f, M = _monotone_lipschitz_data(11, 150, d, norm, mon)
    y = f(x).astype(np.float32)
    # the float32 rounding of y may break consistency by ~1e-8; add margin to M
    M = M * 1.001
    g0 = _rng(12)
    xq = g0.uniform(-0.2, 1.2, (600, d)).astype(np.float32)
    hu, hl, g, au, al = oracle.bounds(x, y, xq, norm, M=M, mon=mon)
    fv = f(xq)
    assert np.all(hl <= fv + 1e-6) and np.all(fv <= hu + 1e-6)
    # interpolation at the data
    hu_d, hl_d, g_d, _, _ = oracle.bounds(x, y, x, norm, M=M, mon=mon)
    np.testing.assert_allclose(g_d, y.astype(np.float64), atol=1e-12)
    np.testing.assert_allclose(hu_d, y.astype(np.float64), atol=1e-12)
    # Lipschitz continuity of H_up, H_lo and g under the symmetric norm
    a_pts = xq[:300]
    b_pts = (a_pts + g0.normal(0, 0.05, a_pts.shape)).astype(np.float32)
    ha = oracle.bounds(x, y, a_pts, norm, M=M, mon=mon)
    hb = oracle.bounds(x, y, b_pts, norm, M=M, mon=mon)
    dab = np.array([np.linalg.norm((a_pts[i].astype(np.float64) - b_pts[i]), ord=KD_P[norm])
                    for i in range(len(a_pts))])
    for k in range(3):
        assert _lipschitz_ok(ha[k], hb[k], dab, M)
    # monotonicity: moving up along coordinate 0 (increasing) never decreases,
    # moving up along coordinate 2 (decreasing) never increases
    step = np.zeros_like(a_pts)
    step[:, 0] = np.abs(g0.normal(0, 0.1, len(a_pts)))
    hp = oracle.bounds(x, y, (a_pts + step).astype(np.float32), norm, M=M, mon=mon)
    for k in range(3):
        assert np.all(hp[k] >= ha[k] - 1e-12)
    step = np.zeros_like(a_pts)
    step[:, 2] = np.abs(g0.normal(0, 0.1, len(a_pts)))
    hp = oracle.bounds(x, y, (a_pts + step).astype(np.float32), norm, M=M, mon=mon)
    for k in range(3):
        assert np.all(hp[k] <= ha[k] + 1e-12)


@pytest.mark.parametrize("norm", NORMS)
def test_range_preservation_any_data(norm):
    """Sec. 6 (range preservation), any data, symmetric distance:
    y[arg_up] <= g <= y[arg_lo] and min y <= g <= max y."""
    p = W.random_problem(13, n=300, q=400, d=4, norm=norm, local=True)
    hu, hl, g, au, al = oracle.bounds(p.x, p.y, p.xq, norm, Mk=p.Mk)
    yd = p.y.astype(np.float64)
    assert np.all(yd[au] <= g + 1e-12) and np.all(g <= yd[al] + 1e-12)
    assert np.all(yd.min() <= g + 1e-12) and np.all(g <= yd.max() + 1e-12)


# ---------------------------------------------------------------- exact rational brute force

def _dyadic_problem(seed, n, d):
    g0 = _rng(seed)
    x = (g0.integers(0, 9, (n, d)) / 8.0).astype(np.float32)
    y = (g0.integers(-8, 9, n) / 4.0).astype(np.float32)
    Mk = (g0.integers(1, 9, n) / 4.0).astype(np.float32)
    xq = (g0.integers(-2, 11, (12, d)) / 8.0).astype(np.float32)
    mon = g0.integers(-1, 2, d).astype(np.int8)
    return x, y, Mk, xq, mon


@pytest.mark.parametrize("norm", [L1, LINF])
@pytest.mark.parametrize("seed", range(6))
def test_exact_rational_brute_force(norm, seed):
    """Tiny dyadic inputs: every operation of Eq. (2)/(4) is exact in FP64, so the
    oracle must equal exact rational arithmetic, ties (lowest index) included."""
    n, d = 8, 3
    x, y, Mk, xq, mon = _dyadic_problem(seed, n, d)
    hu, hl, g, au, al = oracle.bounds(x, y, xq, norm, Mk=Mk, mon=mon)
    Fx = [[Fraction(float(v)) for v in r] for r in x]
    Fy = [Fraction(float(v)) for v in y]
    FM = [Fraction(float(v)) for v in Mk]
    pos = lambda v: v if v > 0 else Fraction(0)
    for j in range(xq.shape[0]):
        q = [Fraction(float(v)) for v in xq[j]]
        cu_all, cl_all = [], []
        for k in range(n):
            cu, cl = [], []
            for i in range(d):
                dl = q[i] - Fx[k][i]
                if mon[i] == 0:
                    cu.append(abs(dl)); cl.append(abs(dl))
                elif mon[i] > 0:
                    cu.append(pos(dl)); cl.append(pos(-dl))
                else:
                    cu.append(pos(-dl)); cl.append(pos(dl))
            agg = sum if norm == L1 else max
            cu_all.append(Fy[k] + FM[k] * agg(cu))
            cl_all.append(Fy[k] - FM[k] * agg(cl))
        eu, el = min(cu_all), max(cl_all)
        assert Fraction(hu[j]) == eu and Fraction(hl[j]) == el
        assert au[j] == cu_all.index(eu) and al[j] == cl_all.index(el)
        assert Fraction(g[j]) == (eu + el) / 2


# ---------------------------------------------------------------- consistency check

@pytest.mark.parametrize("norm", NORMS)
def test_consistency_1d_closed_form(norm):
    """1-D, global M: consistent iff every adjacent slope is <= M (np.diff);
    increasing constraint adds Delta y >= 0.  Counts match scipy pdist pairs."""
    g0 = _rng(21)
    n, M = 80, 1.0
    xs = np.sort(g0.random(n)).astype(np.float32)
    ys = np.cumsum(g0.uniform(-1.3, 1.3, n) * np.r_[0.0, np.diff(xs)]).astype(np.float32)
    X, Y = xs.astype(np.float64), ys.astype(np.float64)
    r = oracle.consistency(xs[:, None], ys, norm, M=M)
    adj_ok = np.all(np.abs(np.diff(Y)) <= M * np.diff(X))
    all_ok = (r["viol_up"].sum() == 0) and (r["viol_lo"].sum() == 0)
    assert adj_ok == all_ok
    assert (np.min(r["slack_up"]) >= 0) == adj_ok
    # number of violating unordered pairs from scipy pdist
    nbad = int(np.sum(pdist(Y[:, None]) > M * pdist(X[:, None])))
    assert r["viol_up"].sum() == nbad and r["viol_lo"].sum() == nbad  # mirror symmetry
    # monotone increasing adds a second condition
    rm = oracle.consistency(xs[:, None], ys, norm, M=M, mon=np.array([1], np.int8))
    adj_mon = adj_ok and np.all(np.diff(Y) >= 0)
    assert (rm["viol_up"].sum() == 0 and rm["viol_lo"].sum() == 0) == adj_mon


def test_consistency_equality_is_allowed():
    """|y_i - y_k| = M d exactly is consistent (the Lipschitz condition is <=)."""
    x = np.array([[0.0], [0.5], [1.5]], np.float32)
    y = np.array([0.0, 1.0, 3.0], np.float32)  # slopes exactly 2
    for norm in NORMS:
        r = oracle.consistency(x, y, norm, M=2.0)
        assert r["viol_up"].sum() == 0 and r["viol_lo"].sum() == 0
        assert np.min(r["slack_up"]) == 0.0
        r = oracle.consistency(x, y, norm, M=1.999)
        assert r["viol_up"].sum() == 3 and r["viol_lo"].sum() == 3


@pytest.mark.parametrize("norm", NORMS)
def test_consistency_iff_interpolation(norm):
    """Sec. 4.1 / Sec. 3: all slacks >= 0 <=> g(x^i) = y_i for every datum."""
    for seed, M in [(31, 8.0), (32, 0.3)]:
        p = W.random_problem(seed, n=120, q=1, d=2, norm=norm,
                             mon=np.array([1, 0], np.int8))
        r = oracle.consistency(p.x, p.y, norm, M=M, mon=p.mon)
        hu, hl, g, _, _ = oracle.bounds(p.x, p.y, p.x, norm, M=M, mon=p.mon)
        consistent = np.all(r["slack_up"] >= 0) and np.all(r["slack_lo"] >= 0)
        interp = np.all(np.abs(g - p.y.astype(np.float64)) <= 1e-12)
        assert consistent == interp
        # the slack is H_up(x^i) - y_i over the other data (excluding i itself)
        up_excl = np.minimum(r["slack_up"], 0.0)
        np.testing.assert_allclose(np.minimum(hu - p.y, 0.0), up_excl, atol=1e-12)


@pytest.mark.parametrize("norm", NORMS)
def test_consistency_injected_violation(norm):
    """Perturb one value: the rows flagged are exactly the pairs predicted by cdist."""
    g0 = _rng(41)
    n, M = 200, 2.0
    x = g0.random((n, 3)).astype(np.float32)
    y = (0.5 * x.astype(np.float64).sum(1) / 3).astype(np.float32)  # slope well below M
    j = 17
    y[j] += np.float32(0.3)
    r = oracle.consistency(x, y, norm, M=M)
    D = cdist(x.astype(np.float64), x.astype(np.float64), SCIPY_METRIC[norm])
    Y = y.astype(np.float64)
    # ordered pair (i,k) violates 'up' when y_i - y_k > M d
    V = (Y[:, None] - Y[None, :]) > M * D
    np.fill_diagonal(V, False)
    np.testing.assert_array_equal(r["viol_up"], V.sum(1))
    np.testing.assert_array_equal(r["viol_lo"], V.sum(0))
    assert r["viol_up"][j] > 0 and r["viol_up"].sum() == r["viol_up"][j]


# ---------------------------------------------------------------- Lipschitz constant estimates

@pytest.mark.parametrize("norm", NORMS)
def test_global_M_1d_adjacent_slopes(norm):
    """In 1-D the largest slope over all pairs is attained by adjacent points."""
    g0 = _rng(51)
    xs = np.sort(g0.random(300)).astype(np.float32)
    ys = g0.standard_normal(300).astype(np.float32)
    st, M, (i, k) = oracle.estimate_M_global(xs[:, None], ys, norm)
    X, Y = xs.astype(np.float64), ys.astype(np.float64)
    sl = np.abs(np.diff(Y)) / np.diff(X)
    assert st == 0
    assert M == pytest.approx(sl.max(), rel=1e-14)
    t = int(np.argmax(sl))
    assert (i, k) == (t, t + 1)


@pytest.mark.parametrize("norm", NORMS)
def test_global_M_matches_pdist(norm):
    p = W.random_problem(52, n=250, q=1, d=3, norm=norm, weighted=True)
    st, M, (i, k) = oracle.estimate_M_global(p.x, p.y, norm, w=p.w)
    w64 = p.w.astype(np.float64)
    R = pdist(p.y.astype(np.float64)[:, None]) / pdist(p.x.astype(np.float64) * w64,
                                                          SCIPY_METRIC[norm])
    assert st == 0 and M == pytest.approx(R.max(), rel=1e-13)
    # recover (i, k) of the pdist argmax (condensed index order is i < k lexicographic)
    n = p.n
    idx = int(np.argmax(R))
    ii = int(n - 2 - np.floor(np.sqrt(-8 * idx + 4 * n * (n - 1) - 7) / 2.0 - 0.5))
    kk = int(idx + ii + 1 - n * (n - 1) // 2 + (n - ii) * ((n - ii) - 1) // 2)
    assert (i, k) == (ii, kk)


def test_global_M_duplicates():
    x = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 0.0], [1.0, 0.0]], np.float32)
    y = np.array([0.0, 1.0, 0.0, 1.0], np.float32)
    st, M, pair = oracle.estimate_M_global(x, y, L2)  # equal duplicates are skipped
    assert st == 0 and M == 1.0 and pair == (0, 1)
    y2 = np.array([0.0, 1.0, 0.5, 1.0], np.float32)
    st, M, pair = oracle.estimate_M_global(x, y2, L2)
    assert st == 3 and pair == (0, 2) and M == np.inf


@pytest.mark.parametrize("norm", NORMS)
def test_knn_M_matches_ckdtree(norm):
    """Sec. 4.3 scalar form: the 16 nearest neighbours from cKDTree, then the max slope."""
    p = W.random_problem(61, n=600, q=1, d=4, norm=norm)
    K = 16
    st, Mi, nbr = oracle.estimate_M_knn(p.x, p.y, norm, K=K)
    assert st == 0
    X = p.x.astype(np.float64)
    dd, ii = cKDTree(X).query(X, k=K + 1, p=KD_P[norm])
    Y = p.y.astype(np.float64)
    for r in range(p.n):
        keep = ii[r] != r
        nb, dist = ii[r][keep][:K], dd[r][keep][:K]
        assert set(nb.tolist()) == set(nbr[r].tolist())
        exp = np.max(np.abs(Y[r] - Y[nb]) / dist)
        assert Mi[r] == pytest.approx(exp, rel=1e-12)


def test_knn_small_n_and_ties():
    # n - 1 < K: all other points are neighbours; ties rank the lower index first
    x = np.array([[0.0], [1.0], [-1.0], [2.0]], np.float32)
    y = np.array([0.0, 1.0, 3.0, 0.0], np.float32)
    st, Mi, nbr = oracle.estimate_M_knn(x, y, L1, K=2)
    assert st == 0
    assert nbr[0].tolist() == [1, 2]  # both at distance 1: lower index first
    assert Mi[0] == 3.0  # max(|0-1|/1, |0-3|/1)
    st, Mi, nbr = oracle.estimate_M_knn(x, y, L1, K=16)
    assert nbr[0].tolist()[:3] == [1, 2, 3] and nbr[0][3] == -1


# ---------------------------------------------------------------- gradients

def _near_kink(p, j, k, up, h):
    """True if the distance from query j to datum k (upper when up, else
    lower) has a kink within h of the query: a coordinate difference within
    2h of 0 (|.| and (.)_+ kinks), or, for linf, its two largest weighted
    components within 2 h max(w) of each other (the maximum switches)."""
    delta = p.xq[j].astype(np.float64) - p.x[k].astype(np.float64)
    if np.any(np.abs(delta) < 2 * h):
        return True
    if p.norm == LINF:
        m = p.mon.astype(np.int64)
        pos, neg = np.maximum(delta, 0.0), np.maximum(-delta, 0.0)
        comp = np.where(m == 0, np.abs(delta), np.where((m > 0) == up, pos, neg)) * p.w
        top = np.sort(comp)[::-1]
        if top.size > 1 and top[0] - top[1] < 2 * h * float(np.max(p.w)):
            return True
    return False


def _fd_check(norm, mon, local, seed, bounds_grads=False):
    """Finite differences of the oracle forward against oracle.grad for the
    objective sum_j dg_j g_j (+ dh_up_j H_up_j + dh_lo_j H_lo_j)."""
    p = W.random_problem(seed, n=200, q=60, d=3, norm=norm, mon=mon, local=local,
                         weighted=(seed % 2 == 0))
    kw = dict(M=p.M, Mk=p.Mk, mon=p.mon, w=p.w)
    hu, hl, g, au, al = oracle.bounds(p.x, p.y, p.xq, norm, **kw)
    dg = p.dg.astype(np.float64)
    gen = W.rng_for(seed, 2)
    dhu = gen.standard_normal(p.q) if bounds_grads else np.zeros(p.q)
    dhl = gen.standard_normal(p.q) if bounds_grads else np.zeros(p.q)
    dxq, dy, dM = oracle.grad(p.x, p.y, p.xq, norm, au, al, dg=dg, dh_up=dhu, dh_lo=dhl, **kw)
    obj = lambda r, j: dg[j] * r[2] + dhu[j] * r[0] + dhl[j] * r[1]
    h = 2.0 ** -14
    checked = 0
    for j in range(p.q):
        if _near_kink(p, j, au[j], True, h) or _near_kink(p, j, al[j], False, h):
            continue
        num = np.zeros(p.d)
        ok = True
        for i in range(p.d):
            xp, xm = p.xq[j:j + 1].copy(), p.xq[j:j + 1].copy()
            xp[0, i] += np.float32(h)
            xm[0, i] -= np.float32(h)
            step = float(xp[0, i]) - float(xm[0, i])
            rp = oracle.bounds(p.x, p.y, xp, norm, **kw)
            rm = oracle.bounds(p.x, p.y, xm, norm, **kw)
            # stay on one piece: the same selected data on both sides
            if not (rp[3][0] == rm[3][0] == au[j] and rp[4][0] == rm[4][0] == al[j]):
                ok = False
                break
            num[i] = (obj(rp, j)[0] - obj(rm, j)[0]) / step
        if not ok:
            continue
        # l1 / linf are linear on the piece (exact up to rounding); l2 has an
        # O(h^2) curvature term
        tol = 1e-5 if norm == L2 else 1e-9
        scale = abs(dg[j]) + abs(dhu[j]) + abs(dhl[j])
        np.testing.assert_allclose(num, dxq[j], rtol=tol, atol=tol * scale)
        checked += 1
    assert checked >= 0.95 * p.q, f"only {checked} of {p.q} queries checked"
    # y and M: g is affine in y and M on a piece; directional differences
    # along seeded random directions (perturbed values rounded to FP32 like
    # every input, the differences taken over the actual perturbation), over
    # the queries whose selection the step leaves unchanged
    rng = W.rng_for(seed, 1)
    for which in ("y", "M"):
        v = rng.standard_normal(p.n)
        if which == "M" and not local:
            e = 2.0 ** -12
            rp = oracle.bounds(p.x, p.y, p.xq, norm, M=p.M + e, mon=p.mon, w=p.w)
            rm = oracle.bounds(p.x, p.y, p.xq, norm, M=p.M - e, mon=p.mon, w=p.w)
        else:
            base = (p.y if which == "y" else p.Mk).astype(np.float64)
            e = 2.0 ** -12 * (1.0 if which == "y" else base)
            vp, vm = (base + e * v).astype(np.float32), (base - e * v).astype(np.float32)
            delta = vp.astype(np.float64) - vm.astype(np.float64)
            if which == "y":
                rp = oracle.bounds(p.x, vp, p.xq, norm, **kw)
                rm = oracle.bounds(p.x, vm, p.xq, norm, **kw)
            else:
                rp = oracle.bounds(p.x, p.y, p.xq, norm, M=p.M, Mk=vp, mon=p.mon, w=p.w)
                rm = oracle.bounds(p.x, p.y, p.xq, norm, M=p.M, Mk=vm, mon=p.mon, w=p.w)
        same = (rp[3] == au) & (rm[3] == au) & (rp[4] == al) & (rm[4] == al)
        assert same.mean() >= 0.9, f"{which}: the step changed {(~same).sum()} selections"
        _, dy_s, dM_s = oracle.grad(p.x, p.y, p.xq[same], norm, au[same], al[same],
                                    dg=dg[same], dh_up=dhu[same], dh_lo=dhl[same], **kw)
        idx = np.nonzero(same)[0]
        full = np.arange(p.q)
        num = float(np.sum((obj(rp, full) - obj(rm, full))[idx]))
        if which == "M" and not local:
            ana = 2 * e * float(dM_s[0])
        else:
            ana = float((dy_s if which == "y" else dM_s) @ delta)
        assert num == pytest.approx(ana, rel=1e-7, abs=1e-12), which


@pytest.mark.parametrize("norm", NORMS)
def test_gradient_matches_finite_differences(norm):
    _fd_check(norm, np.zeros(3, np.int8), False, 71)
    _fd_check(norm, np.array([1, 0, -1], np.int8), True, 72)
    _fd_check(norm, np.array([0, 1, 1], np.int8), False, 73, bounds_grads=True)
    _fd_check(norm, np.array([-1, 0, 0], np.int8), True, 74, bounds_grads=True)


def test_gradient_kink_conventions():
    """Hand-worked subgradients at exact kinks (reading: |.|'(0) = 0,
    (.)_+'(0) = 0, linf takes the lowest coordinate among the largest
    components).  One datum at the origin, y = 0, M = 2, dg = 1, so
    g = (H_up + H_lo) / 2 and dxq = (M grad dist_up - M grad dist_lo) / 2,
    or with dh_up = 1 alone, dxq = M grad dist_up."""
    x = np.zeros((1, 2), np.float32)
    y = np.zeros(1, np.float32)
    one = np.ones(1)
    zero = np.zeros(1, np.int64)
    # H_up = y + M dist_up alone (dh_up = 1): dxq = M grad dist_up.
    # linf, free coordinates, query (1, -1): both components equal 1; the
    # first coordinate carries the subgradient: grad dist = (1, 0)
    dxq, _, _ = oracle.grad(x, y, np.array([[1.0, -1.0]], np.float32), LINF, zero, zero,
                            dh_up=one, M=2.0)
    assert dxq.tolist() == [[2.0, 0.0]]
    # l1 with a zero difference in coordinate 1: |.|'(0) = 0
    dxq, _, _ = oracle.grad(x, y, np.array([[0.5, 0.0]], np.float32), L1, zero, zero,
                            dh_up=one, M=2.0)
    assert dxq.tolist() == [[2.0, 0.0]]
    # a single datum with the symmetric distance: g = y, gradient 0
    dxq, _, _ = oracle.grad(x, y, np.array([[0.3, -0.7]], np.float32), L2, zero, zero, dg=one,
                            M=2.0)
    assert dxq.tolist() == [[0.0, 0.0]]
    # l1, coordinate 0 increasing, query (-0.5, 0.25): dist_up = 0 + 0.25,
    # dist_lo = 0.5 + 0.25; grad up = (0, 1), grad lo = (-1, 1):
    # dxq = (M (0, 1) - M (-1, 1)) / 2 = (1, 0)
    dxq, _, _ = oracle.grad(x, y, np.array([[-0.5, 0.25]], np.float32), L1, zero, zero, dg=one,
                            M=2.0, mon=np.array([1, 0], np.int8))
    assert dxq.tolist() == [[1.0, 0.0]]
    # l2 at distance 0: gradient 0
    dxq, _, _ = oracle.grad(x, y, np.zeros((1, 2), np.float32), L2, zero, zero, dg=one, M=2.0)
    assert dxq.tolist() == [[0.0, 0.0]]
