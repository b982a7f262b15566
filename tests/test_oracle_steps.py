"""Pins of the oracle's step-function local constants (Sec. 4.3).

Each test compares the oracle with something other than its own formulas:
hand-worked examples (tests/golden/step_examples.json), library routines
(numpy's inverted-CDF quantile, scipy cdist / cKDTree), the interpolation
property the section claims for the construction, the oracle's already
pinned global-constant and bound functions in the special cases that reduce
to them, and the structure of the table (non-decreasing steps).
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.spatial import cKDTree
from scipy.spatial.distance import cdist

import oracle

L1, L2, LINF = oracle.L1, oracle.L2, oracle.LINF
NORMS = [L1, L2, LINF]
SCIPY_METRIC = {L1: "cityblock", L2: "euclidean", LINF: "chebyshev"}
KD_P = {L1: 1, L2: 2, LINF: np.inf}
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "step_examples.json")


def _fr(v):
    return float(Fraction(v))


def _problem(seed, n, d, dyadic=False):
    rng = np.random.default_rng(seed)
    x = rng.random((n, d))
    if dyadic:
        x = np.round(x * 64) / 64
    y = np.sin(3 * x[:, 0]) + x[:, -1] ** 2 + 0.05 * rng.standard_normal(n)
    return x.astype(np.float32), y.astype(np.float32)


def test_hand_worked_examples():
    with open(GOLDEN) as f:
        cases = json.load(f)["cases"]
    assert len(cases) == 5
    for c in cases:
        norm = {"l1": L1, "l2": L2, "linf": LINF}[c["norm"]]
        x = np.array([[_fr(v) for v in r] for r in c["x"]], np.float32)
        y = np.array([_fr(v) for v in c["y"]], np.float32)
        kn = np.array([_fr(v) for v in c["knots"]])
        st, d1, V = oracle.local_steps(x, y, kn, norm)
        assert st == 0
        np.testing.assert_array_equal(d1, [_fr(v) for v in c["d1"]], err_msg=c["name"])
        np.testing.assert_array_equal(V, [[_fr(v) for v in r] for r in c["V"]], err_msg=c["name"])
        if not c["queries"]:
            continue
        mon = None if c["mon"] is None else np.array(c["mon"], np.int8)
        xq = np.array([[_fr(v) for v in qq["xq"]] for qq in c["queries"]], np.float32)
        # the bounds multiply the FP32 table rounded up; exact hand values
        # agree to its rounding, the attaining indices (ties included) exactly
        hu, hl, g, au, al = oracle.bounds_step(x, y, xq, norm, kn, d1, oracle.round_up_f32(V),
                                               mon=mon)
        for j, qq in enumerate(c["queries"]):
            for name, got in (("h_up", hu[j]), ("h_lo", hl[j]), ("g", g[j])):
                want = _fr(qq[name])
                assert abs(got - want) <= 1e-6 * max(1.0, abs(want)), (c["name"], j, name)
            assert (au[j], al[j]) == (qq["arg_up"], qq["arg_lo"]), (c["name"], j)


@pytest.mark.parametrize("norm", NORMS)
@pytest.mark.parametrize("m", [1000, 1001])
def test_knots_are_numpy_inverted_cdf_quantiles(norm, m):
    x, _ = _problem(1, 300, 3)
    w = np.array([1.0, 0.5, 2.0])
    rng = np.random.default_rng(2)
    pairs = rng.integers(0, 300, size=(m, 2))
    # m = 1000 puts several p * m exactly on an integer
    probs = np.array([0.001, 0.1, 0.25, 0.5, 0.9, 0.999, 1.0])
    got = oracle.knots(x, pairs, probs, norm, w=w)
    xs = x.astype(np.float64) * w
    dists = np.array([cdist(xs[a:a + 1], xs[b:b + 1], SCIPY_METRIC[norm])[0, 0] for a, b in pairs])
    want = np.quantile(dists, probs, method="inverted_cdf")
    np.testing.assert_allclose(got, want, rtol=1e-14, atol=0)


@pytest.mark.parametrize("norm", NORMS)
def test_table_nearest_and_overall_entries(norm):
    """d1 is the 1-NN distance (cKDTree), V_0 the slope to it, V_{K+1} the
    largest slope over all pairs (cdist), and max_k V_{K+1} the global constant."""
    n, d = 400, 3
    x, y = _problem(3, n, d)
    kn = np.array([0.1, 0.3, 0.6])
    st, d1, V = oracle.local_steps(x, y, kn, norm)
    assert st == 0
    xs = x.astype(np.float64)
    dd, ii = cKDTree(xs).query(xs, k=3, p=KD_P[norm])
    np.testing.assert_allclose(d1, dd[:, 1], rtol=1e-13)
    uniq = dd[:, 2] > dd[:, 1] * (1 + 1e-9)
    slope_nn = np.abs(y[ii[:, 1]].astype(np.float64) - y) / dd[:, 1]
    np.testing.assert_allclose(V[uniq, 0], slope_nn[uniq], rtol=1e-12)
    D = cdist(xs, xs, SCIPY_METRIC[norm])
    np.fill_diagonal(D, np.inf)
    S = np.abs(y[:, None].astype(np.float64) - y[None, :]) / D
    np.testing.assert_allclose(V[:, -1], S.max(1), rtol=1e-12)
    for s in range(len(kn)):
        rad = np.maximum(kn[s], d1)
        want = np.where(D <= rad[:, None] * (1 + 1e-12), S, 0.0).max(1)
        np.testing.assert_allclose(V[:, s + 1], want, rtol=1e-12)
    stg, Mg, _ = oracle.estimate_M_global(x, y, norm)
    assert stg == 0 and V[:, -1].max() == Mg


@pytest.mark.parametrize("norm", NORMS)
def test_table_rows_are_non_decreasing(norm):
    x, y = _problem(4, 500, 4)
    kn = np.array([0.02, 0.2, 0.5, 0.8, 1.5])
    st, d1, V = oracle.local_steps(x, y, kn, norm)
    assert st == 0 and np.all(np.diff(V, axis=1) >= 0)
    # knots below the nearest distance collapse onto the first segment
    below = kn[None, :] <= d1[:, None]
    assert below.any()
    assert np.all(np.where(below, V[:, 1:-1] == V[:, :1], True))


@pytest.mark.parametrize("norm", NORMS)
@pytest.mark.parametrize("seed", [5, 6])
def test_step_bounds_interpolate_the_data(norm, seed):
    """The construction interpolates: g(x^k) = y^k at every datum (exactly in
    FP64, with the table rounded up to FP32), and H_lo <= H_up there."""
    x, y = _problem(seed, 600, 3, dyadic=(seed == 6))
    kn = oracle.knots(x, np.random.default_rng(seed).integers(0, 600, (2000, 2)),
                      [0.05, 0.2, 0.5], norm)
    st, d1, V = oracle.local_steps(x, y, kn, norm)
    assert st == 0
    hu, hl, g, au, al = oracle.bounds_step(x, y, x, norm, kn, d1, oracle.round_up_f32(V))
    np.testing.assert_array_equal(hu, y.astype(np.float64))
    np.testing.assert_array_equal(hl, y.astype(np.float64))
    np.testing.assert_array_equal(g, y.astype(np.float64))


def test_linear_data_reduce_to_global_bounds():
    """1-D linear data: every slope is |a|, so M_k(t) = |a| and the bounds
    equal those of the (separately pinned) global-constant form."""
    xs = np.arange(0, 40, dtype=np.float64)[np.random.default_rng(7).permutation(40)] / 8
    x = xs[:, None].astype(np.float32)
    y = (0.75 * xs - 1.0).astype(np.float32)
    xq = (np.linspace(-1, 6, 301)[:, None]).astype(np.float32)
    for norm in NORMS:
        st, d1, V = oracle.local_steps(x, y, [0.3, 1.0, 2.5], norm)
        assert st == 0 and np.all(V == 0.75)
        a = oracle.bounds_step(x, y, xq, norm, [0.3, 1.0, 2.5], d1, V.astype(np.float32),
                               mon=[1])
        b = oracle.bounds(x, y, xq, norm, M=0.75, mon=[1])
        for u, v in zip(a, b):
            np.testing.assert_array_equal(u, v)


def test_coincident_data():
    x = np.array([[0, 0], [1, 0], [0, 0], [3, 4]], np.float32)
    y = np.array([1, 2, 1, 0], np.float32)
    # the coincident pair (0, 2) has equal values: skipped
    st, d1, V = oracle.local_steps(x, y, [2.0], L2)
    assert st == 0
    # datum 3 = (3, 4) is nearest to (1, 0), at sqrt(20); datum 0 sees (1, 0)
    # at 1 (slope 1) and (3, 4) at 5 (slope 1/5)
    np.testing.assert_array_equal(d1, [1, 1, 1, np.sqrt(20.0)])
    np.testing.assert_array_equal(V[0], [1, 1, 1])
    # different values at coincident points: infinite slope, rows 0 and 2
    y2 = np.array([1, 2, 5, 0], np.float32)
    st, d1, V = oracle.local_steps(x, y2, [2.0], L2)
    assert st == 3 and np.all(np.isinf(V[[0, 2]])) and np.all(np.isfinite(V[[1, 3]]))


def test_single_datum_and_empty_knots():
    x = np.array([[0.5, 0.5]], np.float32)
    y = np.array([2.0], np.float32)
    st, d1, V = oracle.local_steps(x, y, [], L1)
    assert st == 0 and np.isinf(d1[0]) and V.shape == (1, 2) and np.all(V == 0)
    hu, hl, g, au, al = oracle.bounds_step(x, y, [[0.1, 0.9], [3, 3]], L1, [], d1,
                                           V.astype(np.float32))
    assert np.all(hu == 2) and np.all(hl == 2) and np.all(au == 0)
