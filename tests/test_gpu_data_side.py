"""GPU data-side passes against the FP64 oracle.

Both sides evaluate every pair in double precision with the same operation
order, so slacks, partners, violation counts, slopes and neighbour sets are
compared exactly (bit for bit).
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


def _consistency(lf, p, M, Mk, tol=0.0):
    met = lf.Metric(p.d, p.norm, mon=p.mon, w=p.w)
    r = lf.consistency(_t(p.x), _t(p.y), met, M=None if Mk is not None else M, Mk=_t(Mk), tol=tol)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in r.items()}


def _check_worst(g, o):
    """The smallest slack and its pair (lowest i, then k, on ties)."""
    assert g["worst_slack"][0] == o["worst_slack"], (g["worst_slack"], o["worst_slack"])
    assert tuple(g["worst_pair"].tolist()) == o["worst_pair"]


CASES = [
    (1, [0, 0, 0], False, False),
    (2, [1, 0, -1], True, True),
    (3, [1, 1, 0], False, True),
    (2, [0, 0, 0], False, False),
]


@pytest.mark.parametrize("norm,mon,local,weighted", CASES)
def test_consistency_exact(lf, norm, mon, local, weighted):
    for n, M in [(1, 1.0), (2, 0.5), (777, 1.5), (1031, 4.0)]:
        p = W.random_problem(400 + n, n=n, q=1, d=3, norm=norm, mon=np.array(mon, np.int8),
                             local=local, weighted=weighted)
        M32 = float(np.float32(M))
        g = _consistency(lf, p, M32, p.Mk)
        o = oracle.consistency(p.x, p.y, norm, M=M32, Mk=p.Mk, mon=p.mon, w=p.w)
        np.testing.assert_array_equal(g["slack_up"], o["slack_up"])
        np.testing.assert_array_equal(g["slack_lo"], o["slack_lo"])
        np.testing.assert_array_equal(g["partner_up"], o["partner_up"])
        np.testing.assert_array_equal(g["partner_lo"], o["partner_lo"])
        assert g["counts"][0] == o["viol_up"].sum() and g["counts"][1] == o["viol_lo"].sum()
        _check_worst(g, o)


def test_consistency_boundary_ties_and_tolerance(lf):
    """Dyadic 1-D data with slopes exactly M: consistent at M, violated just
    below it; a tolerance absorbs the violations."""
    x = (np.arange(64, dtype=np.float32) / 8.0)[:, None]
    y = (np.arange(64, dtype=np.float32) * 0.25).astype(np.float32)  # slope 2
    p = W.Problem("ties", x, y, 2.0, None, x, 1, np.zeros(1, np.int8), np.ones(1, np.float32))
    for norm in (1, 2, 3):
        p.norm = norm
        g = _consistency(lf, p, 2.0, None)
        assert g["counts"].tolist() == [0, 0]
        g = _consistency(lf, p, float(np.float32(1.999)), None)
        o = oracle.consistency(x, y, norm, M=float(np.float32(1.999)))
        assert g["counts"].tolist() == [o["viol_up"].sum(), o["viol_lo"].sum()] != [0, 0]
        g = _consistency(lf, p, float(np.float32(1.999)), None, tol=1.0)
        assert g["counts"].tolist() == [0, 0]


def test_consistency_monotone_local_workload_sampled_rows(lf):
    """d=4, N=100,000 with per-point M_k and monotone coordinates: every row
    on the GPU, a seeded sample of rows on the oracle, compared exactly; the
    totals against the oracle over all rows of a 6,000-point prefix."""
    p = W.monotone_local(q=1)
    g = _consistency(lf, p, 0.0, p.Mk)
    rows = np.sort(np.random.default_rng(9).choice(p.n, 300, replace=False))
    o = oracle.consistency(p.x, p.y, p.norm, Mk=p.Mk, mon=p.mon, rows=rows)
    for k in ("slack_up", "slack_lo", "partner_up", "partner_lo"):
        np.testing.assert_array_equal(g[k][rows], o[k])
    n2 = 6000
    p2 = W.Problem("prefix", p.x[:n2], p.y[:n2], 0.0, p.Mk[:n2], p.xq, p.norm, p.mon, p.w)
    g2 = _consistency(lf, p2, 0.0, p2.Mk)
    o2 = oracle.consistency(p2.x, p2.y, p.norm, Mk=p2.Mk, mon=p.mon)
    assert g2["counts"].tolist() == [o2["viol_up"].sum(), o2["viol_lo"].sum()]


@pytest.mark.parametrize("norm", [1, 2, 3])
def test_estimate_global_exact(lf, norm):
    for n in (2, 3, 500, 1337):
        p = W.random_problem(500 + n, n=n, q=1, d=4, norm=norm, weighted=(n % 2 == 1))
        met = lf.Metric(p.d, norm, w=p.w)
        M64, M32, pair = lf.estimate_M(_t(p.x), _t(p.y), met, mode="global")
        st, Mo, po = oracle.estimate_M_global(p.x, p.y, norm, w=p.w)
        assert st == 0
        assert M64.item() == Mo and tuple(pair.cpu().tolist()) == po
        f = np.float32(Mo)
        expect = f if float(f) >= Mo else np.nextafter(f, np.float32(np.inf))
        assert np.float32(M32.item()) == expect


def test_estimate_global_duplicates(lf):
    x = np.array([[0, 0], [1, 0], [0, 0], [1, 0], [3, 3]], np.float32)
    y = np.array([0, 1, 0, 1, 2], np.float32)
    met = lf.Metric(2, "l2")
    M64, M32, pair = lf.estimate_M(_t(x), _t(y), met)
    assert pair.cpu().tolist() == [0, 1] and M64.item() == 1.0
    y2 = np.array([0, 1, 0, 1.5, 2], np.float32)
    M64, M32, pair = lf.estimate_M(_t(x), _t(y2), met)
    assert np.isinf(M64.item()) and pair.cpu().tolist() == [1, 3]


@pytest.mark.parametrize("norm", [1, 2, 3])
@pytest.mark.parametrize("K", [1, 5, 16, 32])
def test_estimate_knn_exact(lf, norm, K):
    p = W.random_problem(600 + K, n=1111, q=1, d=3, norm=norm, weighted=True)
    met = lf.Metric(p.d, norm, w=p.w)
    M64, M32, _ = lf.estimate_M(_t(p.x), _t(p.y), met, mode="knn", knn=K)
    st, Mo, nb = oracle.estimate_M_knn(p.x, p.y, norm, K=K, w=p.w)
    np.testing.assert_array_equal(M64.cpu().numpy(), Mo)
    m32 = M32.cpu().numpy().astype(np.float64)
    assert np.all(m32 >= Mo)


def test_estimate_knn_small_n_and_ties(lf):
    x = np.array([[0.0], [1.0], [-1.0], [2.0]], np.float32)
    y = np.array([0.0, 1.0, 3.0, 0.0], np.float32)
    met = lf.Metric(1, "l1")
    for K in (1, 2, 3, 16):
        M64, _, _ = lf.estimate_M(_t(x), _t(y), met, mode="knn", knn=K)
        st, Mo, _ = oracle.estimate_M_knn(x, y, 1, K=K)
        np.testing.assert_array_equal(M64.cpu().numpy(), Mo)


@pytest.mark.parametrize("norm", [1, 2, 3])
def test_estimates_monotone_local_workload_sampled(lf, norm):
    """d=4, N=100,000: kNN-16 constants of sampled rows equal the oracle's;
    the global slope equals the oracle's slope at the GPU's pair and bounds
    every sampled row's slopes."""
    p = W.monotone_local(q=1, norm=norm)
    met = lf.Metric(4, norm)
    M64, M32, _ = lf.estimate_M(_t(p.x), _t(p.y), met, mode="knn", knn=16)
    rows = np.sort(np.random.default_rng(norm).choice(p.n, 48, replace=False))
    st, Mo, _ = oracle.estimate_M_knn(p.x, p.y, norm, K=16, rows=rows)
    np.testing.assert_array_equal(M64.cpu().numpy()[rows], Mo)
    G64, G32, pair = lf.estimate_M(_t(p.x), _t(p.y), met, mode="global")
    i, k = pair.cpu().tolist()
    assert 0 <= i < k < p.n
    sub = np.array([p.x[i], p.x[k]], np.float32)
    st, Mpair, _ = oracle.estimate_M_global(sub, np.array([p.y[i], p.y[k]], np.float32), norm)
    assert G64.item() == Mpair
    # every sampled row's slopes stay below the global maximum
    for r in rows[:8]:
        xs = np.concatenate([p.x[r:r + 1], p.x]).astype(np.float32)
        ys = np.concatenate([p.y[r:r + 1], p.y]).astype(np.float32)
        # pairs (0, k) only: restrict by evaluating the candidates of row r
        d = {1: np.abs(p.x.astype(np.float64) - p.x[r]).sum(1),
             2: np.sqrt(((p.x.astype(np.float64) - p.x[r]) ** 2).sum(1)),
             3: np.abs(p.x.astype(np.float64) - p.x[r]).max(1)}[norm]
        dy = np.abs(p.y.astype(np.float64) - p.y[r])
        msk = d > 0
        assert np.max(dy[msk] / d[msk]) <= G64.item() * (1 + 1e-12)


@pytest.mark.parametrize("norm", [1, 2, 3])
def test_estimate_knn_lattice_ties_chunked(lf, norm):
    """Integer lattice data (many exactly equal distances, duplicated points
    with equal and with different y) at N = 8,000: several column chunks and
    a spatial row order whose windows hold many ties.  Neighbour ranking by
    (distance, index) must match the oracle exactly."""
    rng = np.random.default_rng(81 + norm)
    x = rng.integers(0, 10, (8000, 3)).astype(np.float32)
    y = (x @ np.array([1.0, -2.0, 0.5], np.float32)).astype(np.float32)
    odd = rng.random(8000) < 0.02  # a few duplicates disagree: infinite slopes
    y[odd] += np.float32(0.25)
    met = lf.Metric(3, norm)
    M64, M32, _ = lf.estimate_M(_t(x), _t(y), met, mode="knn", knn=16)
    st, Mo, _ = oracle.estimate_M_knn(x, y, norm, K=16)
    np.testing.assert_array_equal(M64.cpu().numpy(), Mo)


def test_estimate_knn_high_dim_clustered(lf):
    """d = 16, clustered data (the spatial order is coarse at 2 bits per
    coordinate), weighted l2, K = 16 and K = 7."""
    rng = np.random.default_rng(83)
    centres = rng.standard_normal((12, 16))
    x = (centres[rng.integers(0, 12, 3000)] + 0.05 * rng.standard_normal((3000, 16))).astype(np.float32)
    y = rng.standard_normal(3000).astype(np.float32)
    w = (0.5 + rng.random(16)).astype(np.float32)
    met = lf.Metric(16, 2, w=w)
    for K in (16, 7):
        M64, _, _ = lf.estimate_M(_t(x), _t(y), met, mode="knn", knn=K)
        st, Mo, _ = oracle.estimate_M_knn(x, y, 2, K=K, w=w)
        np.testing.assert_array_equal(M64.cpu().numpy(), Mo)


def _patterns(d):
    import itertools
    return [np.array(m, np.int8) for m in itertools.product((-1, 0, 1), repeat=d)]


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_consistency_every_pattern_low_dim(lf, d):
    """Up to d = 4 every free / increasing / decreasing pattern has its own
    kernel; each must reproduce the oracle exactly (all patterns for d <= 3,
    a seeded third of them for d = 4), norms and weights varied."""
    pats = _patterns(d)
    if d == 4:
        rng = np.random.default_rng(4)
        pats = [pats[i] for i in sorted(rng.choice(len(pats), 27, replace=False))]
    for k, mon in enumerate(pats):
        norm = 1 + k % 3
        p = W.random_problem(900 + 10 * d + k, n=333 + 17 * k, q=1, d=d, norm=norm, mon=mon,
                             local=(k % 2 == 0), weighted=(k % 4 == 1))
        g = _consistency(lf, p, 1.25, p.Mk)
        o = oracle.consistency(p.x, p.y, norm, M=1.25, Mk=p.Mk, mon=p.mon, w=p.w)
        for key in ("slack_up", "slack_lo", "partner_up", "partner_lo"):
            np.testing.assert_array_equal(g[key], o[key], err_msg=f"d={d} mon={mon.tolist()} {key}")
        assert g["counts"].tolist() == [o["viol_up"].sum(), o["viol_lo"].sum()], mon.tolist()
        _check_worst(g, o)


def test_consistency_l2_filter_off_for_huge_values(lf):
    """Coordinates ~1e30 make the FP32 slack bound infinite (FP32 squares
    overflow): every pair goes to FP64, results still exact."""
    p = W.random_problem(990, n=700, q=1, d=3, norm=2, mon=np.array([1, 0, 0], np.int8))
    x = p.x.copy()
    x[::3] *= np.float32(1e30)
    p2 = W.Problem("huge", x, p.y, 1.5, None, p.xq, 2, p.mon, p.w)
    g = _consistency(lf, p2, 1.5, None)
    o = oracle.consistency(x, p.y, 2, M=1.5, mon=p.mon)
    for key in ("slack_up", "slack_lo", "partner_up", "partner_lo"):
        np.testing.assert_array_equal(g[key], o[key])
    assert g["counts"].tolist() == [o["viol_up"].sum(), o["viol_lo"].sum()]


@pytest.mark.parametrize("tol", [0.0, 1e-3, 0.25])
def test_consistency_l2_tolerance_band(lf, tol):
    """Slacks spread around -tol (data with a scaled-down M): the FP32
    filter's ambiguous band around the tolerance is decided in FP64."""
    p = W.random_problem(995, n=3000, q=1, d=4, norm=2, mon=np.array([1, 0, -1, 0], np.int8),
                         local=True)
    mk = (p.Mk * np.float32(0.2)).astype(np.float32)
    g = _consistency(lf, p, 0.0, mk, tol=tol)
    o = oracle.consistency(p.x, p.y, 2, Mk=mk, mon=p.mon, tol=tol)
    for key in ("slack_up", "slack_lo", "partner_up", "partner_lo"):
        np.testing.assert_array_equal(g[key], o[key])
    assert g["counts"].tolist() == [o["viol_up"].sum(), o["viol_lo"].sum()]


def test_consistency_l2_tiny_values(lf):
    """Coordinates ~1e-25: FP32 squares of the differences underflow; the
    absolute part of the filter's bound keeps every decision exact."""
    p = W.random_problem(996, n=900, q=1, d=3, norm=2, mon=np.array([0, 1, 0], np.int8))
    x = (p.x * np.float32(1e-25)).astype(np.float32)
    y = (p.y * np.float32(1e-24)).astype(np.float32)
    p2 = W.Problem("tiny", x, y, 1.5, None, p.xq, 2, p.mon, p.w)
    g = _consistency(lf, p2, 1.5, None)
    o = oracle.consistency(x, y, 2, M=1.5, mon=p.mon)
    for key in ("slack_up", "slack_lo", "partner_up", "partner_lo"):
        np.testing.assert_array_equal(g[key], o[key])
    assert g["counts"].tolist() == [o["viol_up"].sum(), o["viol_lo"].sum()]


@pytest.mark.parametrize("d", [5, 8, 12, 16])
@pytest.mark.parametrize("norm", [1, 2, 3])
def test_consistency_exact_higher_dims(lf, d, norm):
    """Dimensions above 4 (the l2 filter kernel holds fewer rows per lane
    there): slacks, partners and counts bit-exact, with and without monotone
    coordinates, per-datum constants and weights, ragged n over several
    column chunks."""
    for k, n in enumerate((130, 1537)):
        mon = np.zeros(d, np.int8) if k == 0 else np.array([1, 0, -1] * 6, np.int8)[:d]
        p = W.random_problem(900 + d + n, n=n, q=1, d=d, norm=norm, mon=mon,
                             local=(k == 1), weighted=(d % 2 == 0))
        M32 = float(np.float32(1.2))
        g = _consistency(lf, p, M32, p.Mk)
        o = oracle.consistency(p.x, p.y, norm, M=M32, Mk=p.Mk, mon=p.mon, w=p.w)
        for key in ("slack_up", "slack_lo", "partner_up", "partner_lo"):
            np.testing.assert_array_equal(g[key], o[key], err_msg=f"d={d} n={n} {key}")
        assert g["counts"].tolist() == [o["viol_up"].sum(), o["viol_lo"].sum()]
        _check_worst(g, o)


def test_consistency_worst_pair_ties_and_tiny_sets(lf):
    """Equal slacks on several rows (dyadic 1-D data, slope exactly above M
    everywhere): the worst pair is the lowest (i, k); n = 1 has none."""
    x = (np.arange(40, dtype=np.float32) / 4.0)[:, None]
    y = (np.arange(40, dtype=np.float32) * 0.75).astype(np.float32)  # slope 3
    p = W.Problem("ties", x, y, 2.0, None, x, 1, np.zeros(1, np.int8), np.ones(1, np.float32))
    for norm in (1, 2, 3):
        p.norm = norm
        g = _consistency(lf, p, 2.0, None)
        o = oracle.consistency(x, y, norm, M=2.0)
        _check_worst(g, o)
    one = W.random_problem(5, n=1, q=1, d=2, norm=2)
    g = _consistency(lf, one, 1.0, None)
    assert np.isinf(g["worst_slack"][0]) and g["worst_pair"].tolist() == [-1, -1]
    # the binding without per-row outputs still reports the worst pair
    p3 = W.random_problem(6, n=2500, q=1, d=4, norm=3, mon=np.array([1, 0, 0, -1], np.int8),
                          local=True)
    met = lf.Metric(4, 3, mon=p3.mon)
    r = lf.consistency(_t(p3.x), _t(p3.y), met, Mk=_t(p3.Mk), per_row=False)
    o = oracle.consistency(p3.x, p3.y, 3, Mk=p3.Mk, mon=p3.mon)
    _check_worst({k: v.cpu().numpy() for k, v in r.items()}, o)


@pytest.mark.slow
def test_consistency_mixed_l2_200k(lf):
    """The FP64 consistency check of the mixed-precision workload's first
    200,000 points (d = 16, l2, M = 1): 256 seeded rows and every row the GPU
    flags, bit-exact; the worst pair's row reproduced by the oracle.  Again
    with M = 0.02, where most rows violate: 512 of the flagged rows."""
    full = W.mixed_l2(q=1)
    n = 200_000
    p = W.Problem("mixed_l2 200k", full.x[:n].copy(), full.y[:n].copy(), 1.0, None, full.xq, 2,
                  full.mon, full.w)
    rng = np.random.default_rng(200)
    for M in (1.0, float(np.float32(0.02))):  # the FP32 constant both sides read
        g = _consistency(lf, p, M, None)
        flagged = np.nonzero((g["slack_up"] < 0) | (g["slack_lo"] < 0))[0]
        if flagged.size > 512:
            flagged = np.sort(rng.choice(flagged, 512, replace=False))
        rows = np.unique(np.concatenate([rng.choice(n, 256, replace=False), flagged,
                                         [int(g["worst_pair"][0])]]))
        o = oracle.consistency(p.x, p.y, 2, M=M, rows=rows)
        for key in ("slack_up", "slack_lo", "partner_up", "partner_lo"):
            np.testing.assert_array_equal(g[key][rows], o[key], err_msg=f"M={M} {key}")
        # the per-row violation counts of the sampled rows add up below the totals
        assert o["viol_up"].sum() <= g["counts"][0] and o["viol_lo"].sum() <= g["counts"][1]
        w = g["worst_slack"][0]
        assert w == min(g["slack_up"].min(), g["slack_lo"].min())
        i, k = (int(v) for v in g["worst_pair"])
        r = int(np.nonzero(rows == i)[0][0])
        assert (o["slack_up"][r] == w and o["partner_up"][r] == k) or \
            (o["slack_lo"][r] == w and o["partner_lo"][r] == k)
        if M == 1.0:
            print(f"M=1: violations {g['counts'].tolist()}, worst slack {w:.6g} at {(i, k)}")


@pytest.mark.slow
@pytest.mark.parametrize("norm", [1, 2, 3])
def test_estimate_global_monotone_local_full(lf, norm):
    """The global constant of the d = 4, N = 100,000 data over all 5e9
    pairs, against the oracle's full brute force: M64 and the pair exact."""
    p = W.monotone_local(q=1, norm=norm)
    met = lf.Metric(4, norm)
    G64, G32, pair = lf.estimate_M(_t(p.x), _t(p.y), met, mode="global")
    st, Mo, po = oracle.estimate_M_global(p.x, p.y, norm)
    assert st == 0
    assert G64.item() == Mo and tuple(pair.cpu().tolist()) == po, (G64.item(), Mo, pair, po)


def test_estimate_infinite_slope_status(lf):
    """Coincident data with different values: +inf through the outputs, and
    LIP_E_VALUE when the synchronous checks are asked for."""
    from paper_2606_04670_amd import LipError
    x = np.array([[0, 0], [1, 0], [0, 0], [3, 3]], np.float32)
    y = np.array([0, 1, 0.5, 2], np.float32)
    met = lf.Metric(2, "l2")
    for mode in ("global", "knn"):
        M64, _, _ = lf.estimate_M(_t(x), _t(y), met, mode=mode, knn=2)
        torch.cuda.synchronize()
        assert np.isinf(M64.cpu().numpy()).any()
        with pytest.raises(LipError) as e:
            lf.estimate_M(_t(x), _t(y), met, mode=mode, knn=2, check_finite=True)
        assert e.value.status == 3  # LIP_E_VALUE
    y2 = np.array([0, 1, 0, 2], np.float32)
    M64, _, _ = lf.estimate_M(_t(x), _t(y2), met, check_finite=True)
    assert np.isfinite(M64.item())
