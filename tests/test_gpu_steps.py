"""GPU parity of the step-function local constants of Sec. 4.3 against the oracle.

Knots and tables are FP64 with the operation order of the definition, so they
must equal the oracle's bit for bit; the bounds are FP32 and follow the
comparison rules of tests/_parity.py (the segment of every pair is decided
in FP64 on both sides, so the two evaluate the same step of M_k).
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from _parity import check_bounds_steps

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
NORMS = [1, 2, 3]


@pytest.fixture(scope="module")
def lf():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2606_04670_amd as lf
    lf.load()
    return lf


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _metric(lf, p, use_mon=True):
    return lf.Metric(p.d, p.norm, mon=p.mon if use_mon else None, w=p.w)


@pytest.mark.parametrize("norm", NORMS)
@pytest.mark.parametrize("m", [1000, 4097])
@pytest.mark.parametrize("weighted", [False, True])
def test_knots_bit_exact(lf, norm, m, weighted):
    p = W.random_problem(10 + m, n=900, q=1, d=5, norm=norm, weighted=weighted)
    pairs = W.rng_for(200, m).integers(0, p.n, size=(m, 2))
    probs = np.array([1 / m, 0.1, 0.25, 0.5, 0.5, 0.75, 0.999, 1.0])
    got = lf.local_knots(_t(p.x), _metric(lf, p), pairs, probs).cpu().numpy()
    want = oracle.knots(p.x, pairs, probs, norm, w=p.w)
    np.testing.assert_array_equal(got, want)


TABLE_CASES = [
    # (n, d, K, weighted)
    (1, 3, 4, False),
    (2, 1, 2, False),
    (777, 1, 3, True),
    (1500, 2, 8, False),
    (1500, 4, 4, False),
    (1300, 4, 5, True),
    (999, 7, 1, False),
    (640, 16, 0, True),
]


@pytest.mark.parametrize("norm", NORMS)
@pytest.mark.parametrize("n,d,K,weighted", TABLE_CASES)
def test_table_bit_exact(lf, norm, n, d, K, weighted):
    p = W.random_problem(300 + n + d, n=n, q=1, d=d, norm=norm, weighted=weighted)
    pairs = W.rng_for(201, n).integers(0, n, size=(2000, 2))
    probs = np.arange(1, K + 1) / (K + 1)
    kn = oracle.knots(p.x, pairs, probs, norm, w=p.w)
    d1, V64, V32 = lf.local_steps(_t(p.x), _t(p.y), _metric(lf, p), kn)
    st, d1o, Vo = oracle.local_steps(p.x, p.y, kn, norm, w=p.w)
    assert st == 0
    np.testing.assert_array_equal(d1.cpu().numpy(), d1o)
    np.testing.assert_array_equal(V64.cpu().numpy(), Vo)
    np.testing.assert_array_equal(V32.cpu().numpy(), oracle.round_up_f32(Vo))


@pytest.mark.parametrize("norm", NORMS)
def test_table_coincident_data(lf, norm):
    g = W.rng_for(202, norm)
    x = g.random((300, 3)).astype(np.float32)
    y = g.random(300).astype(np.float32)
    x[17] = x[5]          # equal values: skipped
    y[17] = y[5]
    x[250] = x[40]        # different values: infinite slope
    y[250] = y[40] + 1.0
    kn = np.array([0.1, 0.4])
    met = lf.Metric(3, norm)
    d1, V64, V32 = lf.local_steps(_t(x), _t(y), met, kn)
    st, d1o, Vo = oracle.local_steps(x, y, kn, norm)
    assert st == 3
    np.testing.assert_array_equal(d1.cpu().numpy(), d1o)
    np.testing.assert_array_equal(V64.cpu().numpy(), Vo)
    assert np.all(np.isinf(V64.cpu().numpy()[[40, 250]]))


FWD_CASES = [
    # (seed, n, q, d, mon, K, weighted)
    (1, 1000, 700, 2, [0, 0], 4, False),
    (2, 1537, 300, 4, [1, 0, 1, 0], 4, False),
    (3, 1200, 2100, 4, [0, -1, 0, 1], 7, True),
    (4, 900, 64, 3, [1, 1, 1], 2, False),
    (5, 2049, 129, 8, [1, 0, 1, 0, 1, 0, 1, 0], 8, False),
    (6, 513, 1000, 16, [0, 1] * 8, 3, True),
    (7, 1, 50, 3, [0, 0, 0], 4, False),
    (8, 700, 333, 1, [1], 0, False),
]


@pytest.mark.parametrize("norm", NORMS)
@pytest.mark.parametrize("seed,n,q,d,mon,K,weighted", FWD_CASES)
def test_fit_eval_steps_parity(lf, norm, seed, n, q, d, mon, K, weighted):
    p = W.random_problem(400 + seed, n=n, q=q, d=d, norm=norm, mon=np.array(mon, np.int8),
                         weighted=weighted)
    pairs = W.rng_for(203, seed).integers(0, n, size=(3000, 2))
    kn = oracle.knots(p.x, pairs, np.arange(1, K + 1) / (K + 1), norm, w=p.w)
    st, d1o, Vo = oracle.local_steps(p.x, p.y, kn, norm, w=p.w)
    V32 = oracle.round_up_f32(Vo)
    out = lf.fit_eval_steps(_t(p.x), _t(p.y), _t(p.xq), _metric(lf, p), kn, _t(d1o), _t(V32))
    torch.cuda.synchronize()
    gpu = {k: v.cpu().numpy() for k, v in out.items()}
    rep = check_bounds_steps(p, gpu, kn, d1o, V32, label=f"steps n={n} q={q} d={d}")
    print(rep)


@pytest.mark.parametrize("norm", NORMS)
def test_queries_at_the_data_interpolate(lf, norm):
    """Sec. 4.3: with the symmetric distance the step construction
    interpolates, g(x^k) = y^k (here to FP32 rounding)."""
    p = W.random_problem(500 + norm, n=2500, q=1, d=3, norm=norm)
    model = lf.StepModel(_t(p.x), _t(p.y), lf.Metric(3, norm), K=4, m=5000, seed=norm)
    out = model(_t(p.x))
    g = out["g"].cpu().numpy().astype(np.float64)
    assert np.max(np.abs(g - p.y)) <= 1e-5 * np.abs(p.y).max()
    # the model's knots are the oracle's for the same sampled pairs
    np.testing.assert_array_equal(
        model.knots, oracle.knots(p.x, model.pairs, model.probs, norm))


@pytest.mark.parametrize("norm", NORMS)
def test_monotone_local_full_size_sampled(lf, norm):
    """d=4, N=1e5 (the monotone local workload): the table on sampled rows
    bit for bit, the bounds of Q=1e6 queries on sampled queries."""
    p = W.monotone_local(norm=norm)
    x, y, xq = _t(p.x), _t(p.y), _t(p.xq)
    met_sym = lf.Metric(4, norm)
    pairs = W.rng_for(204, norm).integers(0, p.n, size=(65536, 2))
    probs = np.arange(1, 5) / 5
    kn = lf.local_knots(x, met_sym, pairs, probs).cpu().numpy()
    np.testing.assert_array_equal(kn, oracle.knots(p.x, pairs, probs, norm))
    d1, V64, V32 = lf.local_steps(x, y, met_sym, kn)
    rows = W.rng_for(205, norm).choice(p.n, size=96, replace=False)
    st, d1o, Vo = oracle.local_steps(p.x, p.y, kn, norm, rows=rows)
    np.testing.assert_array_equal(d1.cpu().numpy()[rows], d1o)
    np.testing.assert_array_equal(V64.cpu().numpy()[rows], Vo)
    out = lf.fit_eval_steps(x, y, xq, _metric(lf, p), kn, d1, V32)
    torch.cuda.synchronize()
    gpu = {k: v.cpu().numpy() for k, v in out.items()}
    qidx = W.rng_for(206, norm).choice(p.q, size=128, replace=False)
    rep = check_bounds_steps(p, gpu, kn, d1.cpu().numpy(), V32.cpu().numpy(), qidx=qidx,
                             label=f"monotone_local steps {norm}")
    print(rep)
