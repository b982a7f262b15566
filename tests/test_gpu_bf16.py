"""BF16-MFMA l2 path (LIP_FLAG_BF16): identical results to the FP32 path.

The matrix cores only select candidate pairs; every candidate is re-scored
with the FP32 pair formula, so values and indices must equal the FP32 path's
bit for bit (compared with ==, so -0.0 and +0.0 count as equal), on every
query.  Sampled queries are also checked against the FP64 oracle.
"""
import numpy as np
import pytest
import torch

import workloads as W
from _parity import check_bounds

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
KEYS = ("g", "h_up", "h_lo", "arg_up", "arg_lo")


@pytest.fixture(scope="module")
def lf():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2606_04670_amd as lf
    lf.load()
    return lf


def _run(lf, p, bf16, Mk=None):
    Mk = p.Mk if Mk is None else Mk
    x = torch.from_numpy(np.ascontiguousarray(p.x)).to(DEV)
    y = torch.from_numpy(np.ascontiguousarray(p.y)).to(DEV)
    xq = torch.from_numpy(np.ascontiguousarray(p.xq)).to(DEV)
    mk = None if Mk is None else torch.from_numpy(np.asarray(Mk, np.float32)).to(DEV)
    met = lf.Metric(p.d, p.norm, mon=p.mon, w=p.w)
    out = lf.fit_eval(x, y, xq, met, M=None if mk is not None else p.M, Mk=mk, bf16=bf16)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _same(lf, p, label, Mk=None):
    ref = _run(lf, p, False, Mk=Mk)
    got = _run(lf, p, True, Mk=Mk)
    for k in KEYS:
        eq = got[k] == ref[k]
        if got[k].dtype.kind == "f":
            eq |= np.isnan(got[k]) & np.isnan(ref[k])
        bad = np.nonzero(~eq)[0]
        assert bad.size == 0, (f"{label}: {k} differs from the FP32 path at {bad.size} queries, "
                               f"first {bad[:5].tolist()}: bf16 {got[k][bad[:5]]} fp32 {ref[k][bad[:5]]}")
    return got


def test_mixed_l2_reduced(lf):
    """d = 16, x ~ N(0, I), y = |x|_1 / 16 + noise, M = 1 at N = 60,000,
    Q = 20,000: identical to FP32, oracle parity on 64 queries."""
    p = W.mixed_l2(n=60_000, q=20_000)
    got = _same(lf, p, "mixed_l2 reduced")
    qidx = np.linspace(0, p.q - 1, 64).astype(int)
    check_bounds(p, got, qidx=qidx, label="bf16 mixed_l2 reduced")


@pytest.mark.parametrize("d", [1, 2, 3, 5, 8, 10, 11, 13, 16])
@pytest.mark.parametrize("n,q", [(1, 5), (31, 63), (1000, 129), (4097, 777)])
def test_random_shapes(lf, d, n, q):
    """Ragged N (partial 32-datum tiles, a single datum), ragged Q (partial
    query blocks), one or two MFMA K-steps, split data chunks at small Q."""
    p = W.random_problem(7000 + 31 * d + n, n=n, q=q, d=d, norm=2, weighted=(d % 2 == 1))
    got = _same(lf, p, f"random d={d} n={n} q={q}")
    check_bounds(p, got, qidx=np.arange(min(q, 32)), label=f"bf16 d={d} n={n} q={q}")


@pytest.mark.parametrize("d", [3, 12])
def test_local_M(lf, d):
    """Per-datum M_k (the tile radius uses the smallest M_k of the tile)."""
    p = W.random_problem(7100 + d, n=5000, q=3000, d=d, norm=2, local=True)
    got = _same(lf, p, f"local M d={d}")
    check_bounds(p, got, qidx=np.arange(40), label=f"bf16 local d={d}")


def test_exact_ties(lf):
    """Integer lattice data and queries: many exactly equal distances and
    duplicated data points; the lowest index must win every tie.  y holds
    -0.0 and +0.0."""
    rng = np.random.default_rng(71)
    d = 4
    x = rng.integers(0, 3, (3000, d)).astype(np.float32)
    y = rng.integers(-2, 3, 3000).astype(np.float32)
    y[y == 0] = np.where(rng.random((y == 0).sum()) < 0.5, -0.0, 0.0).astype(np.float32)
    xq = rng.integers(0, 3, (2000, d)).astype(np.float32)
    p = W.Problem("lattice", x, y, 1.0, None, xq, 2, np.zeros(d, np.int8), np.ones(d, np.float32))
    _same(lf, p, "lattice ties")
    mk = np.where(rng.random(3000) < 0.3, 0.0, 1.0 + rng.integers(0, 3, 3000)).astype(np.float32)
    _same(lf, p, "lattice ties, M_k with zeros", Mk=mk)


def test_constant_data(lf):
    """Every datum identical: every pair ties, every pair is a candidate
    (exercises queue overflow and repeated drains)."""
    d = 6
    x = np.full((2500, d), 0.25, np.float32)
    y = np.full(2500, 0.5, np.float32)
    xq = np.random.default_rng(3).random((300, d)).astype(np.float32)
    p = W.Problem("constant", x, y, 2.0, None, xq, 2, np.zeros(d, np.int8), np.ones(d, np.float32))
    got = _same(lf, p, "constant data")
    assert (got["arg_up"] == 0).all() and (got["arg_lo"] == 0).all()


def test_zero_M(lf):
    """M = 0: H_up = min y, H_lo = max y, every pair a candidate."""
    p = W.random_problem(7200, n=3000, q=500, d=7, norm=2, M=0.0)
    _same(lf, p, "M = 0")


def test_huge_magnitudes(lf):
    """Norms above 2^100 (here |x| ~ 1e31) take the exact path per query /
    per tile; mixed with ordinary rows."""
    p = W.random_problem(7300, n=2000, q=400, d=5, norm=2)
    x = p.x.copy()
    x[::7] *= np.float32(1e31)
    xq = p.xq.copy()
    xq[::5] *= np.float32(1e31)
    p2 = W.Problem("huge", x, p.y, 1.5, None, xq, 2, p.mon, p.w)
    _same(lf, p2, "huge magnitudes")


def test_mixed_l2_full(lf):
    """d = 16, N = 1,000,000, Q = 1,000,000: identical to the FP32 path on
    every query; oracle parity on 16 sampled queries."""
    p = W.mixed_l2()
    got = _same(lf, p, "mixed_l2 full")
    qidx = np.random.default_rng(52).choice(p.q, 16, replace=False)
    check_bounds(p, got, qidx=np.sort(qidx), label="bf16 mixed_l2 full")
