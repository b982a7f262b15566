"""GPU parity of the fused bound kernel (lip_fit_eval) against the FP64 oracle.

Sizes span several argmin tiles with ragged tails; full-size workloads are
checked on sampled queries.  Comparison rules are in tests/_parity.py.
"""
import numpy as np
import pytest
import torch

import workloads as W
from _parity import check_bounds

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lf():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2606_04670_amd as lf
    lf.load()
    return lf


DEV = torch.device("cuda:0")


def run(lf, p, want=("g", "h_up", "h_lo", "arg_up", "arg_lo"), Mk=None, **kw):
    Mk = p.Mk if Mk is None else Mk
    x = torch.from_numpy(p.x).to(DEV)
    y = torch.from_numpy(p.y).to(DEV)
    xq = torch.from_numpy(p.xq).to(DEV)
    mk = None if Mk is None else torch.from_numpy(np.asarray(Mk, np.float32)).to(DEV)
    met = lf.Metric(p.d, p.norm, mon=p.mon, w=p.w)
    out = lf.fit_eval(x, y, xq, met, M=None if mk is not None else p.M, Mk=mk, want=want, **kw)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def test_plain_l2_workload_full(lf):
    """d=2, N=1,000, Q=10,000, l2, M=4: every query against the oracle."""
    p = W.plain_l2()
    rep = check_bounds(p, run(lf, p), label="plain_l2")
    print(rep)


MON_PATTERNS = {
    1: [[0], [1], [-1]],
    2: [[0, 0], [1, 0], [-1, 1]],
    3: [[0, 0, 0], [1, 0, -1], [1, 1, 1]],
    4: [[0, 0, 0, 0], [1, 0, 1, 0], [0, -1, 0, 1]],
    5: [[0] * 5, [1, 0, 0, -1, 0]],
    7: [[0] * 7, [1, -1, 0, 0, 1, 0, 0]],
    8: [[0] * 8, [1, 0, 1, 0, 1, 0, 1, 0]],
    12: [[0] * 12, [1] * 6 + [0] * 6],
    16: [[0] * 16, [0, 1] * 8],
}


@pytest.mark.parametrize("norm", [1, 2, 3])
@pytest.mark.parametrize("d", sorted(MON_PATTERNS))
def test_random_problems(lf, norm, d):
    """Every norm x dimension x monotone pattern, global and per-point M,
    weighted distances; n = 1,337 (ragged tail), q = 777."""
    for k, mon in enumerate(MON_PATTERNS[d]):
        for local in (False, True):
            p = W.random_problem(1000 * d + 10 * k + local, n=1337, q=777, d=d, norm=norm,
                                 mon=np.array(mon, np.int8), local=local, weighted=(k % 2 == 1))
            check_bounds(p, run(lf, p), label=f"d={d} norm={norm} mon={mon} local={local}")


@pytest.mark.parametrize("n,q", [(1, 5), (2, 1), (7, 64), (9, 65), (300, 129), (4097, 3)])
def test_small_and_ragged_sizes(lf, n, q):
    for norm in (1, 2, 3):
        p = W.random_problem(7 + n + q, n=n, q=q, d=3, norm=norm, mon=np.array([1, 0, 0], np.int8),
                             local=True)
        check_bounds(p, run(lf, p), label=f"n={n} q={q} norm={norm}")


def test_zero_queries_is_noop(lf):
    p = W.random_problem(3, n=10, q=0, d=2, norm=2)
    out = run(lf, p)
    assert all(v.size == 0 for v in out.values())


def test_ties_resolve_to_lowest_index(lf):
    """M = 0: every candidate is y_k, so the argmin / argmax are the first
    occurrences of min y / max y; duplicated data points tie exactly."""
    g = np.random.default_rng(5)
    n = 2000
    x = g.random((n, 3)).astype(np.float32)
    y = np.round(g.random(n) * 4).astype(np.float32)  # values in {0..4}: many ties
    xq = g.random((500, 3)).astype(np.float32)
    p = W.Problem("ties", x, y, 0.0, None, xq, 2, np.zeros(3, np.int8), np.ones(3, np.float32))
    out = run(lf, p)
    assert np.all(out["arg_up"] == np.argmin(y)) and np.all(out["arg_lo"] == np.argmax(y))
    assert np.all(out["h_up"] == y.min()) and np.all(out["h_lo"] == y.max())
    # duplicated points: copies 0..n-1 then again; the first copy must win
    x2 = np.concatenate([x, x]).astype(np.float32)
    y2 = np.concatenate([y, y]).astype(np.float32)
    p2 = W.Problem("dups", x2, y2, 1.5, None, xq, 2, np.zeros(3, np.int8), np.ones(3, np.float32))
    o2 = run(lf, p2)
    assert np.all(o2["arg_up"] < n) and np.all(o2["arg_lo"] < n)
    o1 = run(lf, W.Problem("single", x, y, 1.5, None, xq, 2, np.zeros(3, np.int8),
                           np.ones(3, np.float32)))
    for k in o1:
        np.testing.assert_array_equal(o1[k], o2[k])


@pytest.mark.parametrize("norm", [1, 2, 3])
def test_tiling_and_split_do_not_change_results(lf, norm):
    """Tile size, data split and waves per workgroup are performance knobs:
    outputs must be bitwise identical across them (deterministic forward)."""
    p = W.random_problem(11, n=5000, q=3000, d=4, norm=norm, mon=np.array([1, 0, 1, 0], np.int8),
                         local=True)
    ref = None
    try:
        # flags: 1 = l2 filter, 2 = queries in Morton order.  A workgroup's
        # waves merge consecutive chunks:
        # with 8 waves and split 5 it runs 5 waves, split 64 with 8 waves
        # leaves 8 partials, 3 waves of split 64 leave 22 (the last group
        # partly empty)
        for tile, split, waves, fl in [(64, 1, 4, 0), (8, 1, 1, 1), (256, 3, 2, 0), (32, 16, 4, 1),
                                       (128, 64, 3, 1), (32, 8, 8, 0), (16, 5, 8, 1),
                                       (8, 64, 8, 0), (32, 3, 2, 1), (128, 1, 8, 0),
                                       (64, 16, 1, 0), (32, 8, 4, 3), (16, 1, 4, 2),
                                       (64, 64, 8, 3)]:
            lf.tune_set(4, 2, norm, tile=tile, split=split, waves=waves, flags=fl)
            out = run(lf, p)
            if ref is None:
                ref = out
                check_bounds(p, out, label=f"norm={norm}")
            else:
                for k in ref:
                    np.testing.assert_array_equal(out[k], ref[k], err_msg=f"{k} {tile} {split}")
    finally:
        lf.tune_set(4, 2, norm, clear=True)
    out2 = run(lf, p)
    for k in ref:
        np.testing.assert_array_equal(out2[k], ref[k])


@pytest.mark.parametrize("norm", [1, 2, 3])
@pytest.mark.parametrize("d", [1, 2, 5, 7, 8, 9, 11, 15, 16])
def test_chunk_merge_identical(lf, norm, d):
    """Chunks merged in a workgroup (LDS keys, d <= 8), per-chunk partials
    through the combine kernel and both together give the same values and
    indices, including ties across chunks: the data are 40 points repeated,
    so every candidate value occurs in every chunk and the lowest index must
    win (at d >= 9 the waves take different queries instead)."""
    g = W.rng_for(1900, d, norm)
    mon = np.zeros(d, np.int8)
    mon[::2] = 1
    base = g.random((40, d)).astype(np.float32)
    x = np.tile(base, (125, 1))
    y = np.tile(g.standard_normal(40).astype(np.float32), 125)
    xq = g.random((1700, d)).astype(np.float32)
    xq[::9] = base[g.integers(0, 40, len(xq[::9]))]          # queries on data points
    p = W.Problem("repeated", x, y, 1.25, None, xq, norm, mon, np.ones(d, np.float32))
    dm = int(mon.sum())
    outs = []
    try:
        for tile, split, waves in [(8, 16, 1), (8, 16, 8), (16, 12, 4), (8, 40, 8), (8, 1, 4)]:
            lf.tune_set(d, dm, norm, tile=tile, split=split, waves=waves)
            outs.append(run(lf, p))
    finally:
        lf.tune_set(d, dm, norm, clear=True)
    for o in outs[1:]:
        for k in o:
            np.testing.assert_array_equal(o[k], outs[0][k], err_msg=k)
    assert outs[0]["arg_up"].max() < 40 and outs[0]["arg_lo"].max() < 40
    check_bounds(p, outs[1], label=f"chunks d={d} norm={norm}")


@pytest.mark.parametrize("norm", [1, 2, 3])
def test_monotone_local_workload_full_size_sampled(lf, norm):
    """d=4, N=100,000, Q=1,000,000, coordinates 1 and 3 increasing, per-point
    M_k: the GPU evaluates every query, the oracle a seeded sample of 512."""
    p = W.monotone_local(norm=norm)
    out = run(lf, p)
    qidx = np.sort(np.random.default_rng(norm).choice(p.q, 512, replace=False))
    qidx = np.concatenate([[0, p.q - 1], qidx])
    rep = check_bounds(p, out, qidx=qidx, label=f"monotone_local norm={norm}")
    print(rep)
    # determinism at full size
    out2 = run(lf, p)
    for k in out:
        np.testing.assert_array_equal(out[k], out2[k])


def test_diff_l2_workload_full_size_sampled(lf):
    p = W.diff_l2()
    out = run(lf, p)
    qidx = np.sort(np.random.default_rng(3).choice(p.q, 256, replace=False))
    print(check_bounds(p, out, qidx=qidx, label="diff_l2"))


def test_mixed_l2_workload_full_size_sampled(lf):
    """d=16, N=1,000,000, Q=1,000,000 (FP32 VALU path)."""
    p = W.mixed_l2()
    out = run(lf, p)
    qidx = np.sort(np.random.default_rng(5).choice(p.q, 64, replace=False))
    print(check_bounds(p, out, qidx=qidx, label="mixed_l2"))


def test_two_streams_keep_separate_scratch(lf):
    """Calls on two streams at once (each with its own workspace) give the
    same results as one after the other."""
    pa = W.random_problem(41, n=20000, q=30000, d=4, norm=1, mon=np.array([1, 0, 1, 0], np.int8),
                          local=True)
    pb = W.random_problem(42, n=15000, q=25000, d=3, norm=2, weighted=True)
    ref = [run(lf, pa), run(lf, pb)]
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    args = []
    for p in (pa, pb):
        args.append((t(p.x), t(p.y), t(p.xq), lf.Metric(p.d, p.norm, mon=p.mon, w=p.w),
                     None if p.Mk is None else t(p.Mk), p.M))
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(DEV), torch.cuda.Stream(DEV)]
    outs = [None, None]
    for rep in range(3):
        for i, (s, (x, y, xq, met, mk, M)) in enumerate(zip(streams, args)):
            with torch.cuda.stream(s):
                outs[i] = lf.fit_eval(x, y, xq, met, M=None if mk is not None else M, Mk=mk)
        torch.cuda.synchronize()
        for i in range(2):
            for k in ref[i]:
                np.testing.assert_array_equal(outs[i][k].cpu().numpy(), ref[i][k],
                                              err_msg=f"stream {i} {k} rep {rep}")


FILTER_CASES = [
    # (d, monotone pattern, local, weighted)
    (1, [1], False, False),
    (2, [0, -1], True, False),
    (3, [1, 0, 1], False, True),
    (4, [1, 0, 1, 0], True, False),
    (4, [-1, -1, 1, 1], False, True),
    (5, [0, 1, 0, 0, 1], True, True),
    (8, [1, 0] * 4, False, False),
    (12, [0, 0, 1] * 4, True, True),
    (16, [1] * 16, False, False),
    # no monotone coordinate: the flag is accepted and changes nothing
    (2, [0, 0], True, True),
    (8, [0] * 8, False, False),
]


def _with_cfg(lf, p, d, dm, fl, **kw):
    try:
        lf.tune_set(d, dm, 2, tile=32, split=4, waves=4, flags=fl)
        return run(lf, p, **kw)
    finally:
        lf.tune_set(d, dm, 2, clear=True)


@pytest.mark.parametrize("d,mon,local,weighted", FILTER_CASES)
def test_l2_filter_identical(lf, d, mon, local, weighted):
    """The root-free l2 filter (LIP_TILE_L2_FILTER) changes no output: every
    value and index equal to the unfiltered kernel's, on random data, data
    translated by 2^10, and queries placed on data points (distance 0); the
    oracle checks the filtered results."""
    mon = np.array(mon, np.int8)
    dm = int(np.count_nonzero(mon))
    p = W.random_problem(1700 + d, n=3001, q=2500, d=d, norm=2, mon=mon, local=local,
                         weighted=weighted)
    xq = p.xq.copy()
    xq[::7] = p.x[: len(xq[::7])]            # some queries on data points
    p = W.Problem(p.name, p.x, p.y, p.M, p.Mk, xq, 2, mon, p.w)
    for shift in (0.0, 2.0 ** 10):
        ps = W.Problem(p.name, (p.x.astype(np.float64) + shift).astype(np.float32), p.y, p.M,
                       p.Mk, (p.xq.astype(np.float64) + shift).astype(np.float32), 2, mon, p.w)
        off = _with_cfg(lf, ps, d, dm, 0)
        on = _with_cfg(lf, ps, d, dm, 1)
        ordered = _with_cfg(lf, ps, d, dm, 3)
        for k in off:
            np.testing.assert_array_equal(on[k], off[k], err_msg=f"{k} shift={shift}")
            np.testing.assert_array_equal(ordered[k], off[k], err_msg=f"{k} ordered shift={shift}")
        check_bounds(ps, on, label=f"filtered d={d} shift={shift}")


def test_l2_filter_tiny_differences(lf):
    """Components far below 2^-60 (coordinates ~1e-30, queries a few ulp away
    from data) with values near 0, the case the filter's absolute margin
    covers: identical to the unfiltered kernel."""
    g = np.random.default_rng(1801)
    n, d = 2000, 3
    x = (g.random((n, d)) * 1e-30).astype(np.float32)
    y = (g.standard_normal(n) * 1e-38).astype(np.float32)
    xq = x[g.integers(0, n, 1500)].copy()
    xq.view(np.int32)[:] += g.integers(-3, 4, xq.shape).astype(np.int32)  # a few ulp away
    mon = np.array([1, 0, -1], np.int8)
    p = W.Problem("tiny", x, y, 1e8, None, xq, 2, mon, np.ones(d, np.float32))
    off = _with_cfg(lf, p, d, 2, 0)
    on = _with_cfg(lf, p, d, 2, 1)
    for k in off:
        np.testing.assert_array_equal(on[k], off[k], err_msg=k)
