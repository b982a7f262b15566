"""Batched plans (lip_plan_*): one graph launch for many independent fits.

Results must be bitwise identical to per-set lip_fit_eval calls (same wave
body, deterministic merges) and agree with the FP64 oracle on sampled
queries; repeated executions are identical.
"""
import numpy as np
import pytest
import torch

import workloads as W
from _parity import check_bounds

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


def _sets_from(problems, lf):
    sets = []
    for p in problems:
        s = dict(x=_t(p.x), y=_t(p.y), xq=_t(p.xq), metric=lf.Metric(p.d, p.norm, mon=p.mon, w=p.w))
        if p.Mk is not None:
            s["Mk"] = _t(p.Mk)
        else:
            s["M"] = p.M
        sets.append(s)
    return sets


def _per_set(lf, sets):
    outs = []
    for s in sets:
        o = lf.fit_eval(s["x"], s["y"], s["xq"], s["metric"], M=s.get("M"), Mk=s.get("Mk"))
        outs.append(o)
    torch.cuda.synchronize()
    return [{k: v.cpu().numpy() for k, v in o.items()} for o in outs]


def _compare_identical(a, b):
    for i, (oa, ob) in enumerate(zip(a, b)):
        for k in ("g", "h_up", "h_lo", "arg_up", "arg_lo"):
            np.testing.assert_array_equal(oa[k], ob[k], err_msg=f"set {i} {k}")


def test_mixed_shapes_and_edge_sets(lf):
    """Different d, monotone patterns, norms, global / per-datum M, a set
    with no queries, a single datum, and sets large enough to be chunked."""
    probs = []
    specs = [(2, [0, 0], 2, False, 700, 300), (3, [1, 0, -1], 1, True, 1500, 2000),
             (4, [1, 0, 1, 0], 3, True, 20000, 1500), (5, [0] * 5, 2, False, 1, 64),
             (4, [1, 0, 1, 0], 1, False, 33000, 777), (7, [1, 0, 0, 1, 0, 0, 1], 2, True, 4097, 129),
             (2, [0, 1], 3, False, 50, 0), (10, [1] * 5 + [0] * 5, 2, False, 40000, 600)]
    for k, (d, mon, norm, local, n, q) in enumerate(specs):
        probs.append(W.random_problem(900 + k, n=n, q=q, d=d, norm=norm,
                                      mon=np.array(mon, np.int8), local=local, weighted=(k % 3 == 0)))
    sets = _sets_from(probs, lf)
    plan = lf.Plan(sets)
    got = plan.execute()
    torch.cuda.synchronize()
    got = [{k: v.cpu().numpy() for k, v in o.items()} for o in got]
    ref = _per_set(lf, sets)
    _compare_identical(got, ref)
    for k, p in enumerate(probs):
        if p.q == 0:
            continue
        qidx = np.unique(np.linspace(0, p.q - 1, min(p.q, 40)).astype(int))
        check_bounds(p, got[k], qidx=qidx, label=f"batched set {k}")
    # a second execution of the same graph gives the same results
    got2 = plan.execute()
    torch.cuda.synchronize()
    _compare_identical([{k: v.cpu().numpy() for k, v in o.items()} for o in got2], got)
    plan.close()


def test_batched_workload_full(lf):
    """512 sets, N log-uniform in [500, 50,000], d in {2..10}, half the
    coordinates increasing, Q = 4N, l2: identical to per-set launches, and
    oracle parity on 4 sampled queries per set."""
    probs = W.batched()
    sets = _sets_from(probs, lf)
    plan = lf.Plan(sets)
    got = plan.execute()
    torch.cuda.synchronize()
    got = [{k: v.cpu().numpy() for k, v in o.items()} for o in got]
    ref = _per_set(lf, sets)
    _compare_identical(got, ref)
    rng = np.random.default_rng(44)
    for k in range(0, len(probs), 4):
        p = probs[k]
        qidx = np.sort(rng.choice(p.q, 4, replace=False))
        check_bounds(p, got[k], qidx=qidx, label=f"batched workload set {k}")
    plan.close()


def test_autotuned_tiles_used_by_plans(lf, tmp_path, monkeypatch):
    """lip_autotune on a batched shape class (d = 4, two increasing
    coordinates, l2, N = 5,000, Q = 20,000) stores a configuration for that
    size class; a plan built afterwards runs those sets with the tuned tile
    (lip_plan_tiles); its outputs equal those of a plan with the default
    tiles bit for bit; the table round-trips through the cache file."""
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("LIPFIT_TUNE_CACHE", str(cache))
    lf.tune_clear()
    probs = []
    for k, (n, q) in enumerate([(5000, 20000), (4100, 16400), (6000, 24000)]):
        probs.append(W.random_problem(950 + k, n=n, q=q, d=4, norm=2,
                                      mon=np.array([0, 1, 0, 1], np.int8)))
    probs.append(W.random_problem(960, n=700, q=2800, d=3, norm=1, mon=np.array([1, 0, 0], np.int8)))
    sets = _sets_from(probs, lf)
    default = lf.tune_get(4, 2, "l2", 5000, 20000)
    plan0 = lf.Plan(sets)
    assert plan0.tiles(0)["tile"] == default["tile"]
    ref = [{k: v.cpu().numpy() for k, v in o.items()} for o in plan0.execute()]
    torch.cuda.synchronize()
    plan0.close()
    best = lf.autotune(4, 2, "l2", 5000, 20000)
    assert best == lf.tune_get(4, 2, "l2", 5000, 20000)
    assert best == lf.tune_get(4, 2, "l2", 4100, 16400)       # same size class
    assert lf.tune_get(4, 2, "l2", 50, 200)["tile"] == 32   # another size class: default
    # the autotuner wrote the table to LIPFIT_TUNE_CACHE
    import json
    doc = json.loads(cache.read_text())
    assert any(e["d"] == 4 and e["n_mon"] == 2 and e["norm"] == 2 and e["tile"] == best["tile"]
               for e in doc["entries"])
    plan = lf.Plan(sets)
    for i in range(3):
        assert plan.tiles(i)["tile"] == best["tile"], (i, plan.tiles(i), best)
    got = [{k: v.cpu().numpy() for k, v in o.items()} for o in plan.execute()]
    torch.cuda.synchronize()
    plan.close()
    _compare_identical(got, ref)
    _compare_identical(got, _per_set(lf, sets))
    for k, p in enumerate(probs):
        qidx = np.unique(np.linspace(0, p.q - 1, 32).astype(int))
        check_bounds(p, got[k], qidx=qidx, label=f"tuned plan set {k}")
    # the cache file restores the table
    lf.tune_clear()
    assert lf.tune_get(4, 2, "l2", 5000, 20000) == default
    lf.tune_load(str(cache))
    assert lf.tune_get(4, 2, "l2", 5000, 20000) == best
    lf.tune_clear()
