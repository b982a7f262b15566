"""Parity with translated coordinates: the data and the queries shifted by 2^7
and 2^10 in every coordinate, with and without distance weights.

Eq. (2) depends on the coordinates only through x - x^k, so the FP32 error
of every form must scale with the data's extent and the distances, not with
the size of the coordinates.  Each case is compared with the FP64 oracle
under the ordinary rules of tests/_parity.py (1e-5 relative with the data
scale where a value is near 0; indices exact outside the a-priori tie band,
whose width depends on the extent of the box that holds data and queries, not
on its position); the batched plan and the BF16 path must also stay bitwise
equal to the plain FP32 path.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from _parity import check_bounds, check_bounds_regional, check_bounds_steps, value_ok

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
SHIFTS = [2.0 ** 7, 2.0 ** 10]
KEYS = ("g", "h_up", "h_lo", "arg_up", "arg_lo")


@pytest.fixture(scope="module")
def lf():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2606_04670_amd as lf
    lf.load()
    return lf


def _t(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def shifted(p: W.Problem, s: float) -> W.Problem:
    """The same problem with every coordinate of x and xq moved by s (FP32)."""
    x = (p.x.astype(np.float64) + s).astype(np.float32)
    xq = (p.xq.astype(np.float64) + s).astype(np.float32)
    return W.Problem(p.name + f"+{s:g}", x, p.y, p.M, p.Mk, xq, p.norm, p.mon, p.w, p.dg)


def _fit(lf, p, metric=None, **kw):
    met = metric or lf.Metric(p.d, p.norm, mon=p.mon, w=p.w)
    mk = _t(p.Mk)
    out = lf.fit_eval(_t(p.x), _t(p.y), _t(p.xq), met, M=None if mk is not None else p.M, Mk=mk,
                      **kw)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


MON4 = {"free": [0, 0, 0, 0], "mon": [1, 0, 1, 0], "mixed": [0, -1, 0, 1]}


@pytest.mark.parametrize("shift", SHIFTS)
@pytest.mark.parametrize("norm", [1, 2, 3])
@pytest.mark.parametrize("pattern", sorted(MON4))
@pytest.mark.parametrize("weighted", [False, True])
def test_fit_eval_shifted(lf, shift, norm, pattern, weighted):
    for local in (False, True):
        p = W.random_problem(9000 + norm * 10 + local, n=1537, q=700, d=4, norm=norm,
                             mon=np.array(MON4[pattern], np.int8), local=local,
                             weighted=weighted)
        ps = shifted(p, shift)
        print(check_bounds(ps, _fit(lf, ps), label=f"{ps.name} norm={norm} {pattern} "
                                                   f"w={weighted} local={local}"))


@pytest.mark.parametrize("shift", SHIFTS)
def test_fit_eval_shifted_other_dims(lf, shift):
    for d, mon in ((1, [1]), (2, [0, 1]), (7, [1, -1, 0, 0, 1, 0, 0]), (16, [0, 1] * 8)):
        for norm in (1, 2, 3):
            p = W.random_problem(9100 + d * 3 + norm, n=900, q=333, d=d, norm=norm,
                                 mon=np.array(mon, np.int8), local=True, weighted=True)
            ps = shifted(p, shift)
            check_bounds(ps, _fit(lf, ps), label=f"{ps.name} d={d} norm={norm}")


@pytest.mark.parametrize("shift", SHIFTS)
def test_benchmark_workload_shifted_sampled(lf, shift):
    """d = 4, N = 100,000, Q = 1,000,000 shifted, l1 with two increasing
    coordinates (the headline form), oracle on 256 sampled queries."""
    ps = shifted(W.monotone_local(norm=1), shift)
    out = _fit(lf, ps)
    qidx = np.sort(np.random.default_rng(int(shift)).choice(ps.q, 256, replace=False))
    print(check_bounds(ps, out, qidx=qidx, label=f"monotone_local l1 +{shift:g}"))


@pytest.mark.parametrize("shift", SHIFTS)
def test_bf16_shifted_identical_to_fp32(lf, shift):
    p = shifted(W.mixed_l2(n=20_000, q=5_000), shift)
    ref = _fit(lf, p)
    got = _fit(lf, p, bf16=True)
    for k in KEYS:
        np.testing.assert_array_equal(got[k], ref[k], err_msg=k)
    check_bounds(p, got, qidx=np.linspace(0, p.q - 1, 48).astype(int), label=f"bf16 +{shift:g}")


@pytest.mark.parametrize("shift", SHIFTS)
def test_batched_shifted(lf, shift):
    """A plan over shifted sets (different shifts per set, so the origins
    differ) equals per-set calls bit for bit and the oracle on samples."""
    probs = W.batched(n_sets=12, n_scale=0.05, norm=2)[:6] + W.batched(n_sets=12, n_scale=0.05,
                                                                      norm=1)[6:]
    probs = [shifted(p, shift * (1 + i % 3)) for i, p in enumerate(probs)]
    sets = []
    for p in probs:
        s = dict(x=_t(p.x), y=_t(p.y), xq=_t(p.xq), metric=lf.Metric(p.d, p.norm, mon=p.mon, w=p.w),
                 M=p.M)
        s["out"] = lf.fit_eval(s["x"], s["y"], s["xq"], s["metric"], M=p.M)
        sets.append(s)
    plan = lf.Plan([dict(x=s["x"], y=s["y"], xq=s["xq"], metric=s["metric"], M=s["M"])
                    for s in sets])
    outs = plan.execute()
    torch.cuda.synchronize()
    for i, (p, s, o) in enumerate(zip(probs, sets, outs)):
        ref = {k: v.cpu().numpy() for k, v in s["out"].items()}
        got = {k: v.cpu().numpy() for k, v in o.items()}
        for k in KEYS:
            np.testing.assert_array_equal(got[k], ref[k], err_msg=f"set {i} {k}")
        qidx = np.linspace(0, p.q - 1, min(p.q, 64)).astype(int)
        check_bounds(p, got, qidx=qidx, label=f"batched set {i}")


@pytest.mark.parametrize("shift", SHIFTS)
@pytest.mark.parametrize("norm", [1, 2, 3])
def test_topk_shifted(lf, shift, norm):
    for mon, wk, weighted in (([1, 0, 1, 0], [0.5, 0.3, 0.2], False),
                              ([0, -1, 0, 1], [0.25, 0.25, 0.25, 0.25], True)):
        p = shifted(W.random_problem(9200 + norm, n=1537, q=400, d=4, norm=norm,
                                     mon=np.array(mon, np.int8), local=True, weighted=weighted),
                    shift)
        met = lf.Metric(4, norm, mon=p.mon, w=p.w)
        out = lf.fit_eval_k(_t(p.x), _t(p.y), _t(p.xq), met, wk, Mk=_t(p.Mk))
        torch.cuda.synchronize()
        hu, hl, g = oracle.bounds_k(p.x, p.y, p.xq, norm, wk, Mk=p.Mk, mon=p.mon, w=p.w)
        ys = float(np.abs(p.y).max())
        for name, want in (("h_up", hu), ("h_lo", hl), ("g", g)):
            ok, err = value_ok(out[name].cpu().numpy(), want, ys)
            assert ok.all(), f"k-best +{shift:g} norm={norm} {name}: max err {err.max():g}"


@pytest.mark.parametrize("shift", SHIFTS)
@pytest.mark.parametrize("norm", [1, 2, 3])
def test_regional_shifted(lf, shift, norm):
    """Cases I-IV with the interval ends shifted with the data."""
    kinds = np.array([2, 3, 4, 5, 0, 1], np.int8)
    p = shifted(W.random_problem(9300 + norm, n=1200, q=500, d=6, norm=norm, local=True,
                                 weighted=True), shift)
    g = W.rng_for(9301, norm)
    a = (g.uniform(0.1, 0.5, 6) + shift).astype(np.float32)
    b = (a.astype(np.float64) + g.uniform(0.0, 0.5, 6)).astype(np.float32)
    met = lf.Metric(6, norm, mon=kinds, w=p.w, a=a, b=b)
    gpu = _fit(lf, p, metric=met)
    print(check_bounds_regional(p, gpu, kinds, a.astype(np.float64), b.astype(np.float64),
                                label=f"regional +{shift:g} norm={norm}"))


@pytest.mark.parametrize("shift", SHIFTS)
@pytest.mark.parametrize("norm", [1, 2, 3])
def test_steps_shifted(lf, shift, norm):
    p = shifted(W.random_problem(9400 + norm, n=1500, q=900, d=4, norm=norm,
                                 mon=np.array([1, 0, 1, 0], np.int8), weighted=True), shift)
    met = lf.Metric(4, norm, mon=p.mon, w=p.w)
    pairs = W.rng_for(9401, norm).integers(0, p.n, size=(3000, 2))
    kn = oracle.knots(p.x, pairs, np.array([0.2, 0.4, 0.6, 0.8]), norm, w=p.w)
    sym = lf.Metric(4, norm, w=p.w)
    d1, V64, V32 = lf.local_steps(_t(p.x), _t(p.y), sym, kn)
    st, d1o, Vo = oracle.local_steps(p.x, p.y, kn, norm, w=p.w)
    assert st == 0
    np.testing.assert_array_equal(V64.cpu().numpy(), Vo)
    out = lf.fit_eval_steps(_t(p.x), _t(p.y), _t(p.xq), met, kn, d1, V32)
    torch.cuda.synchronize()
    gpu = {k: v.cpu().numpy() for k, v in out.items()}
    print(check_bounds_steps(p, gpu, kn, d1.cpu().numpy(), V32.cpu().numpy(),
                             label=f"steps +{shift:g} norm={norm}"))


@pytest.mark.parametrize("shift", SHIFTS)
@pytest.mark.parametrize("norm", [1, 2, 3])
@pytest.mark.parametrize("prune", [0.0, 1.0 / 3.0])
def test_smooth_shifted(lf, shift, norm, prune):
    from test_gpu_smooth import _check
    p = shifted(W.random_problem(9500 + norm, n=1100, q=1, d=4, norm=norm,
                                 mon=np.array([1, 0, 1, 0], np.int8), local=True, weighted=True,
                                 M=0.8), shift)
    eps = (0.05 * W.rng_for(9501, norm).standard_normal(p.n)).astype(np.float32)
    met = lf.Metric(4, norm, mon=p.mon, w=p.w)
    F, grad = lf.smooth_objective(_t(p.x), _t(p.y), _t(eps), met, Mk=_t(p.Mk), p=0.7,
                                  prune=prune)
    torch.cuda.synchronize()
    _check(p, eps.astype(np.float64), F.item(), grad.cpu().numpy().astype(np.float64), p.M,
           p.Mk, 0.7, f"smooth +{shift:g} norm={norm} prune={prune:g}", prune=prune)
