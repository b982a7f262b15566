"""LIP_FLAG_CHECK_FINITE on every entry point that takes it: a NaN, +Inf or
-Inf in any input array gives LIP_E_NONFINITE (the Lipschitz condition of
Sec. 1 and the constant of Sec. 5 are only defined for finite data), and on
finite inputs the flag changes no result."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
NONFINITE = 4
BAD = [np.nan, np.inf, -np.inf]


@pytest.fixture(scope="module")
def lf():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2606_04670_amd as lf
    lf.load()
    return lf


def _t(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _poisoned(a, k, v):
    b = np.array(a, copy=True)
    b.reshape(-1)[k % b.size] = v
    return b


def _expect_nonfinite(lf, fn):
    with pytest.raises(lf.LipError) as e:
        fn()
        torch.cuda.synchronize()
    assert e.value.status == NONFINITE


@pytest.fixture(scope="module")
def prob():
    return W.random_problem(77, n=700, q=300, d=3, norm=2, mon=np.array([1, 0, 0], np.int8),
                            local=True)


def test_fit_eval_and_bounds(lf, prob):
    p = prob
    met = lf.Metric(3, 2, mon=p.mon)
    ref = lf.fit_eval(_t(p.x), _t(p.y), _t(p.xq), met, Mk=_t(p.Mk))
    got = lf.fit_eval(_t(p.x), _t(p.y), _t(p.xq), met, Mk=_t(p.Mk), check_finite=True)
    for k in ref:
        assert torch.equal(ref[k], got[k]), k
    for i, v in enumerate(BAD):
        for name in ("x", "y", "xq", "Mk"):
            arrs = dict(x=p.x, y=p.y, xq=p.xq, Mk=p.Mk)
            arrs[name] = _poisoned(arrs[name], 37 * i + 5, v)
            _expect_nonfinite(lf, lambda: lf.fit_eval(_t(arrs["x"]), _t(arrs["y"]),
                                                      _t(arrs["xq"]), met, Mk=_t(arrs["Mk"]),
                                                      check_finite=True))
    # the BF16 path takes the same checks
    met2 = lf.Metric(3, 2)
    _expect_nonfinite(lf, lambda: lf.fit_eval(_t(_poisoned(p.x, 3, np.nan)), _t(p.y), _t(p.xq),
                                              met2, M=1.0, bf16=True, check_finite=True))


def test_backward(lf, prob):
    p = prob
    met = lf.Metric(3, 2, mon=p.mon)
    out = lf.fit_eval(_t(p.x), _t(p.y), _t(p.xq), met, Mk=_t(p.Mk))
    args = lambda **kw: dict(dict(dg=_t(p.dg), Mk=_t(p.Mk)), **kw)
    r0 = lf.backward(_t(p.x), _t(p.y), _t(p.xq), met, out["arg_up"], out["arg_lo"],
                     deterministic=True, **args())
    r1 = lf.backward(_t(p.x), _t(p.y), _t(p.xq), met, out["arg_up"], out["arg_lo"],
                     deterministic=True, check_finite=True, **args())
    for a, b in zip(r0, r1):
        assert torch.equal(a, b)
    _expect_nonfinite(lf, lambda: lf.backward(_t(p.x), _t(p.y), _t(p.xq), met, out["arg_up"],
                                              out["arg_lo"], check_finite=True,
                                              **args(dg=_t(_poisoned(p.dg, 9, np.inf)))))
    _expect_nonfinite(lf, lambda: lf.backward(_t(p.x), _t(p.y), _t(_poisoned(p.xq, 4, np.nan)),
                                              met, out["arg_up"], out["arg_lo"],
                                              check_finite=True, **args()))


def test_data_side(lf, prob):
    p = prob
    met = lf.Metric(3, 2, mon=p.mon)
    sym = lf.Metric(3, 2)
    r0 = lf.consistency(_t(p.x), _t(p.y), met, Mk=_t(p.Mk))
    r1 = lf.consistency(_t(p.x), _t(p.y), met, Mk=_t(p.Mk), check_finite=True)
    for k in r0:
        assert torch.equal(r0[k], r1[k]), k
    for v in BAD:
        _expect_nonfinite(lf, lambda: lf.consistency(_t(_poisoned(p.x, 11, v)), _t(p.y), met,
                                                     Mk=_t(p.Mk), check_finite=True))
        _expect_nonfinite(lf, lambda: lf.consistency(_t(p.x), _t(p.y), met,
                                                     Mk=_t(_poisoned(p.Mk, 2, v)),
                                                     check_finite=True))
        for mode in ("global", "knn"):
            _expect_nonfinite(lf, lambda: lf.estimate_M(_t(p.x), _t(_poisoned(p.y, 6, v)), sym,
                                                        mode=mode, check_finite=True))
    kn = np.array([0.2, 0.5])
    _expect_nonfinite(lf, lambda: lf.local_steps(_t(_poisoned(p.x, 1, np.nan)), _t(p.y), sym, kn,
                                                 check_finite=True))


def test_further_forms(lf, prob):
    p = prob
    met = lf.Metric(3, 2, mon=p.mon)
    for v in BAD:
        _expect_nonfinite(lf, lambda: lf.fit_eval_k(_t(p.x), _t(p.y),
                                                    _t(_poisoned(p.xq, 7, v)), met, [0.5, 0.5],
                                                    Mk=_t(p.Mk), check_finite=True))
        eps = _poisoned(np.zeros(p.n, np.float32), 13, v)
        _expect_nonfinite(lf, lambda: lf.smooth_objective(_t(p.x), _t(p.y), _t(eps), met,
                                                          Mk=_t(p.Mk), check_finite=True))
    sym = lf.Metric(3, 2)
    kn = np.array([0.2, 0.5])
    d1, _, V32 = lf.local_steps(_t(p.x), _t(p.y), sym, kn)
    Vb = V32.clone()
    Vb[5, 1] = float("inf")
    _expect_nonfinite(lf, lambda: lf.fit_eval_steps(_t(p.x), _t(p.y), _t(p.xq), met, kn, d1, Vb,
                                                    check_finite=True))
    ok = lf.fit_eval_k(_t(p.x), _t(p.y), _t(p.xq), met, [0.5, 0.5], Mk=_t(p.Mk), check_finite=True)
    ref = lf.fit_eval_k(_t(p.x), _t(p.y), _t(p.xq), met, [0.5, 0.5], Mk=_t(p.Mk))
    for k in ref:
        assert torch.equal(ok[k], ref[k])
