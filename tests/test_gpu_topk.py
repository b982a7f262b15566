"""GPU parity of the k-best weighted bounds (Sec. 5, k > 1) against the oracle.

Values follow the rule of tests/_parity.py (1e-5 relative, max|y| near zero):
each of the k values is an FP32 candidate within the a-priori FP32 error of
the oracle's value of the same rank (a near-tie can swap two candidates of
one rank, whose values then agree to that error as well).  k = 1 must equal
lip_fit_eval's bounds bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from _parity import value_ok

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


CASES = [
    # (seed, n, q, d, mon, wk, local)
    (1, 1000, 700, 2, [0, 0], [0.8, 0.1, 0.1], False),
    (2, 1537, 300, 4, [1, 0, 1, 0], [0.5, 0.5], True),
    (3, 2049, 2500, 4, [0, -1, 0, 1], [0.4, 0.3, 0.2, 0.1], False),
    (4, 3, 100, 3, [1, 1, 1], [0.2, 0.3, 0.5], False),
    (5, 800, 129, 8, [1, 0, 1, 0, 1, 0, 1, 0], [0.7, 0.3], True),
    (6, 513, 64, 16, [0, 1] * 8, [0.25, 0.25, 0.25, 0.25], False),
    (7, 700, 50, 1, [1], [1.0, 0.0, 0.0], False),
]


@pytest.mark.parametrize("norm", [1, 2, 3])
@pytest.mark.parametrize("seed,n,q,d,mon,wk,local", CASES)
def test_fit_eval_k_parity(lf, norm, seed, n, q, d, mon, wk, local):
    p = W.random_problem(700 + seed, n=n, q=q, d=d, norm=norm, mon=np.array(mon, np.int8),
                         local=local, weighted=(seed % 2 == 1))
    met = lf.Metric(d, norm, mon=p.mon, w=p.w)
    mk = None if p.Mk is None else _t(p.Mk)
    out = lf.fit_eval_k(_t(p.x), _t(p.y), _t(p.xq), met, wk, M=None if mk is not None else p.M,
                        Mk=mk)
    torch.cuda.synchronize()
    wk32 = np.asarray(wk, np.float32).astype(np.float64)
    hu, hl, g = oracle.bounds_k(p.x, p.y, p.xq, norm, wk32, M=p.M, Mk=p.Mk, mon=p.mon, w=p.w)
    ys = float(np.abs(p.y).max())
    for name, ov in (("h_up", hu), ("h_lo", hl), ("g", g)):
        ok, err = value_ok(out[name].cpu().numpy(), ov, ys)
        assert ok.all(), f"{name}: max err {err.max():g} at {np.argmax(err)}"


def _wk(k):
    w = 1.0 / np.arange(1, k + 1)
    return (w / w.sum()).tolist()


# k above 4: lists of 8, 16 and 32 values, with split chunks (few queries)
# and k = n
BIG_K = [
    # (seed, n, q, d, mon, k, local)
    (11, 3000, 900, 4, [1, 0, 1, 0], 5, True),
    (12, 2000, 700, 2, [0, 0], 8, False),
    (13, 4097, 500, 3, [1, 0, -1], 13, True),
    (14, 1500, 300, 8, [1, 0] * 4, 16, False),
    (15, 2500, 400, 4, [0, 0, 0, 0], 17, True),
    (16, 5000, 300, 16, [0, 1] * 8, 32, False),
    (17, 32, 100, 2, [1, 0], 32, True),
]


@pytest.mark.parametrize("norm", [1, 2, 3])
@pytest.mark.parametrize("seed,n,q,d,mon,k,local", BIG_K)
def test_fit_eval_k_large_k(lf, norm, seed, n, q, d, mon, k, local):
    test_fit_eval_k_parity(lf, norm, seed, n, q, d, mon, _wk(k), local)


@pytest.mark.parametrize("norm", [1, 2, 3])
def test_k1_equals_fit_eval_bitwise(lf, norm):
    p = W.random_problem(750 + norm, n=5000, q=3000, d=4, norm=norm,
                         mon=np.array([1, 0, 1, 0], np.int8), local=True)
    met = lf.Metric(4, norm, mon=p.mon)
    a = lf.fit_eval_k(_t(p.x), _t(p.y), _t(p.xq), met, [1.0], Mk=_t(p.Mk))
    b = lf.fit_eval(_t(p.x), _t(p.y), _t(p.xq), met, Mk=_t(p.Mk))
    assert torch.equal(a["h_up"], b["h_up"]) and torch.equal(a["h_lo"], b["h_lo"])


@pytest.mark.parametrize("norm", [1, 2, 3])
def test_monotone_local_full_size_sampled(lf, norm):
    """d = 4, N = 1e5, Q = 1e6 with k = 3, w = (0.8, 0.1, 0.1), per-datum M_k:
    sampled queries against the oracle."""
    p = W.monotone_local(norm=norm)
    met = lf.Metric(4, norm, mon=p.mon)
    out = lf.fit_eval_k(_t(p.x), _t(p.y), _t(p.xq), met, [0.8, 0.1, 0.1], Mk=_t(p.Mk))
    torch.cuda.synchronize()
    qi = W.rng_for(760, norm).choice(p.q, 128, replace=False)
    wk = np.asarray([0.8, 0.1, 0.1], np.float32).astype(np.float64)
    hu, hl, g = oracle.bounds_k(p.x, p.y, p.xq[qi], norm, wk, Mk=p.Mk, mon=p.mon)
    ys = float(np.abs(p.y).max())
    for name, ov in (("h_up", hu), ("h_lo", hl), ("g", g)):
        ok, err = value_ok(out[name].cpu().numpy()[qi], ov, ys)
        assert ok.all(), f"{name}: max err {err.max():g}"
