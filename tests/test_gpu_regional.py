"""GPU parity of the bounds with monotonicity on parts of the domain (Sec. 4.2,
cases I-IV on [a_i, b_i]) against the oracle (rules of tests/_parity.py)."""
import numpy as np
import pytest
import torch

import workloads as W
from _parity import check_bounds_regional

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
    # (seed, n, q, kinds, local, weighted)
    (1, 1000, 700, [2], False, False),
    (2, 1537, 300, [3, 0], True, False),
    (3, 2049, 2500, [4, 5, 1, -1], False, True),
    (4, 5, 100, [5, 2, 0], False, False),
    (5, 800, 129, [2, 3, 4, 5, 0, 1, -1, 2], True, True),
    (6, 513, 64, [2, 3, 4, 5] * 4, False, False),
    # free coordinates first in the kernel's order, shared by both distances
    (7, 900, 333, [4, 0, 5, 0], True, False),
    (8, 700, 200, [0, 2, 0, 0, 3, 0, 1, 0, 0, 0, 5, 0, 0, -1, 0, 4], False, True),
]


@pytest.mark.parametrize("norm", [1, 2, 3])
@pytest.mark.parametrize("seed,n,q,kinds,local,weighted", CASES)
def test_regional_parity(lf, norm, seed, n, q, kinds, local, weighted):
    d = len(kinds)
    p = W.random_problem(800 + seed, n=n, q=q, d=d, norm=norm, local=local, weighted=weighted)
    g = W.rng_for(801, seed)
    a = g.uniform(0.1, 0.5, d).astype(np.float32)
    b = (a + g.uniform(0.0, 0.5, d)).astype(np.float32)
    kind = np.array(kinds, np.int8)
    met = lf.Metric(d, norm, mon=kind, w=p.w, a=a, b=b)
    mk = None if p.Mk is None else _t(p.Mk)
    out = lf.fit_eval(_t(p.x), _t(p.y), _t(p.xq), met, M=None if mk is not None else p.M, Mk=mk)
    torch.cuda.synchronize()
    gpu = {k: v.cpu().numpy() for k, v in out.items()}
    print(check_bounds_regional(p, gpu, kind, a.astype(np.float64), b.astype(np.float64),
                                label=f"regional {kinds} norm={norm}"))


def test_regional_kinds_rejected_elsewhere(lf):
    p = W.random_problem(850, n=100, q=10, d=2, norm=2)
    met = lf.Metric(2, 2, mon=[2, 0], a=[0.2, 0.0], b=[0.6, 0.0])
    with pytest.raises(lf.LipError):
        lf.consistency(_t(p.x), _t(p.y), met, M=1.0)
    with pytest.raises(lf.LipError):
        lf.fit_eval(_t(p.x), _t(p.y), _t(p.xq), met, M=1.0, bf16=True)


@pytest.mark.parametrize("norm", [1, 2, 3])
def test_monotone_local_full_size_sampled(lf, norm):
    """d = 4, N = 1e5, Q = 1e6, per-datum M_k, coordinates 1 / 3 as cases III / IV
    on [0.3, 0.6] (the configuration the benchmark times): every query on the GPU,
    a seeded sample of 512 plus the first and last against the oracle, and the same
    outputs on a second call."""
    p = W.monotone_local(norm=norm)
    kind = np.array([4, 0, 5, 0], np.int8)
    a = np.full(4, 0.3, np.float32)
    b = np.full(4, 0.6, np.float32)
    met = lf.Metric(4, norm, mon=kind, a=a, b=b)
    args = (_t(p.x), _t(p.y), _t(p.xq), met)
    out = lf.fit_eval(*args, Mk=_t(p.Mk))
    torch.cuda.synchronize()
    gpu = {k: v.cpu().numpy() for k, v in out.items()}
    qidx = np.sort(W.rng_for(870, norm).choice(p.q, 512, replace=False))
    qidx = np.concatenate([[0, p.q - 1], qidx])
    print(check_bounds_regional(p, gpu, kind, a.astype(np.float64), b.astype(np.float64),
                                qidx=qidx, label=f"regional monotone_local norm={norm}"))
    out2 = lf.fit_eval(*args, Mk=_t(p.Mk))
    for k in out:
        assert torch.equal(out[k], out2[k]), k


@pytest.mark.parametrize("norm", [1, 2, 3])
def test_regional_single_datum(lf, norm):
    p = W.random_problem(880 + norm, n=1, q=300, d=3, norm=norm)
    kind = np.array([2, 0, 5], np.int8)
    a = np.array([0.2, 0.0, 0.4], np.float32)
    b = np.array([0.7, 0.0, 0.5], np.float32)
    met = lf.Metric(3, norm, mon=kind, a=a, b=b)
    out = lf.fit_eval(_t(p.x), _t(p.y), _t(p.xq), met, M=p.M)
    torch.cuda.synchronize()
    gpu = {k: v.cpu().numpy() for k, v in out.items()}
    assert (gpu["arg_up"] == 0).all() and (gpu["arg_lo"] == 0).all()
    print(check_bounds_regional(p, gpu, kind, a.astype(np.float64), b.astype(np.float64),
                                label=f"regional n=1 norm={norm}"))
