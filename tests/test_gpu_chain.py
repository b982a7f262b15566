"""The benchmark's chain end to end: per-datum constants M_k from the 16
nearest data (Sec. 4.3, scalar form) computed on the GPU and fed straight
into the GPU bounds (Eq. 2-3), against the oracle's own chain (its kNN
constants, rounded up to FP32 as the boundary specifies, then its bounds).

The workload is the benchmark's distribution (d = 4, x ~ U[0,1]^4, two
increasing coordinates) at N = 20,000, where the oracle's all-pairs kNN
takes seconds; Q = 200,000 queries run the forward with many data chunks
(workgroup merge with several partials), the oracle checks 2,048 sampled
queries.  The GPU constants must equal the oracle's bit for bit (FP64 and
the rounded-up FP32 copy); the bounds follow the ordinary parity rules.
"""
import numpy as np
import pytest
import torch

import oracle
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


@pytest.mark.parametrize("norm", [1, 2, 3])
def test_knn_constants_then_bounds(lf, norm):
    p = W.monotone_local(n=20_000, q=200_000, norm=norm)
    met = lf.Metric(p.d, norm, mon=p.mon, w=p.w)
    x = torch.from_numpy(p.x).to(DEV)
    y = torch.from_numpy(p.y).to(DEV)
    xq = torch.from_numpy(p.xq).to(DEV)
    M64, M32, _ = lf.estimate_M(x, y, met, mode="knn", knn=16)
    out = lf.fit_eval(x, y, xq, met, Mk=M32)
    torch.cuda.synchronize()
    gpu = {k: v.cpu().numpy() for k, v in out.items()}

    st, Mo, _ = oracle.estimate_M_knn(p.x, p.y, norm, K=16, w=p.w)
    assert st == 0
    Mo32 = oracle.round_up_f32(Mo)
    np.testing.assert_array_equal(M64.cpu().numpy(), Mo)
    np.testing.assert_array_equal(M32.cpu().numpy(), Mo32)

    po = W.Problem(p.name, p.x, p.y, p.M, Mo32, p.xq, norm, p.mon, p.w)
    qidx = np.sort(W.rng_for(2100, norm).choice(p.q, 2048, replace=False))
    print(check_bounds(po, gpu, qidx=qidx, label=f"kNN-16 chain norm={norm}"))
