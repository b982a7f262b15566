"""Pins of the oracle's k-best weighted bounds (Sec. 5, k > 1 with weights).

Against: a hand-worked example, the k = 1 case (the pinned bounds of Eq. 2),
the k = n uniform-weight case (the mean of all candidates, from scipy cdist),
invariance under a permutation of the data (the k best form a multiset), the
order between the k-best and the best bounds, and constant data.
"""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

import oracle

NORMS = [oracle.L1, oracle.L2, oracle.LINF]
SCIPY_METRIC = {oracle.L1: "cityblock", oracle.L2: "euclidean", oracle.LINF: "chebyshev"}


def test_hand_worked_example():
    # x = 0, 1, 3 with y = 0, 1, 0, M = 1 (every norm is |.| in 1-D).
    # query 2:   u = 2, 2, 1 -> 1, 2, 2;    l = -2, 0, -1 -> 0, -1, -2
    #   k = 2, w = (3/4, 1/4): H_up = 3/4 + 2/4 = 5/4, H_lo = 0 - 1/4 = -1/4, g = 1/2
    #   k = 3, w = (1/2, 1/4, 1/4): H_up = 1/2 + 1/2 + 1/2 = 3/2, H_lo = 0 - 1/4 - 1/2 = -3/4
    # query -1:  u = 1, 3, 4;   l = -1, -1, -4
    #   k = 2, w = (3/4, 1/4): H_up = 3/4 + 3/4 = 3/2, H_lo = -3/4 - 1/4 = -1
    x = np.array([[0.0], [1.0], [3.0]], np.float32)
    y = np.array([0.0, 1.0, 0.0], np.float32)
    for norm in NORMS:
        hu, hl, g = oracle.bounds_k(x, y, [[2.0], [-1.0]], norm, [0.75, 0.25], M=1.0)
        np.testing.assert_array_equal(hu, [1.25, 1.5])
        np.testing.assert_array_equal(hl, [-0.25, -1.0])
        np.testing.assert_array_equal(g, [0.5, 0.25])
        hu, hl, g = oracle.bounds_k(x, y, [[2.0]], norm, [0.5, 0.25, 0.25], M=1.0)
        assert (hu[0], hl[0]) == (1.5, -0.75)


@pytest.mark.parametrize("norm", NORMS)
def test_k1_is_the_best_bound(norm):
    rng = np.random.default_rng(1)
    x = rng.random((300, 3)).astype(np.float32)
    y = rng.random(300).astype(np.float32)
    xq = rng.random((50, 3)).astype(np.float32)
    Mk = (0.5 + rng.random(300)).astype(np.float32)
    mon = np.array([1, 0, -1], np.int8)
    a = oracle.bounds_k(x, y, xq, norm, [1.0], Mk=Mk, mon=mon)
    b = oracle.bounds(x, y, xq, norm, Mk=Mk, mon=mon)
    for u, v in zip(a, b[:3]):
        np.testing.assert_array_equal(u, v)


@pytest.mark.parametrize("norm", NORMS)
def test_all_data_uniform_weights_is_the_mean(norm):
    rng = np.random.default_rng(2)
    n = 40
    x = rng.random((n, 2)).astype(np.float32)
    y = rng.random(n).astype(np.float32)
    xq = rng.random((7, 2)).astype(np.float32)
    hu, hl, g = oracle.bounds_k(x, y, xq, norm, np.full(n, 1.0 / n), M=1.5)
    D = cdist(xq.astype(np.float64), x.astype(np.float64), SCIPY_METRIC[norm])
    np.testing.assert_allclose(hu, (y[None, :] + 1.5 * D).mean(1), rtol=1e-13)
    np.testing.assert_allclose(hl, (y[None, :] - 1.5 * D).mean(1), rtol=1e-13)


@pytest.mark.parametrize("norm", NORMS)
def test_permutation_order_and_constant_data(norm):
    rng = np.random.default_rng(3)
    x = rng.random((200, 4)).astype(np.float32)
    y = rng.random(200).astype(np.float32)
    xq = rng.random((30, 4)).astype(np.float32)
    wk = [0.5, 0.3, 0.2]
    a = oracle.bounds_k(x, y, xq, norm, wk, M=0.8)
    perm = rng.permutation(200)
    b = oracle.bounds_k(x[perm], y[perm], xq, norm, wk, M=0.8)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)
    best = oracle.bounds(x, y, xq, norm, M=0.8)
    assert np.all(a[0] >= best[0]) and np.all(a[1] <= best[1])
    c = oracle.bounds_k(x, np.full(200, 2.5, np.float32), xq, norm, wk, M=0.0)
    assert np.all(c[0] == 2.5) and np.all(c[1] == 2.5)
