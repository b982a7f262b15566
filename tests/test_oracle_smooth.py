"""Pins of the oracle's penalty objective of Sec. 4.4 (Eq. 7) and its gradient.

Checked against: the closed form of a two-point problem (objective, gradient
and the analytic minimiser), central finite differences of the objective,
the consistency check (F(0) = 0 exactly when the data violate no
constraint), translation invariance of the pair terms, the conservation of
the pair gradients (each term pushes two corrections equally and oppositely),
and the limit of a large constant (only the (1/p) ||eps||^2 term left).
"""
import numpy as np
import pytest

import oracle

NORMS = [oracle.L1, oracle.L2, oracle.LINF]


def _data(seed, n, d, noise=0.05):
    rng = np.random.default_rng(seed)
    x = rng.random((n, d)).astype(np.float32)
    y = (np.sin(2 * x[:, 0]) + x[:, -1] + noise * rng.standard_normal(n)).astype(np.float32)
    return x, y, rng


@pytest.mark.parametrize("norm", NORMS)
def test_two_point_closed_form(norm):
    # x = 0, 1 with y = 0, 3, M = 1; with D = z_1 - z_0 = 3 + e1 - e0:
    #   F = (e0^2 + e1^2) / p + 2 (D - 1)_+^2 + 2 (-D - 1)_+^2
    #   dF/de1 = 2 e1 / p + 4 (D - 1)_+ - 4 (-D - 1)_+,  dF/de0 = 2 e0 / p - (same pair part)
    x = np.array([[0.0], [1.0]], np.float32)
    y = np.array([0.0, 3.0], np.float32)
    for p in (0.25, 1.0, 3.0):
        for e0, e1 in ((0.0, 0.0), (0.5, -0.25), (-1.0, 2.0), (3.0, -3.5), (2.0, -1.0)):
            D = 3.0 + e1 - e0
            pair = 2 * max(D - 1, 0) ** 2 + 2 * max(-D - 1, 0) ** 2
            dpair = 4 * max(D - 1, 0) - 4 * max(-D - 1, 0)
            F, g = oracle.smooth(x, y, [e0, e1], norm, M=1.0, p=p)
            assert F == pytest.approx((e0 ** 2 + e1 ** 2) / p + pair, rel=1e-14, abs=1e-14)
            np.testing.assert_allclose(g, [2 * e0 / p - dpair, 2 * e1 / p + dpair], rtol=1e-14,
                                       atol=1e-14)
        # the minimiser is e0 = -e1 = 4p / (1 + 4p): zero gradient there
        e = 4 * p / (1 + 4 * p)
        _, g = oracle.smooth(x, y, [e, -e], norm, M=1.0, p=p)
        assert np.max(np.abs(g)) < 1e-12


@pytest.mark.parametrize("norm", NORMS)
@pytest.mark.parametrize("local", [False, True])
def test_gradient_matches_finite_differences(norm, local):
    x, y, rng = _data(1 + norm, 40, 3)
    mon = np.array([1, 0, -1], np.int8)
    w = np.array([1.0, 0.5, 2.0])
    Mk = (0.5 + rng.random(40)).astype(np.float32) if local else None
    eps = 0.1 * rng.standard_normal(40)
    F, g = oracle.smooth(x, y, eps, norm, M=0.7, Mk=Mk, p=2.0, mon=mon, w=w)
    h = 1e-6
    fd = np.empty(40)
    for i in range(40):
        ep, em = eps.copy(), eps.copy()
        ep[i] += h
        em[i] -= h
        fd[i] = (oracle.smooth(x, y, ep, norm, M=0.7, Mk=Mk, p=2.0, mon=mon, w=w)[0] -
                 oracle.smooth(x, y, em, norm, M=0.7, Mk=Mk, p=2.0, mon=mon, w=w)[0]) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-6 * max(1.0, np.abs(g).max()))


@pytest.mark.parametrize("norm", NORMS)
def test_zero_penalty_iff_consistent(norm):
    x, y, _ = _data(5, 60, 2, noise=0.0)
    mon = np.array([0, 1], np.int8)
    for M, expect_zero in ((50.0, True), (0.3, False)):
        F, g = oracle.smooth(x, y, np.zeros(60), norm, M=M, p=1.0, mon=mon)
        c = oracle.consistency(x, y, norm, M=M, mon=mon)
        viol = c["viol_up"].sum() + c["viol_lo"].sum()
        assert (F == 0.0) == (viol == 0) == expect_zero
        if expect_zero:
            assert np.all(g == 0.0)
    # per-datum constants: each constraint uses the constant of its datum k
    for mk, expect_zero in ((50.0, True), (0.3, False)):
        Mk = np.full(60, mk, np.float32)
        F, _ = oracle.smooth(x, y, np.zeros(60), norm, M=50.0 if mk < 1 else 0.3, Mk=Mk, p=1.0,
                             mon=mon)
        c = oracle.consistency(x, y, norm, Mk=Mk, mon=mon)
        viol = c["viol_up"].sum() + c["viol_lo"].sum()
        assert (F == 0.0) == (viol == 0) == expect_zero


@pytest.mark.parametrize("norm", NORMS)
def test_translation_invariance_and_conservation(norm):
    x, y, rng = _data(6, 50, 4)
    mon = np.array([1, 0, 1, 0], np.int8)
    eps = 0.2 * rng.standard_normal(50)
    p = 0.5
    F0, g0 = oracle.smooth(x, y, eps, norm, M=0.5, p=p, mon=mon)
    F1, g1 = oracle.smooth(x, y, eps + 0.75, norm, M=0.5, p=p, mon=mon)
    assert F1 - F0 == pytest.approx((np.sum((eps + 0.75) ** 2) - np.sum(eps ** 2)) / p, rel=1e-9)
    # the pair part of the gradient is unchanged by a common shift
    np.testing.assert_allclose(g1 - 2 * (eps + 0.75) / p, g0 - 2 * eps / p, rtol=1e-9, atol=1e-9)
    # every pair term moves two corrections by equal and opposite amounts
    assert abs(np.sum(g0 - 2 * eps / p)) <= 1e-9 * np.abs(g0).sum()


def test_large_constant_leaves_the_ridge_term():
    x, y, rng = _data(7, 30, 2)
    eps = 0.01 * rng.standard_normal(30)
    F, g = oracle.smooth(x, y, eps, oracle.L2, M=1e6, p=0.5)
    assert F == pytest.approx(np.sum(eps ** 2) / 0.5, rel=1e-14)
    np.testing.assert_allclose(g, 2 * eps / 0.5, rtol=1e-14)
