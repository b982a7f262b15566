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


# ---- pre-screening of Sec. 5 ------------------------------------------------------
# An ordered pair (i, k) leaves the sums when y_i - y_k <= c M_k dist_up and
# y_k - y_i <= c M_k dist_lo on the given data y.  The cases below are worked by
# hand; every value is exact in binary floating point.


@pytest.mark.parametrize("norm", NORMS)
def test_prune_three_points_by_hand(norm):
    # x = 0, 1, 3; y = 0, 0.25, 2; M = 1, p = 1; eps = (2, 0, -4) -> z = (2, 0.25, -2).
    # c = 0.25: c M d = 0.25, 0.75, 0.5 for the pairs {0,1}, {0,2}, {1,2} against
    # |dy| = 0.25, 2, 1.75: only {0,1} is dropped (a tie, kept out by <=), although
    # its z values violate the constraint (a_01 = 1.75 - 1 = 0.75).
    # kept: {0,2}: a_02 = b_20 = 4 - 3 = 1; {1,2}: a_12 = b_21 = 2.25 - 2 = 0.25.
    #   F = (4 + 16) + 2 (1 + 0.0625) = 22.125;  g = (4 + 4, 1, -8 - 4 - 1) = (8, 1, -13)
    # c = 0.24 (or 0) keeps {0,1}: F = 22.125 + 2 * 0.5625 = 23.25, g = (11, -2, -13)
    x = np.array([[0.0], [1.0], [3.0]], np.float32)
    y = np.array([0.0, 0.25, 2.0], np.float32)
    eps = [2.0, 0.0, -4.0]
    F, g = oracle.smooth(x, y, eps, norm, M=1.0, p=1.0, prune=0.25)
    assert F == 22.125
    np.testing.assert_array_equal(g, [8.0, 1.0, -13.0])
    for c in (0.24, 0.0):
        F, g = oracle.smooth(x, y, eps, norm, M=1.0, p=1.0, prune=c)
        assert F == 23.25
        np.testing.assert_array_equal(g, [11.0, -2.0, -13.0])


@pytest.mark.parametrize("norm", NORMS)
def test_prune_directional_distances_by_hand(norm):
    # One increasing coordinate, x = 0, 1, M = 1, p = 1, c = 0.25.
    # (i, k) = (0, 1): dist_up = 0, dist_lo = 1;  (1, 0): dist_up = 1, dist_lo = 0.
    x = np.array([[0.0], [1.0]], np.float32)
    mon = np.array([1], np.int8)
    # y = (0.25, 0) decreases: (0, 1) needs 0.25 <= 0, (1, 0) needs 0.25 <= 0: both
    # kept (|dy| <= c M |dx| would drop them).  eps = 0: a_01 = 0.25 and
    # b_10 = z_0 - z_1 - 0 = 0.25:  F = 2 * 0.0625 = 0.125,  g = (1, -1)
    F, g = oracle.smooth(x, [0.25, 0.0], [0.0, 0.0], norm, M=1.0, p=1.0, mon=mon, prune=0.25)
    assert F == 0.125
    np.testing.assert_array_equal(g, [1.0, -1.0])
    # y = (0, 0.25) increases: (0, 1): -0.25 <= 0 and 0.25 <= 0.25; (1, 0): 0.25 <= 0.25
    # and -0.25 <= 0: both dropped.  eps = (1, -1): F = 2, g = (2, -2); without the
    # pre-screening a_01 = b_10 = 1.75 add 2 * 3.0625: F = 8.125, g = (9, -9)
    F, g = oracle.smooth(x, [0.0, 0.25], [1.0, -1.0], norm, M=1.0, p=1.0, mon=mon, prune=0.25)
    assert F == 2.0
    np.testing.assert_array_equal(g, [2.0, -2.0])
    F, g = oracle.smooth(x, [0.0, 0.25], [1.0, -1.0], norm, M=1.0, p=1.0, mon=mon)
    assert F == 8.125
    np.testing.assert_array_equal(g, [9.0, -9.0])


@pytest.mark.parametrize("norm", NORMS)
def test_prune_uses_the_datums_constant_by_hand(norm):
    # x = 0, 1; y = (0, 0.25); M_k = (1, 0.5); c = 0.25; eps = (1, -1) -> z = (1, -0.75).
    # (0, 1) with M_1: 0.25 <= 0.125 fails -> kept: a_01 = 1.75 - 0.5 = 1.25;
    # (1, 0) with M_0: 0.25 <= 0.25 and -0.25 <= 0.25 -> dropped.
    #   F = 2 + 1.5625 = 3.5625,  g = (2 + 2.5, -2 - 2.5)
    # (With the row's constant M_i instead, (1, 0) would stay: b_10 = 1.75 - 1.)
    x = np.array([[0.0], [1.0]], np.float32)
    F, g = oracle.smooth(x, [0.0, 0.25], [1.0, -1.0], norm, Mk=[1.0, 0.5], p=1.0, prune=0.25)
    assert F == 3.5625
    np.testing.assert_array_equal(g, [4.5, -4.5])


@pytest.mark.parametrize("norm", NORMS)
@pytest.mark.parametrize("local", [False, True])
def test_prune_nested_in_c_and_large_c_limit(norm, local):
    # the dropped sets grow with c (M_k dist >= 0), so F cannot grow; a c beyond every
    # |dy| / (M_k dist) drops all pairs of distinct points (the data here are distinct)
    x, y, rng = _data(20 + norm, 60, 3)
    mon = np.array([1, 0, -1], np.int8)
    Mk = (0.5 + rng.random(60)).astype(np.float32) if local else None
    eps = 0.5 * rng.standard_normal(60)
    Fs = [oracle.smooth(x, y, eps, norm, M=0.3, Mk=Mk, p=2.0, mon=mon, prune=c)[0]
          for c in (0.0, 0.05, 0.2, 1 / 3, 1.0, 4.0)]
    assert all(a >= b for a, b in zip(Fs, Fs[1:]))
    assert Fs[0] > Fs[-2]
    # with monotone coordinates some distances are 0 while dy != 0: only a c beyond
    # every ratio drops everything, so use the free coordinate alone there
    Ff, gf = oracle.smooth(x, y, eps, norm, M=0.3, Mk=Mk, p=2.0, prune=1e9)
    assert Ff == pytest.approx(float(np.sum(eps ** 2)) / 2.0, rel=1e-14)
    np.testing.assert_allclose(gf, eps, rtol=1e-14, atol=0)


@pytest.mark.parametrize("norm", NORMS)
def test_prune_gradient_matches_finite_differences(norm):
    # the dropped set depends on y only, so F stays piecewise quadratic in eps
    x, y, rng = _data(30 + norm, 40, 3)
    mon = np.array([0, 1, 0], np.int8)
    Mk = (0.2 + rng.random(40)).astype(np.float32)
    eps = 0.3 * rng.standard_normal(40)
    F, g = oracle.smooth(x, y, eps, norm, Mk=Mk, p=1.5, mon=mon, prune=1 / 3)
    F0, _ = oracle.smooth(x, y, eps, norm, Mk=Mk, p=1.5, mon=mon)
    assert F < F0
    h = 1e-6
    fd = np.empty(40)
    for i in range(40):
        ep, em = eps.copy(), eps.copy()
        ep[i] += h
        em[i] -= h
        fd[i] = (oracle.smooth(x, y, ep, norm, Mk=Mk, p=1.5, mon=mon, prune=1 / 3)[0]
                 - oracle.smooth(x, y, em, norm, Mk=Mk, p=1.5, mon=mon, prune=1 / 3)[0]) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-6)


def _directional_numpy(x, mon, w, norm):
    """All ordered pairs' directional distances (rows i, columns k) from
    numpy broadcasting: c_up / c_lo per coordinate as in Eq. (4) and its
    mirror (free: |d|), weighted, then the norm."""
    diff = x[:, None, :].astype(np.float64) - x[None, :, :].astype(np.float64)
    pos, neg = np.maximum(diff, 0.0), np.maximum(-diff, 0.0)
    m = np.asarray(mon)[None, None, :]
    cu = np.where(m == 0, np.abs(diff), np.where(m > 0, pos, neg)) * w
    cl = np.where(m == 0, np.abs(diff), np.where(m > 0, neg, pos)) * w
    f = {oracle.L1: lambda c: c.sum(-1), oracle.L2: lambda c: np.sqrt((c * c).sum(-1)),
         oracle.LINF: lambda c: c.max(-1)}[norm]
    return f(cu), f(cl)


@pytest.mark.parametrize("norm", NORMS)
@pytest.mark.parametrize("prune", [0.0, 1.0 / 3.0])
def test_smooth_scale_brute_force(norm, prune):
    """The error scale of Eq. (7) used by the GPU tolerances: A = sum of the
    positive parts of a_ik and b_ik over the kept ordered pairs, row_abs[i] =
    sum of 2 (t)_+ over the four terms that move eps_i, row_cnt[i] = number
    of them above -tau, from an independent numpy evaluation; plus the
    identities sum(row_abs) = 4 A and sum(row_cnt) = 2 x (terms above -tau)."""
    x, y, rng = _data(77, 37, 3)
    mon = np.array([1, 0, -1], np.int8)
    w = np.array([1.0, 0.5, 2.0])
    Mk = rng.uniform(0.3, 1.5, len(y)).astype(np.float32)
    eps = 0.2 * rng.standard_normal(len(y))
    tau = 0.05
    A, ra, rc = oracle.smooth_scale(x, y, eps, norm, tau, Mk=Mk, mon=mon, w=w, prune=prune)
    du, dl = _directional_numpy(x, mon, w, norm)
    yd, mk = y.astype(np.float64), Mk.astype(np.float64)[None, :]
    z = yd + eps
    off = ~np.eye(len(y), dtype=bool)
    keep = off.copy()
    if prune > 0:
        dy = yd[:, None] - yd[None, :]
        keep &= ~((dy <= prune * mk * du) & (-dy <= prune * mk * dl))
    dz = z[:, None] - z[None, :]
    t = np.stack([dz - mk * du, -dz - mk * dl])           # a_ik, b_ik
    v = np.where(keep, np.maximum(t, 0.0), 0.0)
    above = keep & (t > -tau)
    want_A = v.sum()
    want_ra = 2 * v.sum(axis=(0, 2)) + 2 * v.sum(axis=(0, 1))
    want_rc = above.sum(axis=(0, 2)) + above.sum(axis=(0, 1))
    assert want_A > 0
    assert A == pytest.approx(want_A, rel=1e-12)
    np.testing.assert_allclose(ra, want_ra, rtol=1e-12, atol=1e-14)
    np.testing.assert_array_equal(rc, want_rc)
    assert ra.sum() == pytest.approx(4 * A, rel=1e-12)
    assert rc.sum() == 2 * above.sum()
