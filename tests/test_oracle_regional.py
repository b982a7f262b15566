"""Pins of the oracle's monotonicity on parts of the domain (Sec. 4.2).

The section gives the four cases but not their formulas; the oracle's
components (the length of the part of the coordinate segment where f may
rise / fall in the direction of travel) are checked against:
  * a 1-D brute force: the largest and smallest value any admissible function
    can reach, built step by step on a fine dyadic grid from the allowed
    increments of each step (exact in binary floating point);
  * the special cases that reduce to already pinned forms (kinds 0 / +1 / -1,
    an empty or all-covering unrestricted interval);
  * containment in several dimensions: for a separable function that obeys
    every case, H_lo <= f <= H_up at random points and g = f at the data.
"""
import numpy as np
import pytest

import oracle

NORMS = [oracle.L1, oracle.L2, oracle.LINF]
KINDS = [-1, 0, 1, 2, 3, 4, 5]


def _allowed_step(kind, mid, a, b, M, h):
    """(min, max) change of f over one step of length h moving right, for a
    step whose midpoint is mid (inside one of A, AB, B)."""
    if kind == 0:
        return -M * h, M * h
    if kind == 1:
        return 0.0, M * h
    if kind == -1:
        return -M * h, 0.0
    region = "A" if mid < a else ("B" if mid > b else "AB")
    if region == "AB":
        return -M * h, M * h
    inc = {2: True, 3: False, 4: region == "B", 5: region == "A"}[kind]
    return (0.0, M * h) if inc else (-M * h, 0.0)


def _brute_1d(kind, a, b, xk, yk, x, M, h):
    """Largest and smallest f(x) over the admissible f with f(xk) = yk."""
    hi = lo = yk
    t = xk
    if x >= xk:
        while t < x:
            dmin, dmax = _allowed_step(kind, t + h / 2, a, b, M, h)
            hi, lo, t = hi + dmax, lo + dmin, t + h
    else:
        while t > x:
            dmin, dmax = _allowed_step(kind, t - h / 2, a, b, M, h)
            hi, lo, t = hi - dmin, lo - dmax, t - h
    return hi, lo


@pytest.mark.parametrize("kind", KINDS)
def test_1d_brute_force(kind):
    rng = np.random.default_rng(10 + kind)
    h = 1.0 / 64
    for _ in range(40):
        a, b = sorted(rng.integers(-128, 129, 2) * h)
        xk, x = rng.integers(-192, 193, 2) * h
        yk = float(rng.integers(-64, 65) * h)
        M = float(rng.integers(1, 9)) / 4
        hi, lo = _brute_1d(kind, a, b, xk, yk, x, M, h)
        for norm in NORMS:
            hu, hl, _, _, _ = oracle.bounds_reg(np.array([[xk]], np.float32),
                                                np.array([yk], np.float32),
                                                np.array([[x]], np.float32), norm, [kind], [a],
                                                [b], M=M)
            assert (hu[0], hl[0]) == (hi, lo), (kind, a, b, xk, x, M)


@pytest.mark.parametrize("norm", NORMS)
def test_plain_kinds_match_eq4(norm):
    rng = np.random.default_rng(3)
    x = rng.random((200, 3)).astype(np.float32)
    y = rng.random(200).astype(np.float32)
    xq = rng.uniform(-0.2, 1.2, (60, 3)).astype(np.float32)
    kind = np.array([1, 0, -1], np.int8)
    w = np.array([1.0, 2.0, 0.5])
    a = oracle.bounds_reg(x, y, xq, norm, kind, M=1.3, w=w)
    b = oracle.bounds(x, y, xq, norm, M=1.3, mon=kind, w=w)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)
    # case I / II with an empty unrestricted interval are +1 / -1; any case
    # whose unrestricted interval covers everything is free
    for kind_r, kind_p in ((2, 1), (3, -1)):
        a = oracle.bounds_reg(x, y, xq, norm, [kind_r, 0, kind_r], [0.4, 0, 0.6], [0.4, 0, 0.6],
                              M=1.3)
        b = oracle.bounds(x, y, xq, norm, M=1.3, mon=[kind_p, 0, kind_p])
        for u, v in zip(a, b):
            np.testing.assert_array_equal(u, v)
    a = oracle.bounds_reg(x, y, xq, norm, [2, 4, 5], [-1e30] * 3, [1e30] * 3, M=1.3)
    b = oracle.bounds(x, y, xq, norm, M=1.3)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)


def _piece(kind, t, a, b, L):
    """A 1-D function obeying the kind with slopes of magnitude <= L."""
    t = np.asarray(t, np.float64)
    if kind == 0:
        return L * np.sin(3 * t)
    if kind in (1, -1):
        return kind * L * t
    A, B = t < a, t > b
    mid = np.clip(t, a, b)
    if kind == 2:   # up on A, down on AB, up on B
        return np.where(A, L * (t - a), 0) - L * (mid - a) + np.where(B, L * (t - b), 0)
    if kind == 3:   # down on A, up on AB, down on B
        return -np.where(A, L * (t - a), 0) + L * (mid - a) - np.where(B, L * (t - b), 0)
    if kind == 4:   # down on A, half-slope up on AB, up on B
        return -np.where(A, L * (t - a), 0) + 0.5 * L * (mid - a) + np.where(B, L * (t - b), 0)
    return np.where(A, L * (t - a), 0) - 0.5 * L * (mid - a) - np.where(B, L * (t - b), 0)


@pytest.mark.parametrize("norm", NORMS)
def test_containment_and_interpolation(norm):
    rng = np.random.default_rng(20 + norm)
    d = 4
    kinds = np.array([2, 3, 4, 5], np.int8)
    a = np.array([0.2, 0.3, 0.4, 0.25])
    b = np.array([0.6, 0.5, 0.7, 0.9])
    L = 0.8
    M = L * {oracle.L1: 1, oracle.L2: np.sqrt(d), oracle.LINF: d}[norm]
    f = lambda P: sum(_piece(int(kinds[i]), P[:, i], a[i], b[i], L) for i in range(d))
    x = rng.random((300, d)).astype(np.float32)
    y = f(x.astype(np.float64)).astype(np.float32)
    yv = y.astype(np.float64)
    # the stored values are f rounded to FP32: the sampled function is f + e
    # with |e| <= 2^-24 |f|, so allow that much
    slack = 2.0 ** -23 * max(1.0, np.abs(yv).max())
    xq = rng.uniform(-0.1, 1.1, (400, d)).astype(np.float32)
    hu, hl, g, _, _ = oracle.bounds_reg(x, y, xq, norm, kinds, a, b, M=M)
    fq = f(xq.astype(np.float64))
    assert np.all(hl <= fq + slack) and np.all(fq <= hu + slack)
    hu, hl, g, _, _ = oracle.bounds_reg(x, y, x, norm, kinds, a, b, M=M)
    np.testing.assert_allclose(g, yv, atol=2 * slack, rtol=0)
