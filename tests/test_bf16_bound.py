"""Error bound behind the BF16 candidate filter (CPU, no GPU code runs).

The BF16 l2 path computes, per (query a, datum b), L = (1 - cE)(|a|^2 +
|b|^2) - 2 sum bf16(a_i) bf16(b_i) with the norms split into three BF16
pieces, and treats L as a lower bound of the exact squared distance S.  This
test evaluates that expression exactly (float64 sums of BF16 products, which
are exact) on random and adversarial vectors and checks that
    S - L >= (cE - 2^-7 - 2^-16 - 2^-20) (|a|^2 + |b|^2) > 0,
i.e. the BF16 rounding of the cross term stays within the (2^-7 + 2^-16)
share of cE, leaving the margin for FP32 accumulation and the norms.
"""
import numpy as np

CE = 2.0 ** -7 + 2.0 ** -11


def bf16(v):
    """Round-to-nearest-even to BF16 (the device's bit formula), as float64."""
    b = np.asarray(v, np.float32).view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def split3(v):
    v = np.float32(v)
    p1 = bf16(v)
    r1 = np.float32(v - np.float32(p1))
    p2 = bf16(r1)
    r2 = np.float32(r1 - np.float32(p2))
    p3 = bf16(r2)
    return p1 + p2 + p3


def lower_bound(a, b):
    a = np.asarray(a, np.float32)
    b = np.asarray(b, np.float32)
    nq = np.float32(0.0)
    nx = np.float32(0.0)
    for i in range(a.size):  # FP32 sums of squares (order immaterial to the bound)
        nq = np.float32(nq + np.float32(a[i] * a[i]))
        nx = np.float32(nx + np.float32(b[i] * b[i]))
    one_m = np.float32(1.0 - CE)
    m = split3(np.float32(nq * one_m))
    n = split3(np.float32(nx * one_m))
    cross = float(np.sum(bf16(a) * (-2.0 * bf16(b))))
    return m + n + cross


def exact(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(((a - b) ** 2).sum()), float((a ** 2).sum() + (b ** 2).sum())


def _check(a, b):
    L = lower_bound(a, b)
    S, nn = exact(a, b)
    margin = CE - 2.0 ** -7 - 2.0 ** -16 - 2.0 ** -20
    assert S - L >= margin * nn * (1 - 1e-9), (S, L, nn)
    return (S - L) / nn


def test_random_vectors():
    rng = np.random.default_rng(1)
    worst = 1.0
    for d in (1, 2, 4, 8, 16):
        for _ in range(400):
            scale = 10.0 ** rng.uniform(-15, 14)  # squares stay normal and below 2^100
            a = (rng.standard_normal(d) * scale).astype(np.float32)
            b = (a + rng.standard_normal(d) * scale * 10.0 ** rng.uniform(-6, 0)).astype(np.float32)
            worst = min(worst, _check(a, b))
    assert worst >= CE - 2.0 ** -7 - 2.0 ** -16 - 2.0 ** -20


def test_adversarial_rounding():
    """Components just above a BF16 rounding midpoint (relative error close
    to 2^-8 in each factor, same sign so the errors add up), a = b (S = 0)
    and a = -b."""
    d = 16
    base = np.float32(1.0 + 2.0 ** -8 - 2.0 ** -23)  # rounds down by ~2^-8
    a = np.full(d, base, np.float32)
    _check(a, a)
    _check(a, -a)
    _check(a, a * np.float32(1.0000001))
    up = np.float32(1.0 + 2.0 ** -8 + 2.0 ** -22)     # rounds up by ~2^-8
    _check(np.full(d, up, np.float32), np.full(d, up, np.float32))
    _check(np.full(d, base, np.float32), np.full(d, up, np.float32))


def test_query_equals_datum_is_candidate():
    """S = 0 gives L < 0, so a datum at the query always passes the test
    L <= r|r| + 2^-100 whenever r >= 0."""
    rng = np.random.default_rng(5)
    for _ in range(200):
        a = rng.standard_normal(16).astype(np.float32)
        assert lower_bound(a, a) < 0.0
