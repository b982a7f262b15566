"""Seeded synthetic inputs shaped like the paper's scattered-data problems.

This module only draws random numbers and evaluates the test functions that
generate the data (y = f(x) + noise).  It holds none of the method's
arithmetic (no distances, no bounds, no Lipschitz estimates), so both the
oracle-side tests and the GPU-side tests and benchmark can share it.

All arrays are generated in float64 and handed out as float32 (x, y, M, xq),
which is the precision both the GPU path and the oracle read.

Random streams: ``numpy.random.Generator(PCG64(SeedSequence([260604670, c, ...])))``
with ``c`` the workload number; draws happen in the order data points x,
model parameters, noise, query points.

Workloads (the problem is stated in Sec. 1 and 3 of the paper: data set
D = {(x^k, y^k)}, Lipschitz constant M, query points x):

1. ``plain_l2``      d=2,  N=1,000,  Q=10,000,   y = sin(3 x1) + x2 (Lipschitz
                     constant sqrt(10) < M = 4, so the data are consistent), l2.
2. ``monotone_local`` d=4, N=100,000, Q=1,000,000, y = x1 + 0.5 x3^2
                     + 0.3 sin(4 x2) + 0.01 N(0,1), increasing in x1 and x3,
                     per-point M_k (estimated from 16 nearest pairs on the GPU
                     path; a seeded U[0.5, 2] array stands in where a fixed M_k
                     input is needed), l1 / l2 / linf.
3. ``diff_l2``       d=8, N=200,000, Q=262,144, x ~ N(0, I) clipped to [-3, 3],
                     y = tanh(w.x) + 0.05 N(0,1), M = 2, l2, upstream grads ~ N(0,1).
4. ``batched``       512 sets, N log-uniform in [500, 50,000], d uniform in
                     {2..10}, x ~ U[0,1]^d, y = sum of monotone ramps, half the
                     coordinates increasing, Q = 4N, l2 with the ramps' exact
                     Lipschitz constant.
5. ``mixed_l2``      d=16, N=1,000,000, Q=1,000,000, x ~ N(0, I),
                     y = ||x||_1 / 16 + 0.01 N(0,1), M = 1, l2.

Each generator takes optional ``n`` / ``q`` overrides so that tests can draw the
same distributions at sizes the oracle finishes in seconds.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

SEED_ROOT = 260604670

NORM_L1, NORM_L2, NORM_LINF = 1, 2, 3
NORM_NAMES = {NORM_L1: "l1", NORM_L2: "l2", NORM_LINF: "linf"}


def rng_for(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, *key])))


@dataclasses.dataclass
class Problem:
    """One scattered-data problem: data (x, y), Lipschitz data and queries."""
    name: str
    x: np.ndarray            # [n, d] float32, row-major
    y: np.ndarray            # [n] float32
    M: float                 # global Lipschitz constant (ignored when Mk is given)
    Mk: Optional[np.ndarray]  # [n] float32 per-point constants, or None
    xq: np.ndarray           # [q, d] float32
    norm: int
    mon: np.ndarray          # [d] int8 in {-1, 0, 1}
    w: np.ndarray            # [d] float32 > 0 (distance weights)
    dg: Optional[np.ndarray] = None  # [q] float32 upstream gradient for g

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def q(self) -> int:
        return int(self.xq.shape[0])

    @property
    def d(self) -> int:
        return int(self.x.shape[1])


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def plain_l2(n: int = 1000, q: int = 10_000) -> Problem:
    g = rng_for(1)
    x = _f32(g.random((n, 2)))
    xd = x.astype(np.float64)
    y = _f32(np.sin(3.0 * xd[:, 0]) + xd[:, 1])
    xq = _f32(g.random((q, 2)))
    return Problem("plain_l2", x, y, 4.0, None, xq, NORM_L2,
                   np.zeros(2, np.int8), np.ones(2, np.float32))


def monotone_local(n: int = 100_000, q: int = 1_000_000, norm: int = NORM_L1) -> Problem:
    g = rng_for(2)
    x = _f32(g.random((n, 4)))
    xd = x.astype(np.float64)
    noise = g.standard_normal(n)
    y = _f32(xd[:, 0] + 0.5 * xd[:, 2] ** 2 + 0.3 * np.sin(4.0 * xd[:, 1]) + 0.01 * noise)
    xq = _f32(g.random((q, 4)))
    # Stand-in per-point constants for tests that need M_k fixed in advance.
    mk = _f32(0.5 + 1.5 * rng_for(2, 1).random(n))
    mon = np.array([1, 0, 1, 0], np.int8)
    return Problem("monotone_local", x, y, 0.0, mk, xq, norm, mon, np.ones(4, np.float32))


def diff_l2(n: int = 200_000, q: int = 262_144) -> Problem:
    g = rng_for(3)
    x = _f32(np.clip(g.standard_normal((n, 8)), -3.0, 3.0))
    wv = g.standard_normal(8) / math.sqrt(8.0)
    noise = g.standard_normal(n)
    y = _f32(np.tanh(x.astype(np.float64) @ wv) + 0.05 * noise)
    xq = _f32(np.clip(g.standard_normal((q, 8)), -3.0, 3.0))
    dg = _f32(rng_for(3, 1).standard_normal(q))
    return Problem("diff_l2", x, y, 2.0, None, xq, NORM_L2,
                   np.zeros(8, np.int8), np.ones(8, np.float32), dg)


def mixed_l2(n: int = 1_000_000, q: int = 1_000_000) -> Problem:
    g = rng_for(5)
    x = _f32(g.standard_normal((n, 16)))
    noise = g.standard_normal(n)
    y = _f32(np.abs(x.astype(np.float64)).sum(axis=1) / 16.0 + 0.01 * noise)
    xq = _f32(g.standard_normal((q, 16)))
    return Problem("mixed_l2", x, y, 1.0, None, xq, NORM_L2,
                   np.zeros(16, np.int8), np.ones(16, np.float32))


def batched(n_sets: int = 512, n_lo: int = 500, n_hi: int = 50_000, q_factor: int = 4,
            norm: int = NORM_L2, n_scale: float = 1.0) -> List[Problem]:
    """Independent data sets of uneven size and dimension.

    ``n_scale`` shrinks every N (and hence Q) for tests while keeping the mix.
    """
    top = rng_for(4)
    ns = np.rint(np.exp(top.uniform(math.log(n_lo), math.log(n_hi), n_sets))).astype(np.int64)
    ds = top.integers(2, 11, n_sets)
    out = []
    for s in range(n_sets):
        n = max(1, int(round(ns[s] * n_scale)))
        d = int(ds[s])
        g = rng_for(4, 1, s)
        x = _f32(g.random((n, d)))
        a = g.uniform(0.2, 1.0, d)
        c = g.uniform(0.0, 0.8, d)
        sl = g.uniform(0.1, 0.5, d)
        mon_idx = g.permutation(d)[: d // 2]
        xd = x.astype(np.float64)
        y = _f32((a * np.clip((xd - c) / sl, 0.0, 1.0)).sum(axis=1))
        xq = _f32(g.random((q_factor * n, d)))
        mon = np.zeros(d, np.int8)
        mon[mon_idx] = 1
        slopes = a / sl
        # Lipschitz constant of the ramp sum for the chosen norm (dual norm of
        # the slope vector): l2 -> ||.||_2, l1 -> ||.||_inf, linf -> ||.||_1.
        if norm == NORM_L2:
            M = float(np.sqrt((slopes ** 2).sum()))
        elif norm == NORM_L1:
            M = float(slopes.max())
        else:
            M = float(slopes.sum())
        # round the constant up to float32 so the data stay consistent
        M32 = np.float32(M)
        if float(M32) < M:
            M32 = np.nextafter(M32, np.float32(np.inf))
        out.append(Problem(f"batched[{s}]", x, y, float(M32), None, xq, norm, mon,
                           np.ones(d, np.float32)))
    return out


def random_problem(seed: int, n: int, q: int, d: int, norm: int, mon=None,
                   local: bool = False, weighted: bool = False,
                   M: float = 1.5) -> Problem:
    """Generic random problem for edge-case tests (uniform x, smooth y + noise)."""
    g = rng_for(100, seed)
    x = _f32(g.random((n, d)))
    coef = g.standard_normal(d)
    noise = g.standard_normal(n)
    y = _f32(np.sin(x.astype(np.float64) @ coef) + 0.05 * noise)
    xq = _f32(g.uniform(-0.1, 1.1, (q, d)))
    mk = _f32(0.25 + 2.0 * g.random(n)) if local else None
    w = _f32(0.5 + g.random(d)) if weighted else np.ones(d, np.float32)
    if mon is None:
        mon = np.zeros(d, np.int8)
    dg = _f32(g.standard_normal(q))
    return Problem(f"random[{seed}]", x, y, M, mk, xq, norm, np.asarray(mon, np.int8), w, dg)
