"""FP64 CPU oracle for the all-pairs Lipschitz bound evaluation.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product library never imports,
links or runs anything here, and nothing here imports the product.

The arithmetic lives in ``lipfit_oracle.c`` (plain C, double precision,
OpenMP over queries/rows), written from the paper's definitions:
  * bounds / interpolant:   Eq. (2), Eq. (3), directional distance Eq. (4)
  * consistency check:      the Lipschitz condition of Sec. 1 in the pairwise
                            form of Eqs. (5)-(6) with zero corrections
  * global constant:        Sec. 5 (``lipschitz_constant``), max pairwise slope
  * per-point constants:    Sec. 4.3, scalar form over the 16 nearest data
  * subgradients:           chain rule through the selected data points
  * step-function M_k(t):   Sec. 4.3, quantile knots from sampled distances,
                            per-datum tables, bounds with M_k(dist)
  * smoothing penalty:      Sec. 4.4, Eq. (7) and its gradient
  * k best bounds:          Sec. 5 (k > 1 with weights)
  * regional monotonicity:  Sec. 4.2 (cases I-IV on [a_i, b_i])
This module only marshals numpy arrays into that library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lipfit_oracle.c")
_LIB = os.path.join(_HERE, "liblipfit_oracle.so")

L1, L2, LINF = 1, 2, 3


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-std=c99", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, f64 = ctypes.c_int, ctypes.c_long, ctypes.c_double
        lib.orc_num_threads.restype = i32
        lib.orc_bounds.argtypes = [i32, i32, P, P, P, P, i64, f64, P, P, i64, P, P, P, P, P]
        lib.orc_bounds.restype = None
        lib.orc_candidates.argtypes = [i32, i32, P, P, P, P, i64, f64, P, P, P, P]
        lib.orc_candidates.restype = None
        lib.orc_consistency.argtypes = [i32, i32, P, P, P, P, i64, f64, P, f64, P, i64,
                                        P, P, P, P, P, P]
        lib.orc_consistency.restype = None
        lib.orc_estimate_M_global.argtypes = [i32, i32, P, P, P, i64, P, P]
        lib.orc_estimate_M_global.restype = i32
        lib.orc_estimate_M_knn.argtypes = [i32, i32, P, P, P, i64, i32, P, i64, P, P]
        lib.orc_estimate_M_knn.restype = i32
        lib.orc_grad.argtypes = [i32, i32, P, P, P, P, i64, f64, P, P, i64, P, P, P, P, P,
                                 P, P, P]
        lib.orc_grad.restype = None
        lib.orc_knots.argtypes = [i32, i32, P, P, P, i64, P, i32, P]
        lib.orc_knots.restype = None
        lib.orc_local_steps.argtypes = [i32, i32, P, P, P, i64, P, i32, P, i64, P, P]
        lib.orc_local_steps.restype = i32
        lib.orc_bounds_step.argtypes = [i32, i32, P, P, P, P, i64, P, i32, P, P, P, i64,
                                        P, P, P, P, P]
        lib.orc_bounds_step.restype = None
        lib.orc_candidates_step.argtypes = [i32, i32, P, P, P, P, i64, P, i32, P, P, P, P, P]
        lib.orc_candidates_step.restype = None
        lib.orc_smooth.argtypes = [i32, i32, P, P, P, P, i64, f64, P, P, f64, f64, P, P]
        lib.orc_smooth.restype = None
        lib.orc_smooth_scale.argtypes = [i32, i32, P, P, P, P, i64, f64, P, P, f64, f64, P, P, P]
        lib.orc_smooth_scale.restype = None
        lib.orc_bounds_k.argtypes = [i32, i32, P, P, P, P, i64, f64, P, i32, P, P, i64, P, P, P]
        lib.orc_bounds_k.restype = None
        lib.orc_bounds_reg.argtypes = [i32, i32, P, P, P, P, P, P, i64, f64, P, P, i64, P, P, P,
                                       P, P]
        lib.orc_bounds_reg.restype = None
        lib.orc_candidates_reg.argtypes = [i32, i32, P, P, P, P, P, P, i64, f64, P, P, P, P]
        lib.orc_candidates_reg.restype = None
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().orc_num_threads())


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def _common(x, y, w, mon, d):
    x = _f32(x)
    y = _f32(y)
    assert x.ndim == 2 and x.shape[1] == d and y.shape == (x.shape[0],)
    w = np.ones(d, np.float64) if w is None else np.ascontiguousarray(w, np.float64)
    mon = None if mon is None else np.ascontiguousarray(mon, np.int8)
    return x, y, w, mon


def bounds(x, y, xq, norm: int, M: float = 0.0, Mk=None, mon=None, w=None):
    """H_up, H_lo, g (float64) and arg_up, arg_lo (int64) for every query."""
    d = int(np.shape(x)[1])
    x, y, w, mon = _common(x, y, w, mon, d)
    xq = _f32(xq).reshape(-1, d)
    Mk = None if Mk is None else _f32(Mk)
    q = xq.shape[0]
    hu, hl, g = (np.empty(q, np.float64) for _ in range(3))
    au, al = np.empty(q, np.int64), np.empty(q, np.int64)
    _load().orc_bounds(d, norm, _p(w), _p(mon), _p(x), _p(y), x.shape[0], float(M), _p(Mk),
                       _p(xq), q, _p(hu), _p(hl), _p(g), _p(au), _p(al))
    return hu, hl, g, au, al


def candidates(x, y, xq1, norm: int, M: float = 0.0, Mk=None, mon=None, w=None):
    """(u[n], l[n]) float64: every bound candidate of Eq. (2) for one query."""
    d = int(np.shape(x)[1])
    x, y, w, mon = _common(x, y, w, mon, d)
    q1 = _f32(xq1).reshape(d)
    Mk = None if Mk is None else _f32(Mk)
    u, l = np.empty(x.shape[0], np.float64), np.empty(x.shape[0], np.float64)
    _load().orc_candidates(d, norm, _p(w), _p(mon), _p(x), _p(y), x.shape[0], float(M), _p(Mk),
                           _p(q1), _p(u), _p(l))
    return u, l


def consistency(x, y, norm: int, M: float = 0.0, Mk=None, mon=None, w=None, tol: float = 0.0,
                rows: Optional[Sequence[int]] = None):
    """Per-row slacks, partners and violation counts (see lipfit_oracle.c)."""
    d = int(np.shape(x)[1])
    x, y, w, mon = _common(x, y, w, mon, d)
    Mk = None if Mk is None else _f32(Mk)
    rows_a = None if rows is None else np.ascontiguousarray(rows, np.int64)
    nr = x.shape[0] if rows_a is None else rows_a.shape[0]
    su, sl = np.empty(nr, np.float64), np.empty(nr, np.float64)
    pu, pl, vu, vl = (np.empty(nr, np.int64) for _ in range(4))
    _load().orc_consistency(d, norm, _p(w), _p(mon), _p(x), _p(y), x.shape[0], float(M), _p(Mk),
                            float(tol), _p(rows_a), nr, _p(su), _p(sl), _p(pu), _p(pl),
                            _p(vu), _p(vl))
    # the smallest of all slack terms over the rows checked, with its ordered
    # pair (row i, partner k), lowest i then lowest k on ties; no pair: inf
    ri = np.arange(x.shape[0]) if rows_a is None else rows_a
    v, i, k = np.concatenate([su, sl]), np.concatenate([ri, ri]), np.concatenate([pu, pl])
    has = k >= 0
    best = (np.inf, -1, -1)
    if has.any():
        v, i, k = v[has], i[has], k[has]
        j = np.lexsort((k, i, v))[0]
        best = (float(v[j]), int(i[j]), int(k[j]))
    return dict(slack_up=su, slack_lo=sl, partner_up=pu, partner_lo=pl, viol_up=vu, viol_lo=vl,
                worst_slack=best[0], worst_pair=(best[1], best[2]))


def estimate_M_global(x, y, norm: int, w=None):
    """(status, M, (i, k)): max pairwise slope with the symmetric distance."""
    d = int(np.shape(x)[1])
    x, y, w, _ = _common(x, y, w, None, d)
    M = np.zeros(1, np.float64)
    pair = np.full(2, -1, np.int64)
    st = _load().orc_estimate_M_global(d, norm, _p(w), _p(x), _p(y), x.shape[0], _p(M), _p(pair))
    return int(st), float(M[0]), (int(pair[0]), int(pair[1]))


def estimate_M_knn(x, y, norm: int, K: int = 16, w=None, rows: Optional[Sequence[int]] = None):
    """(status, M_i[float64], neighbours[rows, K]) for the requested rows."""
    d = int(np.shape(x)[1])
    x, y, w, _ = _common(x, y, w, None, d)
    rows_a = None if rows is None else np.ascontiguousarray(rows, np.int64)
    nr = x.shape[0] if rows_a is None else rows_a.shape[0]
    M = np.empty(nr, np.float64)
    nbr = np.empty((nr, K), np.int64)
    st = _load().orc_estimate_M_knn(d, norm, _p(w), _p(x), _p(y), x.shape[0], int(K),
                                    _p(rows_a), nr, _p(M), _p(nbr))
    return int(st), M, nbr


def grad(x, y, xq, norm: int, arg_up, arg_lo, dg=None, dh_up=None, dh_lo=None,
         M: float = 0.0, Mk=None, mon=None, w=None):
    """(dxq[q, d], dy[n], dM[1] or [n]) in float64 at the given indices."""
    d = int(np.shape(x)[1])
    x, y, w, mon = _common(x, y, w, mon, d)
    xq = _f32(xq).reshape(-1, d)
    Mk = None if Mk is None else _f32(Mk)
    n, q = x.shape[0], xq.shape[0]
    au = np.ascontiguousarray(arg_up, np.int64)
    al = np.ascontiguousarray(arg_lo, np.int64)
    f64 = lambda a: None if a is None else np.ascontiguousarray(a, np.float64)
    dg, dh_up, dh_lo = f64(dg), f64(dh_up), f64(dh_lo)
    dxq = np.zeros((q, d), np.float64)
    dy = np.zeros(n, np.float64)
    dM = np.zeros(n if Mk is not None else 1, np.float64)
    _load().orc_grad(d, norm, _p(w), _p(mon), _p(x), _p(y), n, float(M), _p(Mk), _p(xq), q,
                     _p(au), _p(al), _p(dg), _p(dh_up), _p(dh_lo), _p(dxq), _p(dy), _p(dM))
    return dxq, dy, dM


def knots(x, pairs, probs, norm: int, w=None):
    """Quantile knots (float64[K]) of the sampled inter-point distances."""
    d = int(np.shape(x)[1])
    x = _f32(x)
    w = np.ones(d, np.float64) if w is None else np.ascontiguousarray(w, np.float64)
    pr = np.ascontiguousarray(pairs, np.int64).reshape(-1, 2)
    pb = np.ascontiguousarray(probs, np.float64)
    out = np.empty(pb.shape[0], np.float64)
    _load().orc_knots(d, norm, _p(w), _p(x), _p(pr), pr.shape[0], _p(pb), pb.shape[0], _p(out))
    return out


def local_steps(x, y, knots_, norm: int, w=None, rows: Optional[Sequence[int]] = None):
    """(status, d1[rows] float64, V[rows, K+2] float64): step tables of Sec. 4.3."""
    d = int(np.shape(x)[1])
    x, y, w, _ = _common(x, y, w, None, d)
    kn = np.ascontiguousarray(knots_, np.float64)
    K = kn.shape[0]
    rows_a = None if rows is None else np.ascontiguousarray(rows, np.int64)
    nr = x.shape[0] if rows_a is None else rows_a.shape[0]
    d1 = np.empty(nr, np.float64)
    V = np.empty((nr, K + 2), np.float64)
    st = _load().orc_local_steps(d, norm, _p(w), _p(x), _p(y), x.shape[0], _p(kn), K,
                                 _p(rows_a), nr, _p(d1), _p(V))
    return int(st), d1, V


def bounds_step(x, y, xq, norm: int, knots_, d1, V32, mon=None, w=None):
    """H_up, H_lo, g (float64), arg_up, arg_lo (int64) with M_k(dist) from the tables."""
    d = int(np.shape(x)[1])
    x, y, w, mon = _common(x, y, w, mon, d)
    xq = _f32(xq).reshape(-1, d)
    kn = np.ascontiguousarray(knots_, np.float64)
    d1 = np.ascontiguousarray(d1, np.float64)
    V32 = _f32(V32)
    assert V32.shape == (x.shape[0], kn.shape[0] + 2)
    q = xq.shape[0]
    hu, hl, g = (np.empty(q, np.float64) for _ in range(3))
    au, al = np.empty(q, np.int64), np.empty(q, np.int64)
    _load().orc_bounds_step(d, norm, _p(w), _p(mon), _p(x), _p(y), x.shape[0], _p(kn),
                            kn.shape[0], _p(d1), _p(V32), _p(xq), q, _p(hu), _p(hl), _p(g),
                            _p(au), _p(al))
    return hu, hl, g, au, al


def candidates_step(x, y, xq1, norm: int, knots_, d1, V32, mon=None, w=None):
    """(u[n], l[n]) float64 for one query with M_k(dist) from the tables."""
    d = int(np.shape(x)[1])
    x, y, w, mon = _common(x, y, w, mon, d)
    q1 = _f32(xq1).reshape(d)
    kn = np.ascontiguousarray(knots_, np.float64)
    d1 = np.ascontiguousarray(d1, np.float64)
    V32 = _f32(V32)
    n = x.shape[0]
    u, l = np.empty(n, np.float64), np.empty(n, np.float64)
    _load().orc_candidates_step(d, norm, _p(w), _p(mon), _p(x), _p(y), n, _p(kn), kn.shape[0],
                                _p(d1), _p(V32), _p(q1), _p(u), _p(l))
    return u, l


def smooth(x, y, eps, norm: int, M: float = 0.0, Mk=None, p: float = 1.0, mon=None, w=None,
           prune: float = 0.0):
    """(F, grad[n]) float64: the penalty objective of Eq. (7) and its gradient at eps;
    prune > 0 drops the pairs of the Sec. 5 pre-screening with that fraction."""
    d = int(np.shape(x)[1])
    x, y, w, mon = _common(x, y, w, mon, d)
    Mk = None if Mk is None else _f32(Mk)
    e = np.ascontiguousarray(eps, np.float64)
    n = x.shape[0]
    assert e.shape == (n,)
    F = np.zeros(1, np.float64)
    g = np.empty(n, np.float64)
    _load().orc_smooth(d, norm, _p(w), _p(mon), _p(x), _p(y), n, float(M), _p(Mk), _p(e),
                       float(p), float(prune), _p(F), _p(g))
    return float(F[0]), g


def smooth_scale(x, y, eps, norm: int, tau: float, M: float = 0.0, Mk=None, mon=None, w=None,
                 prune: float = 0.0):
    """(A, row_abs[n], row_cnt[n]): error scale of Eq. (7) for comparisons."""
    d = int(np.shape(x)[1])
    x, y, w, mon = _common(x, y, w, mon, d)
    Mk = None if Mk is None else _f32(Mk)
    e = np.ascontiguousarray(eps, np.float64)
    n = x.shape[0]
    A = np.zeros(1, np.float64)
    ra = np.empty(n, np.float64)
    rc = np.empty(n, np.int64)
    _load().orc_smooth_scale(d, norm, _p(w), _p(mon), _p(x), _p(y), n, float(M), _p(Mk), _p(e),
                             float(prune), float(tau), _p(A), _p(ra), _p(rc))
    return float(A[0]), ra, rc


def bounds_k(x, y, xq, norm: int, wk, M: float = 0.0, Mk=None, mon=None, w=None):
    """(H_up, H_lo, g) float64: weighted sums of the k best candidates (k = len(wk))."""
    d = int(np.shape(x)[1])
    x, y, w, mon = _common(x, y, w, mon, d)
    xq = _f32(xq).reshape(-1, d)
    Mk = None if Mk is None else _f32(Mk)
    wk = np.ascontiguousarray(wk, np.float64)
    assert 1 <= wk.shape[0] <= x.shape[0]
    q = xq.shape[0]
    hu, hl, g = (np.empty(q, np.float64) for _ in range(3))
    _load().orc_bounds_k(d, norm, _p(w), _p(mon), _p(x), _p(y), x.shape[0], float(M), _p(Mk),
                         wk.shape[0], _p(wk), _p(xq), q, _p(hu), _p(hl), _p(g))
    return hu, hl, g


def _reg(kind, a, b, d):
    kind = np.ascontiguousarray(kind, np.int8)
    a = np.zeros(d) if a is None else np.ascontiguousarray(a, np.float64)
    b = np.zeros(d) if b is None else np.ascontiguousarray(b, np.float64)
    assert kind.shape == a.shape == b.shape == (d,)
    return kind, a, b


def bounds_reg(x, y, xq, norm: int, kind, a=None, b=None, M: float = 0.0, Mk=None, w=None):
    """H_up, H_lo, g, arg_up, arg_lo with monotonicity on parts of the domain:
    kind per coordinate 0 / +1 / -1 / 2..5 (cases I..IV on [a_i, b_i])."""
    d = int(np.shape(x)[1])
    x, y, w, _ = _common(x, y, w, None, d)
    kind, a, b = _reg(kind, a, b, d)
    xq = _f32(xq).reshape(-1, d)
    Mk = None if Mk is None else _f32(Mk)
    q = xq.shape[0]
    hu, hl, g = (np.empty(q, np.float64) for _ in range(3))
    au, al = np.empty(q, np.int64), np.empty(q, np.int64)
    _load().orc_bounds_reg(d, norm, _p(w), _p(kind), _p(a), _p(b), _p(x), _p(y), x.shape[0],
                           float(M), _p(Mk), _p(xq), q, _p(hu), _p(hl), _p(g), _p(au), _p(al))
    return hu, hl, g, au, al


def candidates_reg(x, y, xq1, norm: int, kind, a=None, b=None, M: float = 0.0, Mk=None, w=None):
    d = int(np.shape(x)[1])
    x, y, w, _ = _common(x, y, w, None, d)
    kind, a, b = _reg(kind, a, b, d)
    q1 = _f32(xq1).reshape(d)
    Mk = None if Mk is None else _f32(Mk)
    n = x.shape[0]
    u, l = np.empty(n, np.float64), np.empty(n, np.float64)
    _load().orc_candidates_reg(d, norm, _p(w), _p(kind), _p(a), _p(b), _p(x), _p(y), n,
                               float(M), _p(Mk), _p(q1), _p(u), _p(l))
    return u, l


def round_up_f32(v) -> np.ndarray:
    """float64 -> float32 rounded toward +inf (the constants the bounds multiply)."""
    v = np.asarray(v, np.float64)
    f = v.astype(np.float32)
    low = f.astype(np.float64) < v
    f[low] = np.nextafter(f[low], np.float32(np.inf))
    return f
