"""Comparison rules between the GPU path and the FP64 oracle.

Values: |v_gpu - v_orc| <= 1e-5 * max(|v_orc|, max|y|)  (1e-5 relative, with
the data scale standing in where the value itself is near 0).

Indices: equal to the oracle's wherever the FP64 winner is clear of every
other candidate by more than tau, the a-priori FP32 error bound of one
candidate; otherwise the GPU's index must be a member of the oracle's tau-tie
set {k : u_k <= H_up + tau} (resp. l_k >= H_lo - tau).  tau = 4 gamma_{d+8}
(max|y| + max M * D_max), gamma_n = n u / (1 - n u), u = 2^-24, D_max the
largest query-datum distance (bounded by the box that holds both).
"""
from __future__ import annotations

import numpy as np

import oracle

U32 = 2.0 ** -24
REL = 1e-5


def tau_for(p, Mk=None) -> float:
    d = p.d
    n_ops = d + 8
    gam = n_ops * U32 / (1 - n_ops * U32)
    lo = np.minimum(p.x.min(0), p.xq.min(0)).astype(np.float64)
    hi = np.maximum(p.x.max(0), p.xq.max(0)).astype(np.float64)
    w = p.w.astype(np.float64)
    span = (hi - lo) * w
    dmax = {1: span.sum(), 2: np.sqrt((span ** 2).sum()), 3: span.max()}[p.norm]
    mmax = float(np.max(Mk)) if Mk is not None else float(p.M)
    ymax = float(np.abs(p.y).max())
    return 4.0 * gam * (ymax + mmax * dmax)


def value_ok(gpu, orc, yscale):
    gpu = np.asarray(gpu, np.float64)
    orc = np.asarray(orc, np.float64)
    err = np.abs(gpu - orc)
    lim = REL * np.maximum(np.abs(orc), yscale)
    return err <= lim, err


def check_bounds(p, gpu: dict, qidx=None, Mk=None, label=""):
    """Compare GPU outputs (numpy dict) on queries qidx with the oracle.

    Returns a report dict (max errors, index mismatch counts)."""
    Mk = p.Mk if Mk is None else Mk
    qidx = np.arange(p.q) if qidx is None else np.asarray(qidx)
    orc = oracle.bounds(p.x, p.y, p.xq[qidx], p.norm, M=p.M, Mk=Mk, mon=p.mon, w=p.w)
    cand = lambda xq1: oracle.candidates(p.x, p.y, xq1, p.norm, M=p.M, Mk=Mk, mon=p.mon, w=p.w)
    return _compare(p, gpu, qidx, orc, cand, tau_for(p, Mk), label)


def check_bounds_steps(p, gpu: dict, knots, d1, V32, qidx=None, label=""):
    """As check_bounds, for the step-function constants (tau from the largest
    table entry)."""
    qidx = np.arange(p.q) if qidx is None else np.asarray(qidx)
    orc = oracle.bounds_step(p.x, p.y, p.xq[qidx], p.norm, knots, d1, V32, mon=p.mon, w=p.w)
    cand = lambda xq1: oracle.candidates_step(p.x, p.y, xq1, p.norm, knots, d1, V32, mon=p.mon,
                                              w=p.w)
    return _compare(p, gpu, qidx, orc, cand, tau_for(p, np.asarray(V32).reshape(-1)), label)


def check_bounds_regional(p, gpu: dict, kind, a, b, qidx=None, label=""):
    """As check_bounds, for monotonicity on parts of the domain."""
    qidx = np.arange(p.q) if qidx is None else np.asarray(qidx)
    orc = oracle.bounds_reg(p.x, p.y, p.xq[qidx], p.norm, kind, a, b, M=p.M, Mk=p.Mk, w=p.w)
    cand = lambda xq1: oracle.candidates_reg(p.x, p.y, xq1, p.norm, kind, a, b, M=p.M, Mk=p.Mk,
                                             w=p.w)
    return _compare(p, gpu, qidx, orc, cand, tau_for(p, p.Mk), label)


def _compare(p, gpu, qidx, orc, cand, tau, label):
    hu, hl, g, au, al = orc
    xq = p.xq[qidx]
    yscale = float(np.abs(p.y).max())
    rep = {"label": label, "queries": len(qidx)}
    for name, ov in (("h_up", hu), ("h_lo", hl), ("g", g)):
        if name not in gpu:
            continue
        ok, err = value_ok(gpu[name][qidx], ov, yscale)
        rep[f"max_abs_err_{name}"] = float(err.max()) if err.size else 0.0
        bad = np.nonzero(~ok)[0]
        assert bad.size == 0, (f"{label}: {name} off at {bad.size} queries, e.g. q={qidx[bad[0]]} "
                               f"gpu={gpu[name][qidx[bad[0]]]!r} oracle={ov[bad[0]]!r}")
    for name, orc_idx, orc_val, up in (("arg_up", au, hu, True), ("arg_lo", al, hl, False)):
        if name not in gpu:
            continue
        gi = gpu[name][qidx].astype(np.int64)
        assert np.all((gi >= 0) & (gi < p.n)), f"{label}: {name} out of range"
        mism = np.nonzero(gi != orc_idx)[0]
        for m in mism:
            u, l = cand(xq[m])
            if up:
                assert u[gi[m]] <= orc_val[m] + tau, (
                    f"{label}: {name} q={qidx[m]} gpu picks {gi[m]} (u={u[gi[m]]!r}), oracle "
                    f"{orc_idx[m]} (u={orc_val[m]!r}), tau={tau:g}")
            else:
                assert l[gi[m]] >= orc_val[m] - tau, (
                    f"{label}: {name} q={qidx[m]} gpu picks {gi[m]} (l={l[gi[m]]!r}), oracle "
                    f"{orc_idx[m]} (l={orc_val[m]!r}), tau={tau:g}")
        rep[f"{name}_near_tie"] = int(mism.size)
    return rep
