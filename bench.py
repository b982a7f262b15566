"""Benchmark of the all-pairs Lipschitz bound path on one MI355X.

Workload (monotone local-Lipschitz fit): d = 4, N = 100,000 data points
x ~ U[0,1]^4, y = x1 + 0.5 x3^2 + 0.3 sin(4 x2) + 0.01 N(0,1), increasing in
coordinates 1 and 3, Q = 1,000,000 queries ~ U[0,1]^4, for each of the l1,
l2 and linf distances.  One step runs, per norm, the whole path on inputs
already resident in HBM:
    per-point M_k from the 16 nearest data (FP64)  -> lip_estimate_M
    pairwise consistency check with those M_k (FP64) -> lip_consistency
    forward: H_up, H_lo, g and attaining indices     -> lip_fit_eval
    backward: d/dxq, d/dy, d/dM_k for upstream dg     -> lip_fit_backward
value = 3 * Q * N query x data pair evaluations / mean step time.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("query×data pair-evals/s (d=4, N=1e5, Q=1e6) fwd and fwd+bwd; % VALU peak")

# MI355X: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz -> VALU lane-operations/s.
VALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9
FP32_DATASHEET_TFLOPS = 157.3

# Minimal VALU instructions per (query, datum) pair of the fused bound kernel
# for d = 4 with 2 monotone coordinates (derivation in the design notes):
# coordinate differences / maxima, accumulation, two FMAs for the bounds and
# one min3/max3 per pair for the running min and max.
ALG_OPS_PER_PAIR = {"l1": 11, "l2": 19, "linf": 10}
# Conventional FLOP per pair (each add/sub/min/max/abs-accumulate 1, FMA 2,
# sqrt 1) used for the datasheet comparison.
FLOP_PER_PAIR = {"l1": 16, "l2": 24, "linf": 16}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-queries", type=int, default=8192,
                    help="queries per norm in the oracle's CPU-baseline sample")
    ap.add_argument("--norms", default="l1,l2,linf")
    return ap.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (this build targets a single MI355X); "
              f"--gpus {a.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2606_04670_amd as lf
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    lf.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    norms = a.norms.split(",")
    nid = {"l1": 1, "l2": 2, "linf": 3}

    base = W.monotone_local()
    N, Q, D = base.n, base.q, base.d
    x = torch.from_numpy(base.x).to(dev)
    y = torch.from_numpy(base.y).to(dev)
    xq = torch.from_numpy(base.xq).to(dev)
    dg = torch.from_numpy(np.random.default_rng(7).standard_normal(Q).astype(np.float32)).to(dev)
    mets = {nm: lf.Metric(D, nm, mon=base.mon) for nm in norms}
    stages = ("knn", "consistency", "forward", "backward")

    def one_step(ev=None):
        for nm in norms:
            met = mets[nm]
            e = None if ev is None else ev[nm]
            if e: e["knn"][0].record()
            _, Mk, _ = lf.estimate_M(x, y, met, mode="knn", knn=16)
            if e: e["knn"][1].record(); e["consistency"][0].record()
            lf.consistency(x, y, met, Mk=Mk, per_row=False)
            if e: e["consistency"][1].record(); e["forward"][0].record()
            out = lf.fit_eval(x, y, xq, met, Mk=Mk)
            if e: e["forward"][1].record(); e["backward"][0].record()
            lf.backward(x, y, xq, met, out["arg_up"], out["arg_lo"], dg=dg, Mk=Mk)
            if e: e["backward"][1].record()

    for _ in range(a.warmup):
        one_step()
    torch.cuda.synchronize()

    # timed region: K whole steps; HIP events on the launch stream bracket
    # every stage of every step
    evs = [{nm: {s: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                 for s in stages} for nm in norms} for _ in range(a.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(a.steps):
        one_step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / a.steps
    stage_ms = {nm: {s: float(np.mean([evs[k][nm][s][0].elapsed_time(evs[k][nm][s][1])
                                        for k in range(a.steps)])) for s in stages}
                for nm in norms}

    pairs = float(N) * float(Q)
    value = len(norms) * pairs / (ms_step * 1e-3)
    per_norm = {}
    for nm in norms:
        f = stage_ms[nm]["forward"]
        b = stage_ms[nm]["backward"]
        per_norm[nm] = {
            "fwd_pair_evals_per_s": pairs / (f * 1e-3),
            "fwd_bwd_pair_evals_per_s": pairs / ((f + b) * 1e-3),
            "fwd_ms": f, "bwd_ms": b,
            "knn16_ms": stage_ms[nm]["knn"], "consistency_fp64_ms": stage_ms[nm]["consistency"],
            "valu_frac": ALG_OPS_PER_PAIR[nm] * pairs / (f * 1e-3) / VALU_PEAK_OPS,
            "datasheet_fp32_frac": FLOP_PER_PAIR[nm] * pairs / (f * 1e-3) / 1e12
            / FP32_DATASHEET_TFLOPS,
        }
    # dominant kernel: the forward bound kernel of the slowest norm
    dom = max(norms, key=lambda nm: stage_ms[nm]["forward"])
    f_ms = stage_ms[dom]["forward"]
    achieved = ALG_OPS_PER_PAIR[dom] * pairs / (f_ms * 1e-3) / 1e12
    peak = VALU_PEAK_OPS / 1e12
    roofline = {"bound": "alu", "kernel": f"bounds_fwd_kernel<4,2,{nid[dom]}> ({dom})",
                "achieved": round(achieved, 3), "peak": round(peak, 3), "unit": "Tops/s",
                "frac": round(achieved / peak, 4), "traffic": None,
                "ops_per_pair": ALG_OPS_PER_PAIR[dom]}

    cpu = None
    if not a.no_cpu_baseline:
        import oracle
        qs = min(a.cpu_queries, Q)
        sel = np.random.default_rng(11).choice(Q, qs, replace=False)
        xs = base.xq[sel]
        tc0 = time.perf_counter()
        for nm in norms:
            oracle.bounds(base.x, base.y, xs, nid[nm], Mk=base.Mk, mon=base.mon)
        tc1 = time.perf_counter()
        cpu = {"value": len(norms) * qs * float(N) / (tc1 - tc0), "unit": "pair-evals/s",
               "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"forward bounds (FP64) of {qs} seeded queries x all {N} data, "
                         f"norms {'/'.join(norms)}, {tc1 - tc0:.1f} s"}

    rec = {
        "metric": METRIC, "value": value, "unit": "pair-evals/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "monotone_local", "d": D, "N": N, "Q": Q, "norms": norms,
                   "monotone": "increasing in coordinates 1 and 3", "M": "per-point, kNN-16",
                   "step": "per norm: kNN-16 M_k (f64) + consistency (f64) + forward (f32) "
                           "+ backward (f32)", "parallelism": "single GPU"},
        "per_norm": per_norm, "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
