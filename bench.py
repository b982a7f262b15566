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

# MI355X: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz = VALU issue slots per
# second (one slot = one lane-operation at the base issue rate).
VALU_PEAK_SLOTS = 256 * 4 * 16 * 2.4e9
FP32_DATASHEET_TFLOPS = 157.3

# Issue cost of one instruction in slots, from the measured single-kind
# rates on this chip (profiles/valu_issue_rates_gfx950.txt): v_add/v_sub_f32
# issue at twice the base rate (~65 T lane-ops/s), v_sqrt_f32 at half
# (~19 T), FMA / mul / max / min / med3 / min3 / max3 at the base rate.
SLOT = {"add": 0.5, "fma": 1.0, "max": 1.0, "med3": 1.0, "minmax3": 1.0, "sqrt": 2.0}

# Minimal instruction mix per (query, datum) pair of the fused bound kernel,
# d = 4 with 2 monotone coordinates (derivation in the design notes):
MIX = {
    # 2 sub + 1 add(|a|,|b|) + 2 add + 1 sub; 2 med3; 2 FMA; min3/max3 per 2 pairs x 2 bounds
    "l1": {"add": 6, "med3": 2, "fma": 2, "minmax3": 1},
    # 4 sub; max + 2 max3; 2 FMA; min3/max3
    "linf": {"add": 4, "max": 3, "fma": 2, "minmax3": 1},
    # 4 sub; mul + FMA (free); 2 max + 2 min + 4 FMA (monotone); 2 sqrt; 2 FMA; min3/max3
    "l2": {"add": 4, "fma": 8, "max": 4, "sqrt": 2, "minmax3": 1},
}
SLOTS_PER_PAIR = {nm: sum(SLOT[c] * k for c, k in mix.items()) for nm, mix in MIX.items()}
INSTR_PER_PAIR = {nm: sum(mix.values()) for nm, mix in MIX.items()}
# Conventional FLOP per pair (each add/sub/min/max/abs-accumulate 1, FMA 2,
# sqrt 1) used for the datasheet comparison.
FLOP_PER_PAIR = {"l1": 16, "l2": 24, "linf": 16}
# Minimal instructions per ordered data pair of the consistency kernels at
# d = 4 with the monotone pattern known at compile time.  l1 / linf (FP64
# kernel, one slot each): 4 differences, 4 positive parts (the monotone
# coordinates), 3 + 3 accumulations, 2 x 3 for the bounds (mul, add, sub in
# the definition's order), 2 minima, 2 violation compares = 24.  l2 (FP32
# filter kernel, slots): 4 differences (2), 4 positive parts (4), 2 x (mul
# + 3 FMA) squares (8), 2 v_sqrt_f32 (4), 2 x (FMA + sub) bounds (3), 6
# compares (certain violation, tolerance band, running-minimum candidate for
# each bound) = 27; the rare FP64 re-evaluations come on top.
CONS_SLOTS_PER_PAIR = {"l1": 24, "linf": 24, "l2": 27}


# HBM traffic of the forward kernel, from rocprofv3 FETCH_SIZE / WRITE_SIZE
# runs scaled by a 1 GiB copy kernel (profiles/, with the command that made
# it).  Reported only while the kernel's sources are the ones profiled.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "bounds_fwd_monotone_local_traffic.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2606_04670_amd", "csrc", f)
                  for f in ("bounds_fwd.hpp", "lip_device.hpp", "lip_internal.hpp",
                            "bounds_fwd_l1.hip", "bounds_fwd_l2.hip", "bounds_fwd_linf.hip")]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(norm):
    """Bytes per launch of the forward kernel for `norm`, or None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            for line in fh:
                if line.startswith("TRAFFIC_JSON "):
                    rec = json.loads(line[len("TRAFFIC_JSON "):])
                    if rec.get("source_sha256") != kernel_source_hash():
                        return None
                    return rec["bytes_per_launch"].get(norm)
    except OSError:
        return None
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-queries", type=int, default=65536,
                    help="queries per norm in the oracle's CPU-baseline sample")
    ap.add_argument("--norms", default="l1,l2,linf")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the BF16-vs-FP32, batched-vs-per-set, step-function, "
                         "smoothing, k-best, regional-monotonicity and other-workload runs")
    return ap.parse_args()


def _time_ms(torch, fn, reps):
    """Mean time of fn() over reps runs (one untimed warm-up), HIP events on
    the current stream."""
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def extra_bf16(lf, W, torch, dev, reps=3):
    """l2, d = 16, N = Q = 1e6 (x ~ N(0, I), M = 1): BF16-MFMA filter + FP32
    re-scoring against the plain FP32 path, results compared for identity."""
    p = W.mixed_l2()
    x = torch.from_numpy(p.x).to(dev)
    y = torch.from_numpy(p.y).to(dev)
    xq = torch.from_numpy(p.xq).to(dev)
    met = lf.Metric(p.d, "l2")
    outs = {}

    def run(bf):
        outs[bf] = lf.fit_eval(x, y, xq, met, M=p.M, bf16=bf)

    t32 = _time_ms(torch, lambda: run(False), reps)
    t16 = _time_ms(torch, lambda: run(True), reps)
    same = all(torch.equal(outs[True][k], outs[False][k]) or
               bool(((outs[True][k] == outs[False][k]) |
                     (outs[True][k].isnan() & outs[False][k].isnan())).all())
               for k in outs[True])
    pairs = float(p.n) * float(p.q)
    ks = 1 if p.d + 6 <= 16 else 2
    mfma_flop_per_pair = 2 * 16 * ks  # one 32x32x16 BF16 MFMA per 1024 pairs per K-step
    rate16 = pairs / (t16 * 1e-3)
    return {"workload": f"mixed_l2 d={p.d} N={p.n} Q={p.q} M={p.M} l2",
            "fp32_ms": t32, "bf16_ms": t16, "speedup": t32 / t16,
            "fp32_pair_evals_per_s": pairs / (t32 * 1e-3), "bf16_pair_evals_per_s": rate16,
            "identical_to_fp32": bool(same),
            "bf16_mfma_issued_tflops": mfma_flop_per_pair * rate16 / 1e12,
            "bf16_mfma_frac_of_2500_tflops": mfma_flop_per_pair * rate16 / 2.5e15,
            "note": "bf16_ms includes the y sort and staging of the data (per call)"}


def extra_batched(lf, W, torch, dev, reps=3):
    """512 independent l2 sets (N log-uniform in [500, 50000], d in 2..10,
    Q = 4N): one graph launch of a plan against per-set lip_fit_eval calls."""
    probs = W.batched()
    sets = []
    for pb in probs:
        sets.append(dict(x=torch.from_numpy(pb.x).to(dev), y=torch.from_numpy(pb.y).to(dev),
                         xq=torch.from_numpy(pb.xq).to(dev),
                         metric=lf.Metric(pb.d, pb.norm, mon=pb.mon, w=pb.w), M=pb.M))
    plan = lf.Plan(sets)

    def per_set():
        for s_ in sets:
            lf.fit_eval(s_["x"], s_["y"], s_["xq"], s_["metric"], M=s_["M"])

    t_plan = _time_ms(torch, plan.execute, reps)
    t_sets = _time_ms(torch, per_set, reps)
    plan.close()
    pairs = float(sum(pb.n * pb.q for pb in probs))
    return {"workload": f"batched {len(probs)} sets, l2, sum N*Q = {pairs:.3e}",
            "plan_ms": t_plan, "per_set_ms": t_sets, "speedup": t_sets / t_plan,
            "plan_pair_evals_per_s": pairs / (t_plan * 1e-3)}


def extra_steps(lf, W, torch, dev, base, x, y, xq, norms, scalar_fwd_ms, reps=3):
    """Step-function local constants M_k(t) (Sec. 4.3) on the monotone local
    workload (d = 4, N = 1e5, Q = 1e6): quantile knots from 65,536 sampled
    pairs (K = 4), the FP64 all-pairs tables, and the bounds with M_k(dist),
    against the scalar-M_k forward of the same norm."""
    pairs = W.rng_for(300).integers(0, base.n, size=(65536, 2))
    probs = [0.2, 0.4, 0.6, 0.8]
    out = {"workload": f"monotone_local d={base.d} N={base.n} Q={base.q}, K=4 knots "
                       f"(quantiles 0.2..0.8 of 65536 sampled pair distances)"}
    for nm in norms:
        sym = lf.Metric(base.d, nm)
        mon = lf.Metric(base.d, nm, mon=base.mon)
        kn = {}
        t_knots = _time_ms(torch, lambda: kn.__setitem__(
            "k", lf.local_knots(x, sym, pairs, probs)), reps)
        knots = kn["k"].cpu().numpy()
        tab = {}
        t_tab = _time_ms(torch, lambda: tab.__setitem__("t", lf.local_steps(x, y, sym, knots)),
                         reps)
        d1, _, V32 = tab["t"]
        t_fwd = _time_ms(torch, lambda: lf.fit_eval_steps(x, y, xq, mon, knots, d1, V32), reps)
        pairs_fwd = float(base.n) * float(base.q)
        out[nm] = {"knots_ms": t_knots, "table_ms": t_tab,
                   "table_pairs_per_s": float(base.n) * float(base.n) / (t_tab * 1e-3),
                   "fwd_ms": t_fwd, "fwd_pair_evals_per_s": pairs_fwd / (t_fwd * 1e-3),
                   "fwd_time_vs_scalar_Mk": t_fwd / scalar_fwd_ms[nm]}
    return out


def extra_topk(lf, W, torch, dev, base, x, y, xq, norms, scalar_fwd_ms, reps=3):
    """The k best bounds with weights (Sec. 5, k = 3, w = (0.8, 0.1, 0.1)) on the
    monotone local workload (per-datum M_k of the workload), against the
    k = 1 forward of the same norm."""
    mk = torch.from_numpy(base.Mk).to(dev)
    out = {"workload": f"monotone_local d={base.d} N={base.n} Q={base.q}, k=3, w=(0.8,0.1,0.1)"}
    for nm in norms:
        met = lf.Metric(base.d, nm, mon=base.mon)
        t = _time_ms(torch, lambda: lf.fit_eval_k(x, y, xq, met, [0.8, 0.1, 0.1], Mk=mk), reps)
        out[nm] = {"fwd_ms": t,
                   "fwd_pair_evals_per_s": float(base.n) * float(base.q) / (t * 1e-3),
                   "fwd_time_vs_k1": t / scalar_fwd_ms[nm]}
    return out


def extra_regional(lf, W, torch, dev, base, x, y, xq, norms, scalar_fwd_ms, reps=3):
    """Monotonicity on parts of the domain (Sec. 4.2): coordinates 1 and 3 of
    the monotone local workload as case III and case IV on [0.3, 0.6], the
    others free, per-datum M_k of the workload, against the forward with plain
    monotone coordinates."""
    mk = torch.from_numpy(base.Mk).to(dev)
    out = {"workload": f"monotone_local d={base.d} N={base.n} Q={base.q}, kinds "
                       f"(III, free, IV, free) on [0.3, 0.6]"}
    for nm in norms:
        met = lf.Metric(base.d, nm, mon=[4, 0, 5, 0], a=[0.3] * 4, b=[0.6] * 4)
        t = _time_ms(torch, lambda: lf.fit_eval(x, y, xq, met, Mk=mk), reps)
        out[nm] = {"fwd_ms": t,
                   "fwd_pair_evals_per_s": float(base.n) * float(base.q) / (t * 1e-3),
                   "fwd_time_vs_plain_monotone": t / scalar_fwd_ms[nm]}
    return out


def extra_other_configs(lf, W, torch, dev, base, x, y, norms, reps=3):
    """The remaining workloads, each on its own inputs: the plain fit (d = 2,
    N = 1e3, Q = 1e4, l2, M = 4; launch-bound), the differentiable one (d = 8,
    N = 2e5, Q = 262,144, l2, M = 2: forward and backward through the saved
    indices), the global constant of the monotone local data (N^2 / 2 pairs
    per norm, FP64), and the FP64 consistency check on the first 2e5 points
    of the mixed-precision workload (d = 16, l2, M = 1)."""
    out = {}
    p = W.plain_l2()
    px, py, pq = (torch.from_numpy(a).to(dev) for a in (p.x, p.y, p.xq))
    met = lf.Metric(p.d, "l2")
    t = _time_ms(torch, lambda: lf.fit_eval(px, py, pq, met, M=p.M), 20)
    out["plain_l2"] = {"workload": f"plain_l2 d={p.d} N={p.n} Q={p.q} M={p.M} l2",
                       "fwd_ms": t, "fwd_pair_evals_per_s": float(p.n) * p.q / (t * 1e-3)}
    p = W.diff_l2()
    dx, dy_, dq, dgr = (torch.from_numpy(a).to(dev) for a in (p.x, p.y, p.xq, p.dg))
    met = lf.Metric(p.d, "l2")
    res = {}
    tf = _time_ms(torch, lambda: res.__setitem__("o", lf.fit_eval(dx, dy_, dq, met, M=p.M)), reps)
    o = res["o"]
    tb = _time_ms(torch, lambda: lf.backward(dx, dy_, dq, met, o["arg_up"], o["arg_lo"],
                                             dg=dgr, M=p.M), reps)
    pairs = float(p.n) * p.q
    out["diff_l2"] = {"workload": f"diff_l2 d={p.d} N={p.n} Q={p.q} M={p.M} l2",
                      "fwd_ms": tf, "bwd_ms": tb,
                      "fwd_pair_evals_per_s": pairs / (tf * 1e-3),
                      "fwd_bwd_pair_evals_per_s": pairs / ((tf + tb) * 1e-3)}
    gm = {}
    for nm in norms:
        met = lf.Metric(base.d, nm)
        t = _time_ms(torch, lambda: lf.estimate_M(x, y, met, mode="global"), reps)
        gm[nm] = {"ms": t, "pairs_per_s": float(base.n) * (base.n - 1) / 2 / (t * 1e-3)}
    out["global_M_monotone_local"] = gm
    p = W.mixed_l2(q=1)
    mx, my = (torch.from_numpy(a[:200_000].copy()).to(dev) for a in (p.x, p.y))
    met = lf.Metric(p.d, "l2")
    t = _time_ms(torch, lambda: lf.consistency(mx, my, met, M=p.M, per_row=False), reps)
    nc = 200_000
    out["consistency_mixed_l2_200k"] = {"workload": "mixed_l2 first 2e5 points, d=16, l2, M=1",
                                        "ms": t, "pairs_per_s": float(nc) * (nc - 1) / (t * 1e-3)}
    return out


def extra_smooth(lf, W, torch, dev, base, x, y, norms, reps=3):
    """Penalty objective of the smoothing problem (Sec. 4.4, Eq. 7) and its
    gradient on the monotone local workload's data (N = 1e5, d = 4, global
    M = 2, p = 1): one fused pass over the N^2 ordered pairs per evaluation;
    also with the pre-screening of Sec. 5 (c = 1/3, the exact FP64 decisions
    included)."""
    out = {"workload": f"monotone_local data d={base.d} N={base.n}, M=2, p=1, eps=0; "
                       f"pre-screened: c=1/3"}
    eps = torch.zeros(base.n, device=dev)
    for nm in norms:
        met = lf.Metric(base.d, nm, mon=base.mon)
        t = _time_ms(torch, lambda: lf.smooth_objective(x, y, eps, met, M=2.0, p=1.0), reps)
        tp = _time_ms(torch, lambda: lf.smooth_objective(x, y, eps, met, M=2.0, p=1.0,
                                                         prune=1 / 3), reps)
        out[nm] = {"objective_and_gradient_ms": t,
                   "pairs_per_s": float(base.n) * float(base.n) / (t * 1e-3),
                   "pre_screened_ms": tp}
    return out


def progress(msg):
    """One line per finished stage on stderr (stdout carries only the JSON line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


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
    progress(f"{a.warmup} warm-up steps done")

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
    progress(f"{a.steps} timed steps done: {ms_step:.1f} ms per step")
    stage_ms = {nm: {s: float(np.mean([evs[k][nm][s][0].elapsed_time(evs[k][nm][s][1])
                                        for k in range(a.steps)])) for s in stages}
                for nm in norms}

    pairs = float(N) * float(Q)
    value = len(norms) * pairs / (ms_step * 1e-3)
    per_norm = {}
    for nm in norms:
        f = stage_ms[nm]["forward"]
        b = stage_ms[nm]["backward"]
        rate = pairs / (f * 1e-3)
        per_norm[nm] = {
            "fwd_pair_evals_per_s": rate,
            "fwd_bwd_pair_evals_per_s": pairs / ((f + b) * 1e-3),
            "fwd_ms": f, "bwd_ms": b,
            "knn16_ms": stage_ms[nm]["knn"], "consistency_fp64_ms": stage_ms[nm]["consistency"],
            # fraction of the VALU issue peak spent on the minimal instruction mix
            "valu_frac": SLOTS_PER_PAIR[nm] * rate / VALU_PEAK_SLOTS,
            "datasheet_fp32_frac": FLOP_PER_PAIR[nm] * rate / 1e12 / FP32_DATASHEET_TFLOPS,
            "consistency_valu_frac": CONS_SLOTS_PER_PAIR[nm] * float(N) * float(N)
            / (stage_ms[nm]["consistency"] * 1e-3) / VALU_PEAK_SLOTS,
        }
    # dominant kernel: the forward bound kernel of the slowest norm
    dom = max(norms, key=lambda nm: stage_ms[nm]["forward"])
    f_ms = stage_ms[dom]["forward"]
    achieved = SLOTS_PER_PAIR[dom] * pairs / (f_ms * 1e-3) / 1e12
    peak = VALU_PEAK_SLOTS / 1e12
    roofline = {"bound": "alu", "kernel": f"bounds_fwd_kernel<4,2,{nid[dom]}> ({dom})",
                "achieved": round(achieved, 3), "peak": round(peak, 3),
                "unit": "T VALU-slot/s", "frac": round(achieved / peak, 4),
                "traffic": measured_traffic(dom),
                "slots_per_pair": SLOTS_PER_PAIR[dom], "instructions_per_pair": INSTR_PER_PAIR[dom]}

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
        progress(f"CPU baseline done ({tc1 - tc0:.1f} s)")

    extras = None
    if not a.no_extras:
        fwd = {nm: stage_ms[nm]["forward"] for nm in norms}
        runs = [("bf16_vs_fp32", lambda: extra_bf16(lf, W, torch, dev)),
                ("batched_vs_per_set", lambda: extra_batched(lf, W, torch, dev)),
                ("step_function_Mk",
                 lambda: extra_steps(lf, W, torch, dev, base, x, y, xq, norms, fwd)),
                ("smoothing_objective",
                 lambda: extra_smooth(lf, W, torch, dev, base, x, y, norms)),
                ("k_best_bounds",
                 lambda: extra_topk(lf, W, torch, dev, base, x, y, xq, norms, fwd)),
                ("regional_monotonicity",
                 lambda: extra_regional(lf, W, torch, dev, base, x, y, xq, norms, fwd)),
                ("other_configs",
                 lambda: extra_other_configs(lf, W, torch, dev, base, x, y, norms))]
        extras = {}
        for name, run in runs:
            extras[name] = run()
            progress(f"extra {name} done")

    rec = {
        "metric": METRIC, "value": value, "unit": "pair-evals/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "monotone_local", "d": D, "N": N, "Q": Q, "norms": norms,
                   "monotone": "increasing in coordinates 1 and 3", "M": "per-point, kNN-16",
                   "step": "per norm: kNN-16 M_k (f64) + consistency (f64) + forward (f32) "
                           "+ backward (f32)", "parallelism": "single GPU"},
        "per_norm": per_norm, "roofline": roofline, "cpu_baseline": cpu, "extras": extras,
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
