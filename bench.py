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

# Published MI355X peaks: FP32 vector 157.3 TFLOP/s, FP64 vector 78.6 TFLOP/s,
# dense BF16 MFMA 2.5 PFLOP/s.
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6
BF16_PEAK_TFLOPS = 2500.0

# Algorithmic FLOP per (query, datum) pair at d = 4 with two monotone
# coordinates (the convention of the design notes, section 6): a free
# coordinate costs 2 (l1 / linf: difference, absolute-value accumulate) or 3
# (l2: difference, FMA), a monotone one 3 (l1 / linf) or 5 (l2), l2 adds one
# square root per distance (two with monotone coordinates), every pair adds the
# two bounds (2 FMA = 4) and min + max (2).
FLOP_PER_PAIR = {"l1": 2 * 2 + 2 * 3 + 6, "linf": 2 * 2 + 2 * 3 + 6,
                 "l2": 2 * 3 + 2 * 5 + 2 + 6}
# The consistency pass: the same pair work plus a compare and a count (2),
# l1 / linf in FP64, l2 FP32-filtered (FP64 for the undecided pairs).
CONS_FLOP_PER_PAIR = {nm: f + 2 for nm, f in FLOP_PER_PAIR.items()}
# l2 at d = 16 without monotone coordinates: 16 x 3 + 1 root + 4 + 2
FLOP_PER_PAIR_L2_D16 = 16 * 3 + 1 + 6
CONS_PEAK_TFLOPS = {"l1": FP64_PEAK_TFLOPS, "linf": FP64_PEAK_TFLOPS, "l2": FP32_PEAK_TFLOPS}

# Hardware-counter figures of the forward kernels (VALU instructions per pair,
# issue rate against one wave64 FMA per SIMD every 4 cycles), from the
# rocprofv3 --pmc summary in profiles/; reported only while the kernel sources
# hash to the profiled ones.
COUNTERS_FILE = os.path.join(ROOT, "profiles", "valu_instructions_monotone_local.txt")


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


def _profile_record(path, tag):
    """The JSON record after `tag` in a profile summary, or None when the
    file is missing or was made from other kernel sources."""
    try:
        with open(path) as fh:
            for line in fh:
                if line.startswith(tag + " "):
                    rec = json.loads(line[len(tag) + 1:])
                    return rec if rec.get("source_sha256") == kernel_source_hash() else None
    except OSError:
        return None
    return None


def measured_traffic(norm):
    """Bytes per launch of the forward kernel for `norm`, or None."""
    rec = _profile_record(TRAFFIC_FILE, "TRAFFIC_JSON")
    return None if rec is None else rec["bytes_per_launch"].get(norm)


def measured_valu(norm):
    """VALU instructions per pair and issue rate of the forward kernel for
    `norm` from the counters, or None."""
    rec = _profile_record(COUNTERS_FILE, "COUNTERS_JSON")
    return None if rec is None else rec.get("valu", {}).get(norm)


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
    ap.add_argument("--copy-calib", action="store_true",
                    help="only copy a 1 GiB buffer 4 times (torch's copy kernel): the "
                         "reference for scaling FETCH_SIZE / WRITE_SIZE counters")
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
    issued_flop_per_pair = 2 * 16 * ks  # 32x32x16 MFMA K-steps as issued (K padded)
    algo_flop_per_pair = 2 * p.d        # the cross term x . x^k
    rate16 = pairs / (t16 * 1e-3)
    return {"workload": f"mixed_l2 d={p.d} N={p.n} Q={p.q} M={p.M} l2",
            "fp32_ms": t32, "bf16_ms": t16, "speedup": t32 / t16,
            "fp32_pair_evals_per_s": pairs / (t32 * 1e-3), "bf16_pair_evals_per_s": rate16,
            "fp32_peak_frac": FLOP_PER_PAIR_L2_D16 * pairs / (t32 * 1e-3) / 1e12
            / FP32_PEAK_TFLOPS,
            "identical_to_fp32": bool(same),
            "bf16_cross_term_tflops": algo_flop_per_pair * rate16 / 1e12,
            "bf16_cross_term_frac_of_2500_tflops": algo_flop_per_pair * rate16 / 1e12
            / BF16_PEAK_TFLOPS,
            "bf16_mfma_issued_tflops": issued_flop_per_pair * rate16 / 1e12,
            "note": "bf16_ms includes the y sort and staging of the data (per call); the "
                    "cross-term figure counts 2 d FLOP per pair, the issued one the padded "
                    "K of the MFMA"}


def extra_batched(lf, W, torch, dev, reps=3):
    """512 independent l2 sets (N log-uniform in [500, 50000], d in 2..10,
    Q = 4N): one graph launch of a plan with the default tiles, per-set
    lip_fit_eval calls, and a plan built after lip_autotune has tuned every
    (shape class, size class) the sets fall in (timed on synthetic data at
    the geometric-mean size of the class's sets)."""
    import math

    import numpy as np
    probs = W.batched()
    sets = []
    for pb in probs:
        sets.append(dict(x=torch.from_numpy(pb.x).to(dev), y=torch.from_numpy(pb.y).to(dev),
                         xq=torch.from_numpy(pb.xq).to(dev),
                         metric=lf.Metric(pb.d, pb.norm, mon=pb.mon, w=pb.w), M=pb.M))
    lf.tune_clear()
    plan = lf.Plan(sets)
    outs = [{k: v.clone() for k, v in o.items()} for o in plan.execute()]

    def per_set():
        for s_ in sets:
            lf.fit_eval(s_["x"], s_["y"], s_["xq"], s_["metric"], M=s_["M"])

    t_plan = _time_ms(torch, plan.execute, reps)
    t_sets = _time_ms(torch, per_set, reps)
    plan.close()
    # tune every class the sets fall in
    cls = {}
    for pb in probs:
        key = (pb.d, int(np.count_nonzero(pb.mon)), pb.norm,
               int(math.log2(pb.n)) // 2, int(math.log2(pb.q)) // 2)
        cls.setdefault(key, []).append(pb)
    t0 = time.perf_counter()
    tuned = {}
    for (d, m, nrm, _, _), group in sorted(cls.items()):
        n = int(round(math.exp(np.mean([math.log(g.n) for g in group]))))
        q = int(round(math.exp(np.mean([math.log(g.q) for g in group]))))
        cfg = lf.autotune(d, m, nrm, n, q)
        tuned[f"d={d} mon={m} n~{n} q~{q}"] = cfg["tile"]
    t_tune = time.perf_counter() - t0
    plan_t = lf.Plan(sets)
    got = plan_t.execute()
    torch.cuda.synchronize()
    same = all(torch.equal(a[k], b[k]) for a, b in zip(outs, got) for k in a)
    t_tuned = _time_ms(torch, plan_t.execute, reps)
    tiles = sorted({plan_t.tiles(i)["tile"] for i in range(len(sets))})
    plan_t.close()
    lf.tune_clear()
    pairs = float(sum(pb.n * pb.q for pb in probs))
    return {"workload": f"batched {len(probs)} sets, l2, sum N*Q = {pairs:.3e}",
            "plan_ms": t_plan, "per_set_ms": t_sets, "speedup": t_sets / t_plan,
            "plan_pair_evals_per_s": pairs / (t_plan * 1e-3),
            "tuned_plan_ms": t_tuned, "tuned_vs_default": t_plan / t_tuned,
            "tuned_identical_to_default": bool(same), "classes_tuned": len(cls),
            "autotune_s": t_tune, "tuned_tiles_used": tiles}


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
    if a.copy_calib:
        # the reference of the HBM counters: 4 plain copies of 1 GiB
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib": {"bytes_read_per_copy": src.numel() * 4,
                                         "bytes_written_per_copy": dst.numel() * 4,
                                         "copies": 4}}))
        return
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
        c = stage_ms[nm]["consistency"]
        rate = pairs / (f * 1e-3)
        per_norm[nm] = {
            "fwd_pair_evals_per_s": rate,
            "fwd_bwd_pair_evals_per_s": pairs / ((f + b) * 1e-3),
            "fwd_ms": f, "bwd_ms": b,
            "knn16_ms": stage_ms[nm]["knn"], "consistency_ms": c,
            # algorithmic FLOP (design notes, section 6) over the published peaks
            "fwd_fp32_peak_frac": FLOP_PER_PAIR[nm] * rate / 1e12 / FP32_PEAK_TFLOPS,
            "consistency_peak_frac": CONS_FLOP_PER_PAIR[nm] * float(N) * float(N)
            / (c * 1e-3) / 1e12 / CONS_PEAK_TFLOPS[nm],
            "consistency_peak": "fp64" if CONS_PEAK_TFLOPS[nm] == FP64_PEAK_TFLOPS else "fp32",
        }
    # dominant kernel: the forward bound kernel of the slowest norm, timed by
    # HIP events on its launch stream around each call (origin and staging
    # kernels, a few microseconds, included)
    dom = max(norms, key=lambda nm: stage_ms[nm]["forward"])
    f_ms = stage_ms[dom]["forward"]
    achieved = FLOP_PER_PAIR[dom] * pairs / (f_ms * 1e-3) / 1e12
    kname = (f"bounds_fwd_kernel{'_o4' if dom != 'l1' else ''}<4, 2, {nid[dom]}>")
    valu = measured_valu(dom)
    roofline = {"bound": "alu", "kernel": f"{kname} ({dom} forward)",
                "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                "traffic": measured_traffic(dom),
                "flop_per_pair": FLOP_PER_PAIR[dom], "pairs_per_launch": pairs,
                "launch_ms": round(f_ms, 3),
                "valu_counters": valu}

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
