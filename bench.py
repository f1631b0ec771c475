#!/usr/bin/env python
"""Benchmark: spatiotemporal Hawkes log-likelihood + full gradient on one MI355X.

Workload: the wildfire-like coarsened case, N = 50,000 events in D = 2 (500 km
box, ten years, 30 % of locations latent in discs), synthetic and seeded.  One
step is one complete evaluation through the C ABI (hawkes_grad): validation,
packing, the rate pass, finalize (log-likelihood and the six parameter
gradients, delivered to the host) and the gradient pass (N x D location
gradient in device memory).  Inputs are resident in HBM before timing starts.

Throughput is ordered pair-interactions per second, N (N - 1) per step.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pair-interactions/s for Hawkes loglik+grad (FP64 vs mixed); serve p50/p99 ms"
STAGES = ["prep", "pack", "pass1", "reduce1", "fix1", "final1", "pass2", "fix2", "reduce2"]
KERNEL_NAMES = {"pass1": "k_pass1", "pass2": "k_pass2"}
PROFILED_NAMES = {("pass1", "mixed"): "hawkes::k_pass1_mixed<2, false>", ("pass2", "mixed"): "hawkes::k_pass2_mixed<2>",
                  ("pass1", "fp64"): "hawkes::k_pass1<2, false>", ("pass2", "fp64"): "hawkes::k_pass2<2, false>"}

# Peaks of the chip (256 CUs at 2.4 GHz).  FP32 vector: 157.3 TFLOP/s.  The
# v_exp_f32 issue rate is 32 lanes per CU per clock (measured by the peaks
# microbenchmark), so one exp occupies the issue time of 8 FP32 FLOPs.
PEAK_FP32 = 157.3e12
PEAK_FP64 = 78.6e12
EXP_F32_PER_S = 256 * 2.4e9 * 32
FLOP_EQ_PER_EXP = PEAK_FP32 / EXP_F32_PER_S


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("hawkes_kernels.hpp", "hawkes_common.hpp"):
        with open(os.path.join(ROOT, "paper_2010_02994_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_prefix: str, workload: str):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy of known size),
    or None when the kernels changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "hawkes_grad_c2_n50000_d2.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except OSError:
        return None
    if rec.get("source_sha256_16") != kernel_source_hash() or rec.get("workload") != workload:
        return None
    for k, v in rec["kernels"].items():
        if k.startswith(kernel_prefix):
            return int(v["bytes_read"] + v["bytes_written"])
    return None


def pass_work(d: int, which: str):
    """Algorithmic work per unordered pair (FLOPs with FMA = 2, exps), the
    method's minimum: rate pass -- differences (D+1), r^2 (2D-1), dt^2 (1), two
    exponents (8), nine accumulations (15): 3D+24 and 2 exps; gradient pass --
    recompute (3D+9), weights (6), two-sided scatter (4D): 7D+15 and 2 exps.
    The roofline is priced with these counts for both precisions."""
    return (3 * d + 24, 2) if which == "pass1" else (7 * d + 15, 2)


def pass_work_resplit(d: int, which: str):
    """The same total work as split by a mixed gradient call, which moves the
    two background moments (r^2 and dt^2 sums, row and column: 8 FLOPs) out of
    the rate pass and forms their gradient terms in the gradient pass as two
    weighted sums (4 FLOPs): 3D+16 and 7D+19.  Reported beside the roofline."""
    return (3 * d + 16, 2) if which == "pass1" else (7 * d + 19, 2)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=20,
                    help="untimed steps first (the chip's clock settles over the first ~15 evaluations)")
    ap.add_argument("--n", type=int, default=50000)
    ap.add_argument("--prec", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--fp64-steps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="single-core oracle seconds the CPU baseline's sample is sized for")
    ap.add_argument("--serve-requests", type=int, default=10000,
                    help="requests measured per precision in the long serving run (0 skips serving)")
    ap.add_argument("--serve-sweep-requests", type=int, default=1500,
                    help="requests per offered rate in the serving saturation sweep (0 skips the sweep)")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--cull-steps", type=int, default=5,
                    help="timed steps with exact culling, reported apart from the headline (0 skips)")
    ap.add_argument("--bmds-reps", type=int, default=10,
                    help="timed Bayesian MDS evaluations per case and precision (0 skips)")
    ap.add_argument("--hmc-only", action="store_true",
                    help="run only the leapfrog measurement (for profiling its kernels on their own)")
    ap.add_argument("--bmds-only", action="store_true",
                    help="run only the Bayesian MDS measurement (for profiling its kernels on their own)")
    ap.add_argument("--hmc-trajectories", type=int, default=3,
                    help="timed 20-step device leapfrog trajectories on the gridded 10,000-event workload (0 skips)")
    ap.add_argument("--mwg-steps", type=int, default=3000,
                    help="Metropolis-within-Gibbs location steps timed at one event per step (0 skips)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (one evaluation would shard "
              "over blocks of the unordered-pair triangle). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2010_02994_amd import _lib, api, workloads

    dev = torch.device("cuda:0")
    if args.bmds_only:
        print(json.dumps({"bmds": bmds_bench(dev, max(1, args.bmds_reps))}), flush=True)
        return
    if args.hmc_only:
        print(json.dumps({"hmc": leapfrog_bench(dev, max(1, args.hmc_trajectories))}), flush=True)
        return
    w = workloads.config2(n=args.n)
    n, d = w.n, w.d
    x = torch.tensor(w.x, device=dev)
    t = torch.tensor(w.t, device=dev)
    gx = torch.empty_like(x)
    L = _lib.lib()
    ps = api.params_struct(w.params)
    stream = torch.cuda.current_stream(dev).cuda_stream

    def run(prec: str, steps: int, warmup: int, stage_steps: int, per_step: dict | None = None):
        """Time `steps` calls of hawkes_grad (the product path: the fix-up and
        finalize chain overlaps pass 2 on a side stream), bracketed by device
        synchronizations, with a pair of HIP events on the call's stream
        around every call (per_step receives their median, quartiles and
        mean); then take the per-stage breakdown from `stage_steps` calls of
        hawkes_grad_timed, which runs every stage in sequence on the one
        stream with HIP events around each kernel."""
        pc = api._prec(prec)
        ws = api.workspace(n, d, prec, dev)
        ll = ctypes.c_double()
        gp = (ctypes.c_double * 6)()
        stage = (ctypes.c_float * len(STAGES))()

        def call():
            st = L.hawkes_grad(x.data_ptr(), t.data_ptr(), n, d, ctypes.byref(ps), pc, ws.data_ptr(), ws.numel(),
                               stream, ctypes.byref(ll), gx.data_ptr(), gp)
            assert st == 0, _lib.strerror(st)

        for _ in range(warmup):
            call()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for a, b in evs:
            a.record()
            call()
            b.record()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        if per_step is not None:
            ms = np.array([a.elapsed_time(b) for a, b in evs])
            q1, med, q3 = np.percentile(ms, [25, 50, 75])
            per_step.update({"median_ms": float(med), "iqr_ms": float(q3 - q1), "q1_ms": float(q1),
                             "q3_ms": float(q3), "mean_ms": float(ms.mean()), "min_ms": float(ms.min()),
                             "max_ms": float(ms.max()), "steps": int(steps),
                             "note": "HIP events on the call's stream around each hawkes_grad call"})
        acc = np.zeros(len(STAGES))
        for _ in range(stage_steps if "+cull" not in prec else 0):
            st = L.hawkes_grad_timed(x.data_ptr(), t.data_ptr(), n, d, ctypes.byref(ps), pc, ws.data_ptr(),
                                     ws.numel(), stream, ctypes.byref(ll), gx.data_ptr(), gp, stage)
            assert st == 0, _lib.strerror(st)
            acc += np.array(stage[:])
        return el / steps, acc / max(stage_steps, 1), ll.value

    # the same evaluations enqueued back to back with hawkes_grad_async (results
    # stay on the device, one synchronization at the end), beside the headline's
    # synchronous calls: the difference is the per-call host round trip.  Timed
    # first, so that the headline's stage-timed calls stay the process's last
    # dispatches of the mixed kernels
    async_ms = None
    if args.steps > 0:
        ws_a = api.workspace(n, d, args.prec, dev)
        out8 = torch.empty(8, dtype=torch.float64, device=dev)

        def acall():
            st = L.hawkes_grad_async(x.data_ptr(), t.data_ptr(), n, d, ctypes.byref(ps), api._prec(args.prec),
                                     ws_a.data_ptr(), ws_a.numel(), stream, out8.data_ptr(), gx.data_ptr())
            assert st == 0, _lib.strerror(st)

        for _ in range(args.warmup):
            acall()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            acall()
        torch.cuda.synchronize()
        async_ms = (time.perf_counter() - t0) / args.steps * 1e3
        assert out8[7].item() == 0.0

    step_stats = {}
    sec_mixed, stage_ms, ll_m = run(args.prec, args.steps, args.warmup, max(5, args.steps // 2), step_stats)
    pairs = n * (n - 1)
    value = pairs / sec_mixed

    fp64 = None
    if args.prec == "mixed" and args.fp64_steps > 0:
        st64 = {}
        sec64, stage64, ll_64 = run("fp64", args.fp64_steps, 8, 2, st64)
        fp64 = {"value": pairs / sec64, "ms_per_step": sec64 * 1e3, "per_step": st64,
                "stage_ms": {k: round(float(v), 4) for k, v in zip(STAGES, stage64)},
                "loglik_rel_diff_mixed_vs_fp64": abs(ll_m - ll_64) / abs(ll_64)}

    # exact culling (bitwise-identical results), reported apart from the all-pairs headline
    culling = None
    if args.cull_steps > 0:
        gx_all = gx.clone()
        culling = {"note": "column tiles whose pair terms all underflow are skipped; results bitwise equal"}
        for base in ([args.prec] + (["fp64"] if args.prec == "mixed" and args.fp64_steps > 0 else [])):
            # all-pairs and culled steps timed in three alternating rounds, best
            # of each, so that both see the same clock states
            sec_all = sec_c = float("inf")
            for _ in range(3):
                s_a, _, ll_ref = run(base, args.cull_steps, 1, 0)
                ref = gx.clone()
                s_c, _, ll_c = run(base + "+cull", args.cull_steps, 1, 0)
                sec_all, sec_c = min(sec_all, s_a), min(sec_c, s_c)
            culling[base] = {"ms_per_step": sec_c * 1e3, "all_pairs_ms_per_step": sec_all * 1e3,
                             "speedup_vs_all_pairs": sec_all / sec_c,
                             "bitwise_equal": bool(ll_c == ll_ref and torch.equal(gx, ref))}
        gx.copy_(gx_all)

    # dominant kernel and its roofline (algorithmic work per launch / measured
    # duration, the launch timed with HIP events on its own stream)
    pass_ms = {k: float(stage_ms[STAGES.index(k)]) for k in ("pass1", "pass2")}
    dom = max(pass_ms, key=pass_ms.get)
    flops, exps = pass_work(d, dom)
    pairs_u = n * (n - 1) / 2
    work = pairs_u * (flops + exps * FLOP_EQ_PER_EXP)
    achieved = work / (pass_ms[dom] * 1e-3)
    peak = PEAK_FP32 if args.prec == "mixed" else PEAK_FP64
    rf, re_ = pass_work_resplit(d, dom)
    roof = {"bound": "alu", "kernel": f"{KERNEL_NAMES[dom]}<D={d},{args.prec}>",
            "achieved": round(achieved / 1e12, 3), "peak": peak / 1e12, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4),
            "traffic": measured_traffic(PROFILED_NAMES.get((dom, args.prec), "?"), w.name) if d == 2 else None,
            "work_per_unordered_pair": {"flops": flops, "exps": exps, "flop_eq_per_exp": FLOP_EQ_PER_EXP},
            "units_per_launch": pairs_u, "kernel_ms": round(pass_ms[dom], 4),
            "frac_at_resplit_count": round(pairs_u * (rf + re_ * FLOP_EQ_PER_EXP) / (pass_ms[dom] * 1e-3) / peak, 4),
            "resplit_work_per_unordered_pair": {"flops": rf, "exps": re_}}
    # whole-path roofline: both passes' algorithmic work over the full step time
    f1, e1 = pass_work(d, "pass1")
    f2, e2 = pass_work(d, "pass2")
    path_work = pairs_u * (f1 + f2 + (e1 + e2) * FLOP_EQ_PER_EXP)

    mwg = mwg_bench(w, dev, args.mwg_steps) if args.mwg_steps > 0 else None
    if mwg is not None:
        # the same moves at the size of the paper's wildfire data (N = 2,925,
        # same events per km^2 and day), for the per-state context
        from paper_2010_02994_amd import workloads as _wl
        mwg["n2925"] = mwg_bench(_wl.config2(n=2925, same_density=True), dev, args.mwg_steps)
    hmc = leapfrog_bench(dev, args.hmc_trajectories) if args.hmc_trajectories > 0 else None
    bmds = bmds_bench(dev, args.bmds_reps) if args.bmds_reps > 0 else None

    serve = None
    if args.serve_requests > 0:
        serve = serving(args.serve_requests, args.serve_rate, args.serve_sweep_requests)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, args.cpu_seconds)

    out = {"metric": METRIC, "value": value, "unit": "pair-interactions/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": sec_mixed * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32-pairs/f64-accumulate" if args.prec == "mixed" else "f64",
           "data": "synthetic",
           "config": {"workload": w.name, "n_events": n, "d": d, "precision": args.prec,
                      "pairs_per_step": pairs, "parallelism": "single-gpu"},
           "roofline": roof,
           "path_roofline_frac": round(path_work / sec_mixed / peak, 4),
           "path_roofline_note": "both passes' algorithmic work (10D+39 FLOPs + 4 exps per unordered pair) over "
                                 "ms_per_step, against the same peak",
           "per_step": step_stats,
           "async_back_to_back_ms_per_step": async_ms,
           "async_note": "hawkes_grad_async calls enqueued back to back, one synchronization at the end",
           "stage_ms": {k: round(float(v), 4) for k, v in zip(STAGES, stage_ms)},
           "stage_ms_note": "stages timed in sequence on one stream (hawkes_grad_timed); ms_per_step is "
                            "hawkes_grad, where fix1, final1 and fix2 overlap pass2 on a side stream",
           "fp64": fp64,
           "exact_culling": culling,
           "speedup_mixed_vs_fp64": (value / fp64["value"]) if fp64 else None,
           "mwg": mwg,
           "hmc": hmc,
           "bmds": bmds,
           "serve": serve,
           "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


def mwg_bench(w, dev, steps: int):
    """Metropolis-within-Gibbs location updates on the same workload: each step
    proposes new places for a block of latent events, uniform on each event's
    disc around its observed location (an independence proposal, so the
    threshold is log u), and is decided and applied on the device.  Steps are
    enqueued back to back with no host synchronization; x and the cached
    per-event terms stay resident in HBM."""
    import torch
    from paper_2010_02994_amd import _lib, api
    rng = np.random.default_rng(7)
    latent = np.flatnonzero(w.radius > 0)
    x = torch.tensor(w.x, device=dev)
    t = torch.tensor(w.t, device=dev)
    out = {"workload": f"{w.name}: latent-disc location moves", "state": "fp64 per-event terms"}
    for block, n_steps in ((1, steps), (64, max(1, steps // 6))):
        x.copy_(torch.tensor(w.x, device=dev))   # each block size starts from the workload's state
        terms, _ = api.event_terms(x, t, w.params, prec="fp64")
        idx = np.sort(np.stack([rng.choice(latent, size=block, replace=False) for _ in range(n_steps)]), axis=1)
        ang = rng.uniform(0, 2 * np.pi, idx.shape)
        rad = w.radius[idx] * np.sqrt(rng.uniform(size=idx.shape))
        xn = w.observed[idx] + np.stack([rad * np.cos(ang), rad * np.sin(ang)], axis=-1)
        thr = np.log(rng.uniform(size=n_steps))
        idx_d = torch.tensor(idx.astype(np.int64), device=dev)
        xn_d = torch.tensor(xn, device=dev)
        thr_d = torch.tensor(thr, device=dev)
        outs = torch.empty((n_steps, 3), dtype=torch.float64, device=dev)
        ws = api.mwg_workspace(w.n, dev)
        # the C entry point straight from precomputed pointers, so host-side
        # argument marshalling stays out of the device-bound loop
        L = _lib.lib()
        ps = api.params_struct(w.params)
        stream = torch.cuda.current_stream(dev).cuda_stream
        xp, tp, tmp, wp = x.data_ptr(), t.data_ptr(), terms.data_ptr(), ws.data_ptr()
        ip, np_, hp, op = idx_d.data_ptr(), xn_d.data_ptr(), thr_d.data_ptr(), outs.data_ptr()

        def step(s):
            st = L.hawkes_mwg_step(xp, tp, w.n, w.d, ctypes.byref(ps), tmp, ip + s * block * 8,
                                   np_ + s * block * w.d * 8, block, hp + s * 8, wp, ws.numel(), stream, op + s * 24)
            assert st == 0, _lib.strerror(st)

        warm = min(50, n_steps)
        for s in range(warm):
            step(s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(warm, n_steps):
            step(s)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        o = outs.cpu().numpy()
        timed = n_steps - warm
        # drift of the incrementally updated terms against a fresh evaluation
        fresh, _ = api.event_terms(x, t, w.params, prec="fp64")
        tc, tf = terms.cpu().numpy(), fresh.cpu().numpy()
        lam = w.params[0] * tf[:, 0] + w.params[3] * tf[:, 1]
        drift_ab = float(np.max((w.params[0] * np.abs(tc[:, 0] - tf[:, 0]) + w.params[3] * np.abs(tc[:, 1] - tf[:, 1]))
                                / lam))
        drift_log = float(np.max(np.abs(tc[:, 2] - tf[:, 2])))
        out[f"block{block}"] = {"steps": timed, "us_per_step": el / max(timed, 1) * 1e6,
                                "steps_per_s": timed / el if el > 0 else None,
                                "pair_terms_per_step": block * (w.n - 1) * 2,
                                "accept_rate": float(o[:, 1].mean()), "bad_status": int((o[:, 2] != 0).sum()),
                                "accepted": int(o[:, 1].sum()),
                                "terms_drift": {"rate_rel_max": drift_ab, "log_rate_abs_max": drift_log}}
    x.copy_(torch.tensor(w.x, device=dev))
    return out


def leapfrog_bench(dev, trajectories: int):
    """GPU-driven HMC trajectories on the gridded workload (N = 10,000, D = 2,
    100 m cells): 20 leapfrog steps of 0.002 km, unit mass, momenta N(0, I),
    positions reflected at the cell walls; every gradient is a full
    evaluation, nothing returns to the host between steps."""
    import torch
    from paper_2010_02994_amd import api, workloads
    w = workloads.config1(snapshots=0)
    lo = torch.tensor(w.observed - 0.5 * w.cell, device=dev)
    hi = torch.tensor(w.observed + 0.5 * w.cell, device=dev)
    t = torch.tensor(w.t, device=dev)
    rng = np.random.default_rng(11)
    steps, eps = 20, 0.002
    out = {"workload": f"{w.name}: 20-step leapfrog, reflecting cell walls", "steps": steps, "eps_km": eps}
    for prec in ("mixed", "fp64"):
        x = torch.tensor(w.x, device=dev)
        p = torch.tensor(rng.standard_normal(w.x.shape), device=dev)
        g, out8 = api.leapfrog(x, p, t, w.params, eps, steps, prec=prec, bound="box", b0=lo, b1=hi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(trajectories):
            p.copy_(torch.tensor(rng.standard_normal(w.x.shape), device=dev))
            g, out8 = api.leapfrog(x, p, t, w.params, eps, steps, prec=prec, bound="box", b0=lo, b1=hi,
                                   grad_x=g, have_grad=True, out8=out8)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / trajectories
        inside = bool(((x >= lo) & (x <= hi)).all().item())
        # the same trajectory captured once in a HIP graph and replayed: the
        # launch overhead of ~250 kernels per trajectory leaves the host
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            api.leapfrog(x, p, t, w.params, eps, steps, prec=prec, bound="box", b0=lo, b1=hi,
                         grad_x=g, have_grad=True, out8=out8)
        graph.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(trajectories):
            graph.replay()
        torch.cuda.synchronize()
        elg = (time.perf_counter() - t0) / trajectories
        out[prec] = {"ms_per_trajectory": el * 1e3, "ms_per_step": el * 1e3 / steps,
                     "pair_interactions_per_s": steps * w.n * (w.n - 1) / el,
                     "graph_ms_per_trajectory": elg * 1e3,
                     "status": float(out8[7].item()), "inside_cells": inside}
        del graph
    out["flu_joint"] = flu_leapfrog_bench(dev, trajectories)
    return out


def flu_leapfrog_bench(dev, trajectories: int):
    """The influenza model's HMC (N = 4,733 cases, D = 6, 64 countries): 20
    unconstrained leapfrog steps whose every gradient is the Hawkes
    log-likelihood gradient plus the Bayesian MDS gradient."""
    import torch
    from paper_2010_02994_amd import api, workloads
    w, dl, sigma = workloads.flu_case_device(device=dev)
    t = torch.tensor(w.t, device=dev)
    rng = np.random.default_rng(12)
    steps, eps = 20, 0.001
    out = {"workload": f"{w.name}: 20-step leapfrog on the Hawkes + MDS potential", "steps": steps, "eps": eps}
    for prec in ("mixed", "fp64"):
        x = torch.tensor(w.x, device=dev)
        p = torch.tensor(rng.standard_normal(w.x.shape), device=dev)
        g, out8, out4 = api.leapfrog_bmds(x, p, t, w.params, dl, sigma, eps, steps, prec=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(trajectories):
            p.copy_(torch.tensor(rng.standard_normal(w.x.shape), device=dev))
            g, out8, out4 = api.leapfrog_bmds(x, p, t, w.params, dl, sigma, eps, steps, prec=prec, grad_x=g,
                                              have_grad=True, out8=out8, out4=out4)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / trajectories
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            api.leapfrog_bmds(x, p, t, w.params, dl, sigma, eps, steps, prec=prec, grad_x=g, have_grad=True,
                              out8=out8, out4=out4)
        graph.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(trajectories):
            graph.replay()
        torch.cuda.synchronize()
        elg = (time.perf_counter() - t0) / trajectories
        out[prec] = {"ms_per_trajectory": el * 1e3, "ms_per_step": el * 1e3 / steps,
                     "graph_ms_per_trajectory": elg * 1e3, "hawkes_status": float(out8[7].item()),
                     "mds_status": float(out4[3].item())}
        del graph
    return out


def bmds_bench(dev, reps: int):
    """Bayesian MDS log-likelihood + gradients: the influenza-like case
    (N = 4,733 cases in D = 6, 64 countries, dissimilarities between country
    centres, same-country pairs unobserved) and a larger N = 20,000, D = 6 case
    (|z_n - z_n'| plus folded normal noise), both drawn on the device.  The pass reads the strict lower triangle of the float64
    matrix once, so its roofline is HBM: 4 N (N - 1) bytes per evaluation.  Beside it, the VALU roofline of the pair
    arithmetic: per pair 7D + 8 FLOPs (differences D, squared distance 2D - 1, residual and its square 3, the log Phi
    and rho z sums 3, the coefficient 3, gradient rows and columns 4D) and three special functions (the distance's
    square root and reciprocal, the normal density's exponential, log Phi) at 8 FLOP-equivalents each, against the
    float32 (157.3) or float64 (78.6 TFLOP/s) vector peak."""
    import torch
    from paper_2010_02994_amd import api, workloads
    out = {}
    cases = [("flu_n4733_d6_64countries",) + workloads.bmds_case_device(4733, 4733, 6, groups=64, device=dev),
             ("dense_n20000_d6",) + workloads.bmds_case_device(20000, 20000, 6, device=dev)]
    for name, x, dl, sigma in cases:
        n = x.shape[0]
        rec = {"n": n, "d": int(x.shape[1]), "delta_bytes_read": 4 * n * (n - 1)}
        for prec in ("mixed", "fp64"):
            o, gx = api.bmds(x, dl, sigma, prec=prec)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                o, gx = api.bmds(x, dl, sigma, prec=prec, grad_x=gx, out4=o)
            torch.cuda.synchronize()
            el = (time.perf_counter() - t0) / reps
            flop_eq = 7 * x.shape[1] + 8 + 3 * 8
            valu_tflops = 0.5 * n * (n - 1) * flop_eq / el / 1e12
            rec[prec] = {"ms": el * 1e3, "pair_interactions_per_s": n * (n - 1) / el,
                         "delta_GB_per_s": 4 * n * (n - 1) / el / 1e9,
                         "hbm_frac": 4 * n * (n - 1) / el / 8e12, "status": float(o[3].item()),
                         "valu_flop_eq_per_pair": flop_eq, "valu_tflops": valu_tflops,
                         "valu_frac": valu_tflops / (157.3 if prec == "mixed" else 78.6)}
        out[name] = rec
        del x, dl
    return out


def serving(n_requests: int, rate: float, sweep_requests: int):
    """64 HMC chains over 64 datasets with N log-uniform in [1e3, 1e5] (D = 2,
    coarsened to a 100 m grid), open-loop Poisson arrivals.  For each precision:
    the long run (n_requests measured after a 5 s warm-up at `rate`), then an
    offered-rate sweep up to and beyond saturation (sweep_requests each, 1 s
    warm-up), whose highest achieved throughput is the measured capacity."""
    from paper_2010_02994_amd import loadgen
    from paper_2010_02994_amd.serve import Server
    out = {"chains": 64, "n_range": [1000, 100000], "offered_rate_req_s": rate, "streams": 3, "max_slots": 64,
           "hbm_budget_GiB": 24}
    sweeps = {"mixed": [400.0, 800.0, 1600.0, 3200.0], "fp64": [300.0, 600.0, 1200.0]}
    with Server(hbm_budget_bytes=24 << 30, max_slots=64, streams=3) as srv:
        chains = loadgen.Chains(srv, count=64)
        for prec in ("mixed", "fp64"):
            out[prec] = loadgen.run(srv, chains, rate=rate, n_requests=n_requests, prec=prec, warmup_s=5.0)
            print(f"serve {prec} at {rate:.0f} req/s: p50 {out[prec]['p50_ms']:.2f} ms, "
                  f"p99 {out[prec]['p99_ms']:.2f} ms", file=sys.stderr, flush=True)
            sw = []
            for r in sweeps[prec] if sweep_requests > 0 else []:
                res = loadgen.run(srv, chains, rate=r, n_requests=sweep_requests, prec=prec, warmup_s=1.0)
                sw.append({k: res[k] for k in ("offered_rate", "submit_rate_req_s", "throughput_req_s", "pairs_per_s",
                                               "p50_ms", "p99_ms", "queue_wait_ms", "admit_to_start_ms",
                                               "service_ms", "requests", "errors", "unfinished")})
                print(f"serve {prec} sweep {r:.0f} req/s: {res['throughput_req_s']:.0f} req/s, "
                      f"p50 {res['p50_ms']:.1f} ms", file=sys.stderr, flush=True)
            out[prec + "_sweep"] = sw
            if sw:
                best = max(sw, key=lambda e: e["throughput_req_s"] or 0.0)
                out[prec + "_capacity_req_s"] = best["throughput_req_s"]
                out[prec + "_capacity_pairs_per_s"] = best["pairs_per_s"]
        out["batches_launched"] = srv.stats()["batches_launched"]
    return out


def _cpu_model() -> str:
    try:
        import subprocess
        out = subprocess.run(["lscpu"], stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, text=True).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, seconds: float):
    """The oracle as it stands, on the first N_s events of the same workload
    (N_s sized so that three single-core runs take about `seconds`): its
    single-threaded build on one core and its OpenMP build (rows split over
    threads; the same arithmetic per row) on every core of the host, both on
    that same sample, three runs each (median and interquartile range of the
    times).  value = the all-core rate at the median time."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    n0 = 1500
    t0 = time.perf_counter()
    oracle.loglik_grad(w.x[:n0], w.t[:n0], w.params, threads=False)
    dt0 = time.perf_counter() - t0
    ns = int(min(w.n, max(n0, n0 * (seconds / 3 / max(dt0, 1e-3)) ** 0.5)))
    x, t = w.x[:ns], w.t[:ns]

    def runs(threaded):
        el, ll = [], None
        for _ in range(3):
            t0 = time.perf_counter()
            st, ll, _, _ = oracle.loglik_grad(x, t, w.params, threads=threaded)
            el.append(time.perf_counter() - t0)
        q1, med, q3 = (float(v) for v in np.percentile(el, [25, 50, 75]))
        return {"median_s": round(med, 4), "iqr_s": round(q3 - q1, 4), "runs_s": [round(v, 4) for v in el]}, ll

    one, ll1 = runs(False)
    allc, ll2 = runs(True)
    pairs = ns * (ns - 1)
    return {"value": pairs / allc["median_s"], "unit": "pair-interactions/s", "cores": threads, "kind": "oracle",
            "sample": f"oracle loglik+grad (C, float64) on the first {ns} of {w.n} events of {w.name}",
            "seconds": allc["median_s"], "times": allc,
            "single_core": {"value": pairs / one["median_s"], "cores": 1, "seconds": one["median_s"], "times": one,
                            "build": "single-threaded oracle"},
            "all_cores_build": "OpenMP over rows", "same_result": bool(ll1 == ll2),
            "cpu_model": _cpu_model(), "nproc": os.cpu_count()}


if __name__ == "__main__":
    main()
