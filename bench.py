#!/usr/bin/env python3
"""Bench of the bin_packing feasibility check on one MI355X.

Workload (one step = the whole hot path once): the single large residual
instance -- n = 10,000 unpacked sizes U[C/10, C/2], C = 100,000, m = 4,000
bins with remaining capacity U[C/2, C] -- already resident in HBM.  A step
reduces it on the device (one virtual item per loaded bin), sorts, builds
prefix sums, evaluates L1, L2 and the six dual-feasible-function sweeps over
every integer parameter and takes the verdict.

Prints one JSON line.  value = (item x parameter) evaluations per second of
the six sweeps over the timed steps (E = r * sum of range sizes per step).
Extra fields: checks/s of this workload, the roofline of the dominant kernel
(the sweep) from HIP events on its stream, the plain single-check latency
(p50/p99) of the small partial packing, and the oracle's CPU rate on a
bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Full-rate VALU issue slots per (item, parameter) evaluation of each sweep,
# from the instruction sequences of the inner loops (32-bit add, sub and
# shift-right issue at twice the full rate on gfx950 and count 1/2).
OPS_PER_EVAL = {"MT": 2.5, "RAD2": 3.0, "FS1": 9.0, "CCM1": 2.0, "VB2": 2.5, "BJ1": 4.0}
PEAK_VALU = 256 * 64 * 2.4e9  # full-rate lane-instructions/s: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz
DFF_NAMES = ("MT", "RAD2", "FS1", "CCM1", "VB2", "BJ1")


def percentile(xs, p):
    import numpy as np
    return float(np.percentile(np.asarray(xs), p)) if len(xs) else None


def cpu_baseline(C, items, target_s: float):
    """The oracle as it stands, on a strided sample of every sweep's parameters."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor

    import oracle as O

    O._load()
    threads = min(16, os.cpu_count() or 1)
    # rate probe: one parameter of each function
    t0 = time.perf_counter()
    ev = 0
    for d in O.DFFS:
        lo, hi = O.default_range(d, C)
        ev += O.dff_bound_strided(d, C, items, lo, lo, 1)[2]
    rate1 = ev / max(time.perf_counter() - t0, 1e-9)
    total_params = sum(max(0, O.default_range(d, C)[1] - O.default_range(d, C)[0] + 1) for d in O.DFFS)
    want_evals = rate1 * threads * target_s
    stride = max(1, int(total_params * len(items) / max(want_evals, 1)))
    jobs = []
    for d in O.DFFS:
        lo, hi = O.default_range(d, C)
        if lo > hi:
            continue
        # split each function's strided parameters into chunks for the pool
        per = max(1, (hi - lo + 1) // (threads * 4))
        start = lo
        while start <= hi:
            end = min(hi, start + per - 1)
            jobs.append((d, start, end))
            start = end + 1

    def run(job):
        d, a, b = job
        first = a + ((-(a - O.default_range(d, C)[0])) % stride)
        if first > b:
            return 0
        return O.dff_bound_strided(d, C, items, first, b, stride)[2]

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        evals = sum(ex.map(run, jobs))
    dt = time.perf_counter() - t0
    return {"value": evals / dt, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"every {stride}th parameter of each of the six sweeps of this instance "
                      f"({evals} evaluations, {dt:.1f} s on {threads} threads)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--latency-checks", type=int, default=2000)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU layout is "
              "described in DESIGN.md and not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2402_14821_amd as bp
    from paper_2402_14821_amd import workloads as W

    dev = torch.device("cuda:0")
    C, m, residual, unpacked = W.large_residual(seed=1)
    d_res = torch.from_numpy(residual).to(dev)
    d_unp = torch.from_numpy(unpacked).to(dev)
    d_out = torch.zeros(bp.BOUNDS_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)
    sp = stream.cuda_stream
    ctx = bp.Context(0)

    def step():
        ctx.feasible_dev(C, m, d_res.data_ptr(), len(unpacked), d_unp.data_ptr(), d_out.data_ptr(), sp,
                         flags=bp.BP_NO_EARLY_EXIT)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    rec = bp.bounds_to_dict(np.frombuffer(d_out.cpu().numpy().tobytes(), dtype=bp.BOUNDS_DTYPE)[0])
    assert rec["status"] == 0, rec
    r = rec["r"]
    evals_per_step = rec["evals"]

    # timed region: K whole steps, inputs resident in HBM
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt * 1e3 / args.steps

    # stage timing of the same step (kernels launched one by one, HIP events on this stream)
    ctx.set_timing(True)
    prep_ms, sweep_ms, fin_ms = [], [], []
    for _ in range(max(5, args.steps // 2)):
        step()
        a, b, c = ctx.stage_times()
        prep_ms.append(a)
        sweep_ms.append(b)
        fin_ms.append(c)
    ctx.set_timing(False)
    sweep_avg = float(np.mean(sweep_ms))

    import oracle as O  # ranges only (the bench's oracle leg)
    ops = 0.0
    for name, d in zip(DFF_NAMES, O.DFFS):
        lo, hi = O.default_range(d, C)
        ops += OPS_PER_EVAL[name] * r * max(0, hi - lo + 1)
    achieved = ops / (sweep_avg * 1e-3)

    # plain single-check latency on the small partial packing (host in, host out)
    lat = []
    smalls = [W.small_partial_packing(seed=s) for s in range(64)]
    for i in range(args.latency_checks):
        Cs, ms_, rs, us = smalls[i % len(smalls)]
        t1 = time.perf_counter()
        ctx.feasible(Cs, rs, us)
        lat.append((time.perf_counter() - t1) * 1e6)

    line = {
        "metric": "(item x param) bound evals/s + feasibility checks/s, batched vs plain; p99 us",
        "value": evals_per_step * args.steps / dt,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (seeded)",
        "config": {"workload": "single large residual instance: n=10000 sizes U[C/10,C/2], C=100000, "
                               "m=4000 residual capacities U[C/2,C], full parameter sweeps (exact, no VB2 cut)",
                   "r": r, "evals_per_step": evals_per_step, "parallelism": "single GPU"},
        "checks_per_s": args.steps / dt,
        "stages_ms": {"prep": float(np.mean(prep_ms)), "sweep": sweep_avg, "finalize": float(np.mean(fin_ms))},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_VALU / 1e12, "unit": "TOP/s",
                     "frac": achieved / PEAK_VALU, "traffic": None, "kernel": "k_sweep",
                     "ops_per_eval": OPS_PER_EVAL},
        "plain_small_check_us": {"p50": percentile(lat, 50), "p99": percentile(lat, 99), "n": len(lat),
                                 "workload": "n=50 sizes U[20,100], m=20, C=150, 30% pre-packed; host in/out"},
        "verdict": rec["verdict"], "lb": rec["lb"],
    }
    if not args.no_cpu_baseline:
        import oracle as O
        items = O.residual_reduce(C, residual, unpacked)
        line["cpu_baseline"] = cpu_baseline(C, items, args.cpu_seconds)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
