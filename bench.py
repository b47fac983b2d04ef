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
# counted in the inner loops of the sweep kernel as built for gfx950 with 2
# parameters per lane, the default shape.  Weights from the measured issue
# rates (profiles/valu_rates_gfx950.txt, `bench.py --valu-rates`): 32-bit
# add, sub, and, xor and shifts issue at 1.69-1.88x the full rate and count
# 1/2; v_mul_hi_u32, v_mad_u64_u32, v_add3_u32, v_sad_u32, compares, selects
# and fp64 issue at 0.90-0.98x and count 1.  Per evaluation:
#   MT   v_sub_u32, v_ashrrev_i32, v_and_b32 (1/2 each), 1/2 v_add3_u32      = 2.0
#   RAD2 two families of v_sub_u32 + v_lshrrev_b32 (1/2 each), 1/2 v_add3_u32 x 2 = 3.0
#   FS1  2 v_fma_f64, 2 v_mul_f64, 2 v_add_f64, 2 v_cndmask_b32, v_floor_f64,
#        v_cmp_eq_f64, 1/2 conversion                                        = 10.25
#   CCM1 v_mul_hi_u32, v_lshrrev_b32 (1/2), 1/2 v_add3_u32                  = 2.0
#   VB2  v_mul_hi_u32, v_mad_u64_u32, 1/2 v_add3_u32                        = 2.5
#   BJ1  v_mul_hi_u32, v_lshrrev_b32 (1/2), v_mad_u64_u32, v_sad_u32,
#        1/2 v_add3_u32                                                      = 4.0
# (v_add3_u32 adds two items' increments at once, hence 1/2 per evaluation.)
# Where the quotient's product is at most 2^32 one high multiply gives it
# (CCM1: a lambda, BJ1: w lambda over the tile's largest lambda; VB2: a c),
# and the evaluation drops the shift or the v_mad_u64_u32:
#   CCM1 v_mul_hi_u32, 1/2 v_add3_u32                                       = 1.5
#   VB2  v_mul_hi_u32, 1/2 v_add3_u32                                       = 1.5
#   BJ1  v_mul_hi_u32, v_mad_u64_u32, v_sad_u32, 1/2 v_add3_u32             = 3.5
# and BJ1 over tiles whose parameters all exceed c/2 (floor(c / lambda) = 1:
# f is a clamp, two absolute differences): 2 v_sad_u32                      = 2.0
OPS_PER_EVAL = {"MT": 2.0, "RAD2": 3.0, "FS1": 10.25, "CCM1": 2.0, "VB2": 2.5, "BJ1": 4.0}
OPS_PER_EVAL_SHORT = {"CCM1": 1.5, "VB2": 1.5, "BJ1": 3.5}
OPS_PER_EVAL_BJ1_UPPER = 2.0
PEAK_VALU = 256 * 64 * 2.4e9  # full-rate lane-instructions/s: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz
DFF_NAMES = ("MT", "RAD2", "FS1", "CCM1", "VB2", "BJ1")


def log(msg: str) -> None:
    """Progress line on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def percentile(xs, p):
    import numpy as np
    return float(np.percentile(np.asarray(xs), p)) if len(xs) else None


def cpu_baseline(C, items, target_s: float):
    """The oracle as it stands, on a strided sample of every sweep's parameters."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor

    import oracle as O

    O._load()
    host = host_cpu()
    # every core this process may run on, up to the 16-core share one GPU's process gets on the box
    threads = max(1, min(16, host["affinity"]))
    ranges = [(d, *O.default_range(d, C)) for d in O.DFFS]
    ranges = [(d, lo, hi) for d, lo, hi in ranges if lo <= hi]

    def pass_evals(stride):
        t0 = time.perf_counter()
        ev = sum(O.dff_bound_strided(d, C, items, lo, hi, stride)[2] for d, lo, hi in ranges)
        return ev, time.perf_counter() - t0

    # probe on every 1024th parameter (single thread), then size the sample to about target_s core-seconds
    ev_probe, t_probe = pass_evals(1024)
    full_core_s = t_probe * 1024
    stride = max(1, int(round(full_core_s / target_s)))
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
            "nproc": host["nproc"], "affinity": host["affinity"], "cpu_model": host["model"],
            "sample": f"every {stride}th parameter of each of the six sweeps of the same instance "
                      f"({evals} (item, parameter) evaluations in {dt:.2f} s wall on {threads} threads of "
                      f"{host['nproc']} logical CPUs, {host['affinity']} in this process's affinity, "
                      f"{host['model']}; a single-thread probe puts the whole instance at {full_core_s:.1f} core-s)"}


def tuning_cache_path() -> str:
    """File of the autotuner's cache: $BP_TUNING_CACHE, else under ~/.cache
    (or the temporary directory when that is not writable)."""
    env = os.environ.get("BP_TUNING_CACHE")
    if env:
        return env
    for base in (os.path.expanduser("~/.cache"), os.environ.get("TMPDIR", "/tmp")):
        try:
            os.makedirs(base, exist_ok=True)
            path = os.path.join(base, "libbp_tuning.txt")
            with open(path, "a"):
                pass
            return path
        except OSError:
            continue
    return None


def host_cpu():
    """Logical CPU count, the CPUs this process may use, and the CPU model."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = os.cpu_count() or 1
    return {"nproc": os.cpu_count() or 1, "affinity": aff, "model": model}


def plain_latency(bp, W, ctx, checks: int):
    """Plain single-check latency on the small partial packing (host in, host
    out): one bp_feasible call through ctypes with its arguments marshalled
    beforehand, so the figure is the library call and not numpy conversions.
    Returns the per-call microseconds."""
    import ctypes

    import numpy as np

    lib = bp.load()
    lat = []
    smalls = []
    for s in range(64):
        Cs, ms_, rs, us = W.small_partial_packing(seed=s)
        rs = np.ascontiguousarray(rs, dtype=np.int32)
        us = np.ascontiguousarray(us, dtype=np.int32)
        smalls.append((Cs, len(rs), rs.ctypes.data_as(bp._P32), us.ctypes.data_as(bp._P32), len(us), rs, us))
    v32, lb64, rec_small = ctypes.c_int32(0), ctypes.c_int64(0), bp.bp_bounds()
    pv, plb, prec = ctypes.byref(v32), ctypes.byref(lb64), ctypes.byref(rec_small)
    fz = lib.bp_feasible
    for i in range(checks):
        Cs, ms_, prs, pus, nus, _, _ = smalls[i % len(smalls)]
        t1 = time.perf_counter()
        st = fz(ctx.handle, Cs, ms_, prs, pus, nus, 0, pv, plb, prec)
        lat.append((time.perf_counter() - t1) * 1e6)
        if st != 0:
            raise bp.BpError(st, lib.bp_last_error().decode())
    return lat


def valu_rates(blocks_per_cu: int = 8, iters: int = 4000, reps: int = 3):
    """Issue rate of each opcode of the sweep's inner loops, measured by the
    microbenchmark library (hand-written gfx950 kernels, one opcode each on
    eight independent chains per lane), as lane-operations/s and as a
    fraction of the full rate PEAK_VALU."""
    import ctypes

    import paper_2402_14821_amd as bp

    bp._preload_torch_hip_runtime()
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2402_14821_amd", "libbp_ubench.so"))
    lib.bpu_num_ops.restype = ctypes.c_int
    lib.bpu_op_name.restype = ctypes.c_char_p
    lib.bpu_op_name.argtypes = [ctypes.c_int]
    lib.bpu_valu_rate.argtypes = [ctypes.c_int] * 5 + [ctypes.POINTER(ctypes.c_double)] * 3
    lib.bpu_valu_rate.restype = ctypes.c_int
    rows = []
    for op in range(lib.bpu_num_ops()):
        rate, ms, per_lane = ctypes.c_double(0), ctypes.c_double(0), ctypes.c_double(0)
        st = lib.bpu_valu_rate(0, op, blocks_per_cu, iters, reps, ctypes.byref(rate), ctypes.byref(ms),
                               ctypes.byref(per_lane))
        name = lib.bpu_op_name(op).decode()
        if st != 0:
            raise RuntimeError(f"microbenchmark of {name} failed with HIP error {st}")
        rows.append({"op": name, "lane_ops_per_s": rate.value, "frac_of_full_rate": rate.value / PEAK_VALU,
                     "ms": ms.value})
        log(f"valu rate {name}: {rate.value / PEAK_VALU:.3f} of the full rate")
    return {"full_rate_lane_ops_per_s": PEAK_VALU, "blocks_per_cu": blocks_per_cu, "waves_per_cu": 4 * blocks_per_cu,
            "insts_per_lane": iters * 128, "reps": reps, "rates": rows}


def sweep_ops(bp, C, items, lanes_params: int = 2):
    """Algorithmic VALU slots of the six sweeps of one instance (exact ranges,
    as the library's own bp_default_sweep states them): every parameter
    times the sizes its sweep streams (MT, RAD2, CCM1 and VB2 the big and
    small classes, FS1 and BJ1 every size strictly between 0 and c; sizes 0,
    c/2 and c are counted, not streamed), each evaluation at the weight of
    the form the kernel takes for it: tiles of 64 x lanes_params parameters
    from the range's start, and per tile the sizes whose quotient fits one
    high multiply on the short form."""
    import numpy as np

    C = int(C)
    w = np.asarray(items, dtype=np.int64)
    w = w[(w > 0) & (w < C)]
    a = np.sort(np.where(2 * w > C, C - w, w)[2 * w != C])  # CCM1 and VB2 stream these (big and small)
    ws = np.sort(w)                                           # BJ1 streams the sizes 0 < w < c
    sw = bp.default_sweep(C)
    width = 64 * lanes_params
    ops = 0.0
    for j, name in enumerate(DFF_NAMES):
        b = bp.BP_MT + j
        lo, hi = int(sw.lo[b]), int(sw.hi[b])
        if hi < lo:
            continue
        if name not in OPS_PER_EVAL_SHORT:
            ops += OPS_PER_EVAL[name] * (len(ws) if name == "FS1" else len(a)) * (hi - lo + 1)
            continue
        full, short = OPS_PER_EVAL[name], OPS_PER_EVAL_SHORT[name]
        vals = ws if name == "BJ1" else a
        if name == "VB2":
            n_short = np.searchsorted(vals, 0xFFFFFFFF // C, side="right")
            ops += (hi - lo + 1) * (short * n_short + full * (len(vals) - n_short))
            continue
        t0 = np.arange(lo, hi + 1, width, dtype=np.int64)
        t1 = np.minimum(t0 + width - 1, hi)
        lim = np.where(t0 >= 2, 0xFFFFFFFF // t1, -1)
        n_short = np.searchsorted(vals, lim, side="right")
        per = short * n_short + full * (len(vals) - n_short)
        if name == "BJ1":
            per = np.where(2 * t0 > C, OPS_PER_EVAL_BJ1_UPPER * len(vals), per)
        ops += float(((t1 - t0 + 1) * per).sum())
    return ops


def kernel_source_sha256() -> str:
    import hashlib

    src = os.path.join(ROOT, "paper_2402_14821_amd", "csrc", "bp_kernels.hip")
    with open(src, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def load_profile(name: str):
    """key: value pairs of a counter summary in profiles/, or None when it is
    missing or the kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("#") and "sha256" in line and ":" in line:
                vals["kernel_source_sha256"] = line.rsplit(":", 1)[1].strip()
            elif ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_source_sha256():
        return None
    return vals


def load_traffic(kernel: str):
    """HBM bytes per launch of a kernel, from the counter summary in profiles/,
    or None when the kernel source changed since the counters were taken."""
    vals = load_profile(f"{kernel}_traffic.txt")
    if not vals or "hbm_bytes_per_launch" not in vals:
        return None
    return float(vals["hbm_bytes_per_launch"])


def load_valu_insts(kernel: str):
    """Wave-level VALU instructions per launch (SQ_INSTS_VALU), or None."""
    vals = load_profile(f"{kernel}_large_residual_sq_counters.txt")
    if not vals or "SQ_INSTS_VALU" not in vals:
        return None
    return float(vals["SQ_INSTS_VALU"])


def bench_batched(bp, W, ctx, seed: int = 2, count: int = 4096, reps: int = 3, plain_max: int = 4096,
                  segments: bool = True, tuning_cache: str | None = None):
    """Uneven batch: one batched call vs one plain call per instance (host in, host out)."""
    import numpy as np

    b = W.uneven_batch(seed, count=count)
    items_list = [b.instance(i)[2] for i in range(len(b))]
    Cs, ks = b.C, b.k
    out = ctx.lower_bounds_batch(Cs, ks, items_list)  # warm-up (sizes the workspaces, captures the graph)
    assert (out["status"] == 0).all()
    # the default shape, then the autotuner's (cached on disk by batch shape)
    t0 = time.perf_counter()
    ctx.lower_bounds_batch(Cs, ks, items_list)
    t_default = time.perf_counter() - t0
    default_tuning = ctx.get_tuning()
    t0 = time.perf_counter()
    tuned, tuned_ms, from_cache = ctx.autotune_batch_cached(Cs, ks, items_list, tuning_cache, reps=1)
    t_tune = time.perf_counter() - t0
    ctx.lower_bounds_batch(Cs, ks, items_list)  # warm-up of the tuned shape
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        out = ctx.lower_bounds_batch(Cs, ks, items_list)
        ts.append(time.perf_counter() - t0)
    t_batch = min(ts)
    evals = int(out["evals"].sum())
    # the sweep kernel of the same batch, timed with HIP events on the context's stream
    ctx.set_timing(True)
    for _ in range(reps):
        ctx.lower_bounds_batch(Cs, ks, items_list)
    (prep_ms, sweep_ms, fin_ms), runs = ctx.stage_times(with_runs=True)
    ctx.set_timing(False)
    lpl = int(ctx.get_tuning()["lanes_params"])
    ops = sum(sweep_ops(bp, int(c), it, lpl) for c, it in zip(Cs, items_list))
    fails = int((out["verdict"] == 0).sum())
    assert np.array_equal(out["verdict"] == 0, b.expect_fail), "batched verdicts differ from the construction"
    # plain: one call per instance, each synchronous, with the default shape
    # (the batch's tuned shape is chosen for a whole batch)
    n_plain = min(plain_max, len(b))
    per = np.zeros(n_plain)
    ctx.set_tuning(*[default_tuning[k] for k in ("lanes_params", "waves_per_cu", "tasks_per_wave", "min_chunk")])
    for i in range(n_plain):
        C, k, it = b.instance(i)
        t0 = time.perf_counter()
        ctx.lower_bounds(C, k, it)
        per[i] = time.perf_counter() - t0
    ctx.set_tuning(*[tuned[k] for k in ("lanes_params", "waves_per_cu", "tasks_per_wave", "min_chunk")])
    classes = {}
    for c in sorted(set(int(x) for x in Cs)):
        idx = np.flatnonzero(Cs[:n_plain] == c)
        sub = b.subset(np.flatnonzero(Cs == c))
        sub_items = [sub.instance(i)[2] for i in range(len(sub))]
        ctx.lower_bounds_batch(sub.C, sub.k, sub_items)  # warm-up
        tb = []
        for _ in range(reps):
            t0 = time.perf_counter()
            ctx.lower_bounds_batch(sub.C, sub.k, sub_items)
            tb.append(time.perf_counter() - t0)
        plain = float(len(idx) / per[idx].sum())
        batched = float(len(sub) / min(tb))
        classes[str(c)] = {"instances": int(len(idx)), "plain_checks_per_s": plain,
                           "plain_mean_us": float(per[idx].mean() * 1e6),
                           "batched_instances": int(len(sub)), "batched_checks_per_s": batched,
                           "batched_over_plain": batched / plain}
    plain_rate = n_plain / per.sum()
    seg = None
    if segments:
        try:
            seg = bench_batched_segments(bp, b, ctx, Cs, ks, items_list, out, t_batch, n_plain, reps, default_tuning)
        except bp.BpError as e:
            seg = {"error": str(e)}

    return {"workload": f"{count} instances, n lognormal(median 400, sigma 1) clipped to [50, 5000], "
                        "C in {1e3, 1e4, 1e6}, sizes U[1, C], 40% built to fail; host in/out",
            "batched_s": t_batch, "batched_checks_per_s": len(b) / t_batch, "batched_evals_per_s": evals / t_batch,
            "plain_checks_per_s": plain_rate, "batched_over_plain": (len(b) / t_batch) / plain_rate,
            "evals": evals, "fails": fails, "per_class": classes, "segments": seg,
            "stages_ms": {"prep": prep_ms, "sweep": sweep_ms, "finalize": fin_ms, "runs": runs},
            "sweep_roofline": {"bound": "alu", "achieved": ops / (sweep_ms * 1e-3) / 1e12, "peak": PEAK_VALU / 1e12,
                               "unit": "TOP/s", "frac": ops / (sweep_ms * 1e-3) / PEAK_VALU},
            "tuning": ctx.get_tuning(), "tuning_default": default_tuning,
            "tuning_from_cache": from_cache, "tuning_s": t_tune, "tuning_sweep_ms": tuned_ms,
            "batched_s_default_shape": t_default}


def bench_batched_segments(bp, b, ctx, Cs, ks, items_list, out, t_batch, n_plain, reps, default_tuning):
    """The uneven batch and its plain calls again with the segment sums (same records)."""
    import numpy as np

    seg_sweeps = [bp.default_sweep(int(c), 0, 0, bp.BP_SWEEP_SEGMENTS) for c in Cs]
    out_s = ctx.lower_bounds_batch(Cs, ks, items_list, seg_sweeps)
    if not (np.array_equal(out_s["value"], out["value"]) and np.array_equal(out_s["argmax_lambda"], out["argmax_lambda"])):
        return {"error": "segment records differ from the dense records"}
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        ctx.lower_bounds_batch(Cs, ks, items_list, seg_sweeps)
        ts.append(time.perf_counter() - t0)
    t_batch_seg = min(ts)
    per_s = np.zeros(n_plain)
    tuned = ctx.get_tuning()
    ctx.set_tuning(*[default_tuning[k] for k in ("lanes_params", "waves_per_cu", "tasks_per_wave", "min_chunk")])
    for i in range(n_plain):
        C, k, it = b.instance(i)
        t0 = time.perf_counter()
        ctx.lower_bounds(C, k, it, seg_sweeps[i])
        per_s[i] = time.perf_counter() - t0
    ctx.set_tuning(*[tuned[k] for k in ("lanes_params", "waves_per_cu", "tasks_per_wave", "min_chunk")])
    plain = n_plain / per_s.sum()
    return {"batched_s": t_batch_seg, "batched_checks_per_s": len(b) / t_batch_seg, "plain_checks_per_s": plain,
            "batched_over_plain": (len(b) / t_batch_seg) / plain, "batched_speedup_vs_dense": t_batch / t_batch_seg,
            "per_class_plain_checks_per_s": {
                str(c): float((Cs[:n_plain] == c).sum() / per_s[Cs[:n_plain] == c].sum())
                for c in sorted(set(int(x) for x in Cs))}}


def triplet_windows(bp, C: int, width: int = 8192):
    """Low-end and high-end windowed sweeps of capacity C: every DFF range
    longer than two windows keeps its first (resp. last) `width` parameters;
    shorter ranges and L2 stay whole."""
    full = bp.default_sweep(int(C))
    sides = []
    for side in (0, 1):
        lo, hi = [0] * bp.BP_NB, [-1] * bp.BP_NB
        for b in range(1, bp.BP_NB):
            dlo, dhi = int(full.lo[b]), int(full.hi[b])
            if b == bp.BP_L2 or dhi - dlo + 1 <= 2 * width:
                lo[b], hi[b] = (dlo, dhi) if dlo <= dhi else (1, 0)
            else:
                lo[b], hi[b] = (dlo, dlo + width - 1) if side == 0 else (dhi - width + 1, dhi)
        sides.append(bp.make_sweep(lo, hi))
    return sides


def bench_triplets(bp, W, ctx, seed: int = 5, count: int = 1024, reps: int = 3):
    """Triplet-tight batch: 1 024 instances, m ~ U[300, 1000] bins of three sizes
    in (C/4, C/2) summing exactly to C, C ~ U[10^6, 2^31 - 1], half missing a
    bin; every DFF range cut to windows of 8 192 at both ends, L2 exact."""
    import numpy as np

    tb = W.triplet_batch(seed, count=count)
    Cs, ks, its, sweeps, owner = [], [], [], [], []
    for i in range(len(tb)):
        C, k, items = tb.instance(i)
        for sw in triplet_windows(bp, C):
            Cs.append(C)
            ks.append(k)
            its.append(items)
            sweeps.append(sw)
            owner.append(i)
    Cs, ks = np.array(Cs), np.array(ks)
    out = ctx.lower_bounds_batch(Cs, ks, its, sweeps)  # warm-up
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        out = ctx.lower_bounds_batch(Cs, ks, its, sweeps)
        ts.append(time.perf_counter() - t0)
    t = min(ts)
    verdict = np.ones(len(tb), dtype=np.int32)
    for j, i in enumerate(owner):
        verdict[i] &= out["verdict"][j]
    assert np.array_equal(verdict == 0, tb.expect_fail), "triplet verdicts differ from the construction"
    evals = int(out["evals"].sum())
    return {"workload": "1024 triplet-tight instances, m~U[300,1000], n=3m, C~U[1e6,2^31-1], half missing a bin; "
                        "DFF ranges cut to windows of 8192 at both ends, L2 exact; host in/out",
            "instances": len(tb), "launch_instances": len(Cs), "batched_s": t, "checks_per_s": len(tb) / t,
            "evals": evals, "evals_per_s": evals / t, "fails": int((verdict == 0).sum())}


def bench_fidelity(bp, W, ctx, reps: int = 3):
    """Paper-fidelity study.  (1) The paper's VB2 cut (Sec. 4) against the
    exact range: bounds and verdicts it changes, and time, on the single large
    instance and the uneven batch.  (2) The order of the functions (Alg. 2
    visits MT, RAD2, FS1, CCM1, VB2, BJ1 and returns after the first bound
    above k; Table 1 ranks CCM1 strongest) against early exit: on instances
    that only a DFF refutes (k = L1 < the best bound), the work done before
    the refutation, on the GPU per schedule order and in Alg. 2's
    sequential model."""
    import numpy as np

    res = {}
    # (1) VB2 cut on the large instance
    C, m, residual, unpacked = W.large_residual(seed=1)
    items = ctx.residual_reduce(C, residual, unpacked)
    rows = {}
    for name, flags in (("exact", 0), ("paper_vb2_cut", bp.BP_SWEEP_PAPER_VB2_CLAMP)):
        sw = bp.default_sweep(C)
        sw.flags = flags
        rec = ctx.lower_bounds(C, m, items, sw)
        t0 = time.perf_counter()
        for _ in range(reps):
            rec = ctx.lower_bounds(C, m, items, sw)
        rows[name] = {"ms": (time.perf_counter() - t0) * 1e3 / reps, "vb2": int(rec["value"][bp.BP_VB2]),
                      "vb2_argmax": int(rec["argmax"][bp.BP_VB2]), "lb": rec["lb"], "evals": rec["evals"]}
    res["vb2_cut_large_instance"] = rows
    # (1') VB2 cut on the uneven batch
    b = W.uneven_batch(2, count=4096)
    its = [b.instance(i)[2] for i in range(len(b))]
    ex = ctx.lower_bounds_batch(b.C, b.k, its)
    sweeps_cut = []
    for c in b.C:
        sw = bp.default_sweep(int(c))
        sw.flags = bp.BP_SWEEP_PAPER_VB2_CLAMP
        sweeps_cut.append(sw)
    cut = ctx.lower_bounds_batch(b.C, b.k, its, sweeps_cut)
    res["vb2_cut_uneven_batch"] = {
        "instances": len(b),
        "vb2_lower": int((cut["value"][:, bp.BP_VB2] < ex["value"][:, bp.BP_VB2]).sum()),
        "lb_lower": int((cut["lb"] < ex["lb"]).sum()),
        "verdicts_changed": int((cut["verdict"] != ex["verdict"]).sum()),
        "evals_exact": int(ex["evals"].sum()), "evals_cut": int(cut["evals"].sum())}
    # (2) order against early exit, on instances only a DFF refutes
    pool = W.uneven_batch(7, count=2048, capacities=(1_000, 10_000))
    pits = [pool.instance(i)[2] for i in range(len(pool))]
    full = ctx.lower_bounds_batch(pool.C, pool.k, pits)
    dff_best = full["value"][:, bp.BP_MT:].max(axis=1)
    l1 = full["value"][:, bp.BP_L1]
    sel = np.flatnonzero((dff_best > l1) & (full["value"][:, bp.BP_L2] <= l1))
    sub = pool.subset(sel)
    sub_its = [sub.instance(i)[2] for i in range(len(sub))]
    k = l1[sel].astype(np.int32)  # L1 and L2 pass: the verdict needs a DFF
    vals = full["value"][sel]
    names = ["MT", "RAD2", "FS1", "CCM1", "VB2", "BJ1"]
    orders = {"alg2": [bp.BP_MT, bp.BP_RAD2, bp.BP_FS1, bp.BP_CCM1, bp.BP_VB2, bp.BP_BJ1],
              "table1": [bp.BP_CCM1, bp.BP_MT, bp.BP_BJ1, bp.BP_VB2, bp.BP_FS1, bp.BP_RAD2],
              "longest_first": None}
    gpu = {}
    exhaustive = 0
    for name, order in orders.items():
        ctx.set_order(order)
        ctx.feasible_batch(sub.C, k, sub_its)  # warm-up
        t0 = time.perf_counter()
        for _ in range(reps):
            v, lb, rec = ctx.feasible_batch(sub.C, k, sub_its, records=True)
        dt = (time.perf_counter() - t0) / reps
        assert (v == 0).all(), "every selected instance is refuted by a DFF"
        exhaustive = int(rec["evals"].sum())
        gpu[name] = {"batched_s": dt, "evals_done": int(rec["evals_done"].sum()),
                     "early_exits": int(rec["early_exit"].sum())}
    ctx.set_order(None)
    # sequential Alg. 2 model: bounds in order, each over its whole range, stop after the first above k
    ranges = {}
    seq = {}
    for name, order in (("alg2", orders["alg2"]), ("table1", orders["table1"])):
        work = 0
        for j in range(len(sel)):
            C = int(sub.C[j])
            sw = ranges.setdefault(C, bp.default_sweep(C))
            r = len(sub_its[j])
            for bd in order:
                work += r * max(0, int(sw.hi[bd]) - int(sw.lo[bd]) + 1)
                if vals[j][bd] > k[j]:
                    break
        seq[name] = work
    res["order_vs_early_exit"] = {
        "instances": int(len(sel)), "pool": len(pool),
        "refuting_function_counts": {n: int((vals[:, bp.BP_MT + i] > k).sum()) for i, n in enumerate(names)},
        "gpu": gpu, "sequential_alg2_work": seq, "exhaustive_work": exhaustive}
    return res


def bench_search(bp, W, ctx, time_limit: float = 0.5, n: int = 100, ablation: bool = False):
    """The resolution procedure of Sec. 5 around the check, on synthetic
    Weibull instances built as the paper builds them (scale 1000, c = sigma x
    the largest size): n = 100, shape 0.5 .. 5.0 in steps of 0.5, sigma 1.0 ..
    2.0 in steps of 0.2, one seed per shape (60 instances; the paper has 552
    with n in {100, 200} and shape steps of 0.1).  Every instance is solved
    with the DFF check (bp_feasible on the GPU) and with L1 and L2 only
    (bp_lower_bounds with empty DFF ranges, on the GPU), under the same time
    limit each; with ablation, the DFF search again without the dominance
    rules and without the symmetry rules (the paper's ablation table)."""
    import numpy as np

    shapes = [0.5 * i for i in range(1, 11)]
    sigmas = [1.0, 1.2, 1.4, 1.6, 1.8, 2.0]
    modes = [("DFFs", bp.BP_SOLVE_DFFS, 0), ("L2", bp.BP_SOLVE_L2, 0)]
    if ablation:
        modes += [("DFFs_no_dominance", bp.BP_SOLVE_DFFS, bp.BP_SOLVE_OFF_FILL | bp.BP_SOLVE_OFF_SINGLE),
                  ("DFFs_no_symmetry", bp.BP_SOLVE_DFFS, bp.BP_SOLVE_OFF_SYMMETRY),
                  ("DFFs_no_knapsack", bp.BP_SOLVE_DFFS, bp.BP_SOLVE_OFF_KNAPSACK)]
    insts = []
    for shape in shapes:
        for sigma in sigmas:
            C, sizes = W.weibull_instance(seed=int(round(shape * 10)), n=n, shape=shape, sigma=sigma)
            insts.append((shape, sigma, C, sizes))
    bp.solve(insts[0][2], insts[0][3], ctx=ctx, max_nodes=1)  # warm-up (plans, graphs)
    out = {"workload": f"{len(insts)} Weibull instances, n={n}, shape 0.5..5.0 step 0.5, sigma 1.0..2.0 step 0.2, "
                       "scale 1000, seed = 10 x shape", "time_limit_s": time_limit, "modes": {}}
    solved_by = {}
    for name, mode, disable in modes:
        agg = {"solved": 0, "solved_time_s": 0.0, "solved_nodes": 0, "nodes": 0, "checks": 0, "check_fails": 0,
               "filter_fails": 0, "check_s": 0.0, "total_s": 0.0, "root_lb_sum": 0}
        solved_by[name] = set()
        for idx, (shape, sigma, C, sizes) in enumerate(insts):
            res, bin_of = bp.solve(C, sizes, ctx=ctx, mode=mode, time_limit_s=time_limit, disable=disable)
            load = np.bincount(bin_of, weights=sizes, minlength=res["bins"])
            assert load.max() <= C and bin_of.max() < res["bins"], "invalid packing"
            agg["nodes"] += res["nodes"]
            agg["checks"] += res["checks"]
            agg["check_fails"] += res["check_fails"]
            agg["filter_fails"] += res["filter_fails"]
            agg["check_s"] += res["check_seconds"]
            agg["total_s"] += res["seconds"]
            agg["root_lb_sum"] += res["lower"]
            if res["status"] == bp.BP_SOLVE_OPTIMAL:
                agg["solved"] += 1
                agg["solved_time_s"] += res["seconds"]
                agg["solved_nodes"] += res["nodes"]
                solved_by[name].add(idx)
        agg["check_us_mean"] = agg["check_s"] * 1e6 / max(1, agg["checks"])
        agg["check_share"] = agg["check_s"] / max(1e-12, agg["total_s"])
        out["modes"][name] = agg
        log(f"search leg {name}: {agg['solved']}/{len(insts)} solved")
    out["solved_only_by_DFFs"] = len(solved_by["DFFs"] - solved_by["L2"])
    out["solved_only_by_L2"] = len(solved_by["L2"] - solved_by["DFFs"])
    both = solved_by["DFFs"] & solved_by["L2"]
    out["both_solved"] = len(both)
    out["paper_weibull_table"] = {"instances": 552, "L2_solved": 375, "DFFs_GPU_solved": 418,
                                  "DFFs_CPU_solved": 402, "time_limit_s": 600,
                                  "note": "the paper's own runs (RTX 3080, 10 min per instance); context only"}
    return out


def per_bound_table(bp, W, ctx, reps: int = 5):
    """Sweep stage time of each DFF bound alone on the single large residual
    instance, dense and segment form (the other ranges empty), from the
    library's stage events; both forms must give the same bounds."""
    C, m, residual, unpacked = W.large_residual(seed=1)
    items = ctx.residual_reduce(C, residual, unpacked)
    full = bp.default_sweep(C)
    rows = []
    for name, bounds in [(n, {bp.BP_MT + j}) for j, n in enumerate(DFF_NAMES)] + [("ALL", set(range(bp.BP_MT, 8)))]:
        row = {"bound": name}
        vals = []
        for form, flags in (("dense", 0), ("segments", bp.BP_SWEEP_SEGMENTS)):
            lo = [full.lo[b] if b in bounds else 1 for b in range(8)]
            hi = [full.hi[b] if b in bounds else 0 for b in range(8)]
            sw = bp.make_sweep(lo, hi, flags)
            rec = ctx.lower_bounds(C, m, items, sw)  # warm-up (plan, graph)
            ctx.set_timing(True)
            for _ in range(reps):
                ctx.lower_bounds(C, m, items, sw)
            (p_ms, s_ms, _), _ = ctx.stage_times(with_runs=True)
            ctx.set_timing(False)
            row[form] = {"prep_us": p_ms * 1e3, "sweep_us": s_ms * 1e3}
            vals.append(list(rec["value"]))
        row["same_bounds"] = vals[0] == vals[1]
        rows.append(row)
        log(f"per-bound {name} done")
    return {"workload": "single large residual instance, each DFF bound's full range alone", "r": int(len(items)),
            "reps": reps, "rows": rows}


def bench_served(bp, W, ctx, rate: float, duration: float, seed: int, budget: int = 8 << 30, flags: int = 0,
                 max_slots: int = 8192, warmup: float = 0.25):
    """Open-loop Poisson arrivals of the simulated search's requests into a
    bp_queue.  Roots go in as partial packings (checked exhaustively: the
    search expands them), children as (parent ticket, commits) without their
    instances; a request whose parent was rejected is dropped with its
    subtree.  A shorter stream of another seed first warms the queue (its
    contexts' launch shapes and buffers) and is not counted.  Latency from
    the library's clock; evaluations as performed."""
    import ctypes
    import threading

    import numpy as np

    lib = bp.load()
    q = bp.Queue(ctx, budget, max_slots)

    def run_stream(reqs):
        m_of = {}
        structs, keep = [], []
        for i, r in enumerate(reqs):
            if r.parent < 0:
                res = np.ascontiguousarray(r.residual, dtype=np.int32)
                unp = np.ascontiguousarray(r.unpacked, dtype=np.int32)
                keep.append((res, unp))
                m_of[i] = len(res)
                structs.append(bp.bp_request(r.C, len(res), len(unp), res.ctypes.data_as(bp._P32),
                                             unp.ctypes.data_as(bp._P32), i, flags | bp.BP_NO_EARLY_EXIT, 0, 0,
                                             None, 0, 0))
            else:
                m_of[i] = m_of[r.parent]
                cm = (bp.bp_commit * max(1, len(r.commits)))(*[bp.bp_commit(w, b) for w, b in r.commits])
                keep.append(cm)
                structs.append(bp.bp_request(r.C, m_of[i], 0, None, None, i, flags, 0, 0, cm, len(r.commits), 0))
        results = []
        done = threading.Event()
        submitted = [0]

        def poller():
            arr = (bp.bp_result * 4096)()
            got = ctypes.c_int32(0)
            while True:
                lib.bp_queue_poll(q.handle, ctypes.cast(arr, ctypes.c_void_p), 4096, ctypes.byref(got), 2000)
                for j in range(got.value):
                    a = arr[j]
                    results.append((a.tag, a.submit_us, a.done_us, a.status, a.bounds.evals, a.bounds.evals_done,
                                    a.from_parent, a.verdict))
                if done.is_set() and len(results) >= submitted[0]:
                    return

        th = threading.Thread(target=poller, daemon=True)
        th.start()
        # the open-loop submitter runs natively (bp_queue_replay): a Python
        # loop cannot keep 5 us between arrivals
        n = len(reqs)
        arr = (bp.bp_request * n)(*structs)
        arrival = np.ascontiguousarray([r.t for r in reqs], dtype=np.float64)
        parent = np.ascontiguousarray([r.parent for r in reqs], dtype=np.int64)
        tickets = np.zeros(n, dtype=np.uint64)
        status = np.zeros(n, dtype=np.int32)
        late_c = ctypes.c_double(0)
        submitted[0] = n  # an upper bound until the replay returns
        t0 = time.perf_counter()
        st = lib.bp_queue_replay(q.handle, ctypes.cast(arr, ctypes.c_void_p),
                                 arrival.ctypes.data_as(ctypes.c_void_p), parent.ctypes.data_as(ctypes.c_void_p), n,
                                 tickets.ctypes.data_as(ctypes.c_void_p), status.ctypes.data_as(ctypes.c_void_p),
                                 ctypes.byref(late_c))
        if st != 0:
            raise bp.BpError(st, lib.bp_last_error().decode())
        t_submit = time.perf_counter() - t0
        other = status[(status != 0) & (status != bp.BP_ERR_AGAIN) & (status != bp.BP_ERR_STATE)]
        if len(other):
            raise bp.BpError(int(other[0]), "replay submit failed")
        submitted[0] = int((status == 0).sum())
        done.set()
        th.join(timeout=120)
        t_end = time.perf_counter() - t0
        return results, status, late_c.value, t_submit, t_end, arrival

    t_gen = time.perf_counter()
    reqs = W.dfs_requests(seed, rate=rate, duration=duration, instances="roots")
    t_gen = time.perf_counter() - t_gen
    if warmup > 0:
        run_stream(W.dfs_requests(seed + 7919, rate=rate, duration=warmup, instances="roots"))
    s0 = q.stats()
    results, status, late, t_submit, t_end, arrival = run_stream(reqs)
    stats = q.stats()
    q.close()
    rejected = int((status == bp.BP_ERR_AGAIN).sum())
    dropped = int((status == bp.BP_ERR_STATE).sum())
    ok = [x for x in results if x[3] == 0]
    lat = np.array([d - s for _, s, d, *_ in ok])
    # the second half of the stream's arrivals: steady state
    late_half = np.array([d - s for tag, s, d, *_ in ok if arrival[tag] >= duration / 2])
    # the stream's span on the library's clock: first submit to last result
    span = (max(x[2] for x in ok) - min(x[1] for x in ok)) * 1e-6 if ok else t_end
    evals_nominal = sum(x[4] for x in ok)
    evals_done = sum(x[5] for x in ok)
    return {"rate_per_s": rate, "duration_s": duration, "warmup_s": warmup, "requests": len(reqs),
            "submitted": int((status == 0).sum()),
            "completed": int(len(ok)), "rejected": rejected, "dropped_with_rejected_parent": dropped,
            "checks_per_s": len(ok) / span, "evals_per_s": evals_done / span,
            "nominal_evals_per_s": evals_nominal / span, "span_s": span, "wall_s": t_end,
            "p50_us": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_us": float(np.percentile(lat, 99)) if len(lat) else None,
            "p99_us_second_half": float(np.percentile(late_half, 99)) if len(late_half) else None,
            "from_parent": int(stats["from_parent"] - s0["from_parent"]),
            "full_sweeps": int(stats["full_sweeps"] - s0["full_sweeps"]),
            "node_evictions": int(stats["node_evictions"] - s0["node_evictions"]),
            "batches": stats["batches"] - s0["batches"],
            "peak_bytes": stats["bytes_peak"], "max_slots": max_slots, "max_submit_lateness_s": late,
            "submit_s": t_submit, "generate_s": t_gen, "segments": bool(flags & bp.BP_SEGMENTS),
            "fails": int(sum(1 for x in ok if x[7] == 0)),
            "workload": "simulated search: roots n~U[200,5000], sizes U[C/20,C/2], C=10000, m = best-fit-decreasing "
                        "bins; children commit 1-3 items by decreasing best fit, 30% backtracking, a new root every "
                        "64 nodes; roots exhaustive, children from their parents' sums; HBM budget 8 GB; a 0.25 s "
                        "stream of another seed warms the queue first"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="core-seconds of oracle work to time")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--latency-checks", type=int, default=2000)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--per-bound", action="store_true",
                    help="only time each DFF sweep alone on the large instance, dense and segment form, and exit")
    ap.add_argument("--no-pipelined", action="store_true",
                    help="skip the checks of the large instance with several in flight on separate streams")
    ap.add_argument("--no-segments", action="store_true",
                    help="skip the segment-sum legs (profiling runs of the dense kernel alone)")
    ap.add_argument("--served-seconds", type=float, default=2.0)
    ap.add_argument("--no-search", action="store_true", help="skip the Weibull search leg")
    ap.add_argument("--search-seconds", type=float, default=0.5, help="time limit per instance and mode")
    ap.add_argument("--search-ablation", action="store_true",
                    help="only run the Weibull search leg, with the rule ablation, and exit")
    ap.add_argument("--latency-only", action="store_true",
                    help="only time the plain small checks (--latency-checks of them) and exit")
    ap.add_argument("--valu-rates", action="store_true",
                    help="only measure the VALU issue rate of each inner-loop opcode and exit")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run device copies of MIB MiB (scale for the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU layout is "
              "described in DESIGN.md and not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.valu_rates:
        print(json.dumps(valu_rates()), flush=True)
        return

    if args.calibrate_copy:
        n = args.calibrate_copy << 20
        src = torch.ones(n // 4, dtype=torch.int32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n, "copies": 5, "read_bytes_per_copy": n, "write_bytes_per_copy": n}))
        return

    import paper_2402_14821_amd as bp
    from paper_2402_14821_amd import workloads as W

    if args.latency_only:
        with bp.Context(0) as lctx:
            plain_latency(bp, W, lctx, 200)  # warm-up
            lat = plain_latency(bp, W, lctx, args.latency_checks)
        print(json.dumps({"plain_small_check_us": {"p50": percentile(lat, 50), "p99": percentile(lat, 99),
                                                   "n": len(lat)}}), flush=True)
        return

    if args.search_ablation:
        with bp.Context(0) as sctx:
            print(json.dumps({"search": bench_search(bp, W, sctx, args.search_seconds, ablation=True)}), flush=True)
        return

    if args.per_bound:
        with bp.Context(0) as pctx:
            print(json.dumps(per_bound_table(bp, W, pctx)), flush=True)
        return

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

    # timed region: K whole steps, inputs resident in HBM.  The kernels run
    # one by one with HIP events around each on this stream, so the sweep
    # kernel's mean duration over exactly these K steps is known.
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt * 1e3 / args.steps
    (prep_avg, sweep_avg, fin_avg), runs = ctx.stage_times(with_runs=True)
    ctx.set_timing(False)
    assert runs == args.steps, (runs, args.steps)

    # the same steps replayed as one HIP graph each (the default launch path)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms_per_step_graph = (time.perf_counter() - t1) * 1e3 / args.steps

    # the same steps with the segment sums (same results, less work per parameter)
    def step_seg():
        ctx.feasible_dev(C, m, d_res.data_ptr(), len(unpacked), d_unp.data_ptr(), d_out.data_ptr(), sp,
                         flags=bp.BP_NO_EARLY_EXIT | bp.BP_SEGMENTS)

    def bench_segments():
        for _ in range(args.warmup):
            step_seg()
        torch.cuda.synchronize()
        rec_seg = bp.bounds_to_dict(np.frombuffer(d_out.cpu().numpy().tobytes(), dtype=bp.BOUNDS_DTYPE)[0])
        if not all(np.array_equal(rec_seg[f], rec[f]) for f in ("value", "argmax")):
            return {"error": "segment record differs from the dense record"}
        ctx.set_timing(True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for _ in range(args.steps):
            step_seg()
        torch.cuda.synchronize()
        dt_seg = time.perf_counter() - t2
        (sprep, ssweep, sfin), sruns = ctx.stage_times(with_runs=True)
        ctx.set_timing(False)
        return {"ms_per_step": dt_seg * 1e3 / args.steps, "checks_per_s": args.steps / dt_seg,
                "nominal_evals_per_s": evals_per_step * args.steps / dt_seg,
                "speedup_vs_dense": dt / dt_seg,
                "stages_ms": {"prep": sprep, "sweep": ssweep, "finalize": sfin, "runs": sruns},
                "note": "MT, CCM1 and BJ1 sums from threshold sums over the sorted sizes, VB2 mirrored "
                        "(BP_SEGMENTS); identical bounds; nominal evals = r x sum of range sizes, not "
                        "evaluations performed"}

    segments = None
    if not args.no_segments:
        try:
            segments = bench_segments()
        except bp.BpError as e:  # reported, never the headline
            ctx.set_timing(False)
            segments = {"error": str(e)}

    def bench_pipelined(nstreams: int):
        """Independent checks of the same instance, each the plain path, on
        `nstreams` contexts and streams in turn: a stream of checks with
        several in flight (one sweep's tail and the next check's prep and
        finalize overlap).  Reported beside the one-stream headline."""
        ctxs = [bp.Context(0) for _ in range(nstreams)]
        strs = [torch.cuda.Stream(dev) for _ in range(nstreams)]
        outs = [torch.zeros(bp.BOUNDS_DTYPE.itemsize, dtype=torch.uint8, device=dev) for _ in range(nstreams)]
        try:
            def one(i):
                j = i % nstreams
                ctxs[j].feasible_dev(C, m, d_res.data_ptr(), len(unpacked), d_unp.data_ptr(), outs[j].data_ptr(),
                                     strs[j].cuda_stream, flags=bp.BP_NO_EARLY_EXIT)
            for i in range(max(args.warmup, nstreams)):
                one(i)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            for i in range(args.steps):
                one(i)
            torch.cuda.synchronize()
            dtp = time.perf_counter() - t3
            for j in range(nstreams):
                got = bp.bounds_to_dict(np.frombuffer(outs[j].cpu().numpy().tobytes(), dtype=bp.BOUNDS_DTYPE)[0])
                if not all(np.array_equal(got[f], rec[f]) for f in ("value", "argmax")):
                    return {"error": "a pipelined record differs from the single-stream record"}
            return {"streams": nstreams, "ms_per_check": dtp * 1e3 / args.steps, "checks_per_s": args.steps / dtp,
                    "evals_per_s": evals_per_step * args.steps / dtp}
        finally:
            for c in ctxs:
                c.close()

    pipelined = None
    if not args.no_pipelined:
        pipelined = [bench_pipelined(k) for k in (2, 3)]

    # the reduced items (Fig. 3): the unpacked sizes and one virtual item per bin that is not empty
    items_red = np.concatenate([unpacked, C - residual[residual < C]])
    assert len(items_red) == r
    ops = sweep_ops(bp, C, items_red, int(ctx.get_tuning()["lanes_params"]))
    achieved = ops / (sweep_avg * 1e-3)
    traffic = load_traffic("k_sweep")
    valu_insts = load_valu_insts("k_sweep")

    lat = plain_latency(bp, W, ctx, args.latency_checks)

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
        "ms_per_step_graph": ms_per_step_graph,
        "stages_ms": {"prep": prep_avg, "sweep": sweep_avg, "finalize": fin_avg, "runs": runs},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_VALU / 1e12, "unit": "TOP/s",
                     "frac": achieved / PEAK_VALU, "traffic": traffic, "kernel": "k_sweep",
                     "ops_per_eval": OPS_PER_EVAL, "ops_per_eval_short": OPS_PER_EVAL_SHORT,
                     "ops_per_eval_bj1_upper": OPS_PER_EVAL_BJ1_UPPER,
                     "weights": "profiles/valu_rates_gfx950.txt",
                     "slots_per_launch": ops,
                     # every VALU instruction the kernel issued (SQ_INSTS_VALU x 64 lanes) as one full slot
                     "frac_issue": (valu_insts * 64 / (sweep_avg * 1e-3) / PEAK_VALU) if valu_insts else None,
                     "tuning": ctx.get_tuning()},
        "plain_small_check_us": {"p50": percentile(lat, 50), "p99": percentile(lat, 99), "n": len(lat),
                                 "workload": "n=50 sizes U[20,100], m=20, C=150, 30% pre-packed; host in/out"},
        "verdict": rec["verdict"], "lb": rec["lb"],
        "segments": segments,
        "pipelined": pipelined,
    }
    log(f"large instance done: {ms_per_step:.3f} ms/step")
    if not args.no_batched:
        line["batched"] = bench_batched(bp, W, ctx, segments=not args.no_segments, tuning_cache=tuning_cache_path())
        log("batched leg done")
        line["triplets"] = bench_triplets(bp, W, ctx)
        log("triplet leg done")
        line["fidelity"] = bench_fidelity(bp, W, ctx)
        log("fidelity study done")
    if not args.no_search:
        line["search"] = bench_search(bp, W, ctx, args.search_seconds)
        log("search leg done")
    if not args.no_served:
        line["served"] = []
        legs = [(0, 20_000.0, 3), (0, 200_000.0, 4)]
        if not args.no_segments:
            legs.append((bp.BP_SEGMENTS, 200_000.0, 4))  # the roots' sweeps in segment form
        for flags, rate, seed in legs:
            line["served"].append(bench_served(bp, W, ctx, rate, args.served_seconds, seed, flags=flags))
            log(f"served leg at {rate:.0f}/s (flags {flags}) done")
    if not args.no_cpu_baseline:
        import oracle as O
        items = O.residual_reduce(C, residual, unpacked)
        line["cpu_baseline"] = cpu_baseline(C, items, args.cpu_seconds)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
