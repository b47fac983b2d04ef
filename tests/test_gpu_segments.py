"""GPU parity of the segment sums (BP_SWEEP_SEGMENTS / BP_SEGMENTS).

The segment form computes the MT, RAD2, CCM1 and BJ1 sums from threshold
sums over the sorted sizes instead of one evaluation per (item, parameter),
and half of the VB2 sums from the other half (mirror); the bounds are the
same integers.  Every record is compared with the CPU oracle (the dense
definition) field by field; at full size both with the oracle's dense record
and per parameter, and with the dense GPU path.
BP_SEGMENT_KCUT forces segment tiles of BJ1 wherever floor(c / lambda) <= K,
so that many windows per tile are exercised on small instances too.
"""
import os
import random
import sys
import time

import numpy as np
import pytest

import oracle as O
import oracle_par
import paper_2402_14821_amd as bp
from paper_2402_14821_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def make_ctx(kcut=None):
    old = os.environ.get("BP_SEGMENT_KCUT")
    if kcut is None:
        os.environ.pop("BP_SEGMENT_KCUT", None)
    else:
        os.environ["BP_SEGMENT_KCUT"] = str(kcut)
    try:
        return bp.Context(0)
    finally:
        if old is None:
            os.environ.pop("BP_SEGMENT_KCUT", None)
        else:
            os.environ["BP_SEGMENT_KCUT"] = old


@pytest.fixture(scope="module")
def ctx():
    c = make_ctx()
    yield c
    c.close()


@pytest.fixture(scope="module")
def ctx64():
    c = make_ctx(64)
    yield c
    c.close()


def same(got, want, what=""):
    assert got["status"] == 0, (what, got)
    assert np.array_equal(got["value"], want["value"]), (what, got["value"], want["value"])
    assert np.array_equal(got["argmax"], want["argmax"]), (what, got["argmax"], want["argmax"])
    assert got["lb"] == want["lb"] and got["lb_arg"] == want["lb_arg"], (what, got, want)
    assert got["verdict"] == want["verdict"], what


def seg_sweep(C, lo=None, hi=None):
    if lo is None:
        return bp.default_sweep(C, 0, 0, bp.BP_SWEEP_SEGMENTS)
    return bp.make_sweep(lo, hi, bp.BP_SWEEP_SEGMENTS)


def rand_instance(rng, cmax=300, nmax=40):
    C = rng.randint(1, cmax)
    n = rng.randint(0, nmax)
    pool = [0, C, C // 2, (C + 1) // 2, 1, C - 1]
    items = [rng.choice(pool) if rng.random() < 0.2 else rng.randint(0, C) for _ in range(n)]
    return C, [min(max(w, 0), C) for w in items]


@pytest.mark.parametrize("which", ["model", "kcut64"])
def test_random_small_instances(ctx, ctx64, which):
    c = ctx if which == "model" else ctx64
    rng = random.Random(1101 if which == "model" else 1102)
    for t in range(200):
        C, items = rand_instance(rng, cmax=400 if t % 2 else 40, nmax=60)
        k = rng.randint(0, len(items) + 1)
        say("segments random", which, t, C, len(items))
        same(c.lower_bounds(C, k, items, seg_sweep(C)), O.bounds(C, k, items), (which, C, k, items))


@pytest.mark.parametrize("which", ["model", "kcut64"])
def test_dense_sizes_many_windows(ctx, ctx64, which):
    # more sizes than capacity: narrow buckets, long windows, many equal sizes
    c = ctx if which == "model" else ctx64
    rng = np.random.default_rng(77)
    for t, C in enumerate((64, 150, 997, 1000, 4096)):
        for dist in ("uniform", "clustered"):
            r = int(rng.integers(C // 2, 3 * C))
            if dist == "uniform":
                items = rng.integers(0, C + 1, size=r)
            else:
                centers = rng.integers(1, C, size=4)
                items = np.clip(rng.choice(centers, size=r) + rng.integers(-2, 3, size=r), 0, C)
            items = items.astype(np.int32)
            k = int(items.sum() // C + 1)
            say("segments dense sizes", which, C, dist, r)
            same(c.lower_bounds(C, k, items, seg_sweep(C)), O.bounds(C, k, items), (which, C, dist))


def test_batch_with_and_without_segments(ctx, ctx64):
    rng = random.Random(1202)
    insts = [rand_instance(rng, cmax=3000, nmax=300) for _ in range(150)]
    Cs = [c for c, _ in insts]
    ks = [rng.randint(0, len(it) + 1) for _, it in insts]
    items = [it for _, it in insts]
    want = O.bounds_many([(C, k, it) for (C, it), k in zip(insts, ks)])
    # every other instance in segment form, the rest dense, in one launch
    sweeps = [seg_sweep(C) if i % 2 == 0 else bp.default_sweep(C) for i, C in enumerate(Cs)]
    for c, name in ((ctx, "model"), (ctx64, "kcut64")):
        say("segments batch", name)
        out = c.lower_bounds_batch(Cs, ks, items, sweeps)
        for i in range(len(insts)):
            same(bp.bounds_to_dict(out[i]), want[i], (name, i))


def test_subranges(ctx64):
    rng = random.Random(1303)
    for t in range(60):
        C, items = rand_instance(rng, cmax=5000, nmax=80)
        dlo, dhi = zip(*(O.default_range(b, C) for b in range(O.NB)))
        lo, hi = list(dlo), list(dhi)
        for b in range(1, O.NB):
            if dlo[b] <= dhi[b] and rng.random() < 0.7:
                x, y = sorted(rng.randint(dlo[b], dhi[b]) for _ in range(2))
                lo[b], hi[b] = x, y
            elif rng.random() < 0.1:
                lo[b], hi[b] = 1, 0
        say("segments subrange", t, C)
        got = ctx64.lower_bounds(C, 3, items, seg_sweep(C, lo, hi))
        same(got, O.bounds(C, 3, items, lo, hi, l2_dense=True), ("sub", C, items, lo, hi))


def test_huge_capacity_windows(ctx, ctx64):
    # thresholds up to c + 1 near 2^31, 64-bit products of K and lambda
    rng = random.Random(1404)
    for C in (2**31 - 1, 2**31 - 2, 1_999_999_973, 2**30 + 1, 2**25 + 3, 1_000_000):
        for t in range(3):
            n = rng.randint(1, 60)
            pool = [C, C - 1, C // 2, C // 2 + 1, (C + 1) // 2, 1, C // 3, C // 4 + 1]
            items = [rng.choice(pool) if rng.random() < 0.4 else rng.randint(0, C) for _ in range(n)]
            for side in ("low", "high"):
                lo, hi = [0] * O.NB, [-1] * O.NB
                for b in range(1, O.NB):
                    dlo, dhi = O.default_range(b, C)
                    if b == O.L2:
                        lo[b], hi[b] = dlo, dhi
                        continue
                    if dlo > dhi:
                        lo[b], hi[b] = 1, 0
                        continue
                    w = 200
                    lo[b], hi[b] = (dlo, min(dhi, dlo + w - 1)) if side == "low" else (max(dlo, dhi - w + 1), dhi)
                for c, name in ((ctx, "model"), (ctx64, "kcut64")):
                    say("segments huge C", C, t, side, n, name)
                    got = c.lower_bounds(C, n, items, seg_sweep(C, lo, hi))
                    same(got, O.bounds(C, n, items, lo, hi, l2_dense=False), ("huge", C, side, items, name))


def test_edge_cases(ctx64):
    cases = [
        (1, []), (1, [0]), (1, [1, 1, 0]), (2, [1, 1, 2]), (3, [1, 2, 3, 0]), (7, [7] * 5),
        (10, [0] * 9), (10, [5] * 7), (11, [6, 5, 6, 5]), (64, list(range(65))), (65, [1] * 200),
    ]
    for C, items in cases:
        for k in (0, len(items)):
            say("segments edge", C, len(items), k)
            same(ctx64.lower_bounds(C, k, items, seg_sweep(C)), O.bounds(C, k, items), (C, items, k))


def test_partial_packings_flag(ctx):
    for seed in range(30):
        C, m, res, unp = W.small_partial_packing(seed)
        items = O.residual_reduce(C, res, unp)
        want = O.bounds(C, m, items)
        say("segments config-1 seed", seed)
        got = ctx.feasible(C, res, unp, flags=bp.BP_NO_EARLY_EXIT | bp.BP_SEGMENTS)
        same(got, want, ("cfg1", seed))
        early = ctx.feasible(C, res, unp, flags=bp.BP_SEGMENTS)
        assert early["verdict"] == want["verdict"]


def test_large_residual_instance_full(ctx, ctx64):
    # full size: every field of the segment record against the oracle's dense
    # record, and equal to the dense GPU record
    C, m, res, unp, items, want = oracle_par.large_residual_record(1)
    say("segments config-2 full size, dense oracle record")
    dense = ctx.feasible(C, res, unp, flags=bp.BP_NO_EARLY_EXIT)
    for c, name in ((ctx, "model"), (ctx64, "kcut64")):
        seg = c.feasible(C, res, unp, flags=bp.BP_NO_EARLY_EXIT | bp.BP_SEGMENTS)
        same(seg, want, name)
        same(seg, dense, name)
        assert seg["evals"] == dense["evals"] and seg["r"] == dense["r"] == len(items)


def test_large_residual_per_parameter_values(ctx, ctx64):
    # copies of the large instance in one batch, each with single-parameter or
    # short-window ranges and the segment flag: per-parameter values
    C, m, res, unp, items, _ = oracle_par.large_residual_record(1)
    rng = random.Random(78)
    dlo, dhi = zip(*(O.default_range(b, C) for b in range(O.NB)))
    sweeps = []
    for t in range(256):
        lo, hi = [1] * O.NB, [0] * O.NB
        for b in range(O.L2, O.NB):
            if t < 192:
                lam = rng.randint(dlo[b], dhi[b])
                lo[b], hi[b] = lam, lam
            else:
                a = rng.randint(dlo[b], dhi[b])
                lo[b], hi[b] = a, min(dhi[b], a + rng.choice([5, 64, 127, 128, 129, 700]) - 1)
        sweeps.append((lo, hi))
    want = O.bounds_many([(C, m, items, lo, hi) for lo, hi in sweeps], threads=oracle_par.pool_threads(),
                         l2_dense=True)
    for c, name in ((ctx, "model"), (ctx64, "kcut64")):
        say("segments config-2 per-parameter values", name)
        out = c.lower_bounds_batch([C] * len(sweeps), [m] * len(sweeps), [items] * len(sweeps),
                                   [bp.make_sweep(lo, hi, bp.BP_SWEEP_SEGMENTS) for lo, hi in sweeps])
        for i in range(len(sweeps)):
            same(bp.bounds_to_dict(out[i]), want[i], (name, i, sweeps[i]))


def test_uneven_batch_equals_dense(ctx):
    b = W.uneven_batch(2, count=512)
    items = [b.instance(i)[2] for i in range(len(b))]
    say("segments uneven batch 512")
    dense = ctx.lower_bounds_batch(b.C, b.k, items)
    seg = ctx.lower_bounds_batch(b.C, b.k, items, [seg_sweep(int(C)) for C in b.C])
    for i in range(len(b)):
        same(bp.bounds_to_dict(seg[i]), bp.bounds_to_dict(dense[i]), ("uneven", i))
    assert np.array_equal(seg["verdict"] == 0, b.expect_fail)


def test_queue_requests_with_segments(ctx):
    reqs = W.dfs_requests(3, rate=20_000.0, duration=1.0, max_requests=24)
    say("segments queue of", len(reqs))
    q = bp.Queue(ctx, 1 << 30, 64)
    try:
        for i, r in enumerate(reqs):
            fl = bp.BP_NO_EARLY_EXIT | (bp.BP_SEGMENTS if i % 2 == 0 else 0)
            q.submit(r.C, r.residual, r.unpacked, tag=i, flags=fl)
        got = {}
        t0 = time.time()
        while len(got) < len(reqs):
            assert time.time() - t0 < 60.0, f"only {len(got)} of {len(reqs)} results"
            for rr in q.poll(256, timeout_us=20000):
                got[rr.tag] = rr
    finally:
        q.close()
    for i, rr in got.items():
        r = reqs[i]
        assert rr.status == 0
        want = ctx.feasible(r.C, r.residual, r.unpacked, flags=bp.BP_NO_EARLY_EXIT)
        say("segments queue tag", i)
        same(bp.bounds_to_dict(rr.bounds), want, ("queue", i))


def test_mirrored_vb2(ctx):
    # VB2 in segment form reuses each dense sum at lambda for c - lambda (needs
    # >= 256 sizes); odd, even, prime and highly composite capacities, full and
    # partial ranges, compared with the oracle field by field
    rng = np.random.default_rng(1505)
    for C in (1009, 1000, 1024, 4096, 5040, 9973):
        for t in range(3):
            r = int(rng.integers(256, 700))
            items = rng.integers(0, C + 1, size=r)
            items[: r // 10] = rng.choice([C, C // 2, (C + 1) // 2, 1, C - 1], size=r // 10)
            items = items.astype(np.int32)
            lo = [O.default_range(b, C)[0] for b in range(O.NB)]
            hi = [O.default_range(b, C)[1] for b in range(O.NB)]
            if t == 1:
                lo[O.VB2], hi[O.VB2] = sorted(int(x) for x in rng.integers(2, C + 1, size=2))
            elif t == 2:
                lo[O.VB2], hi[O.VB2] = C // 2 - 40, C // 2 + 60
            say("mirrored VB2", C, t, r, lo[O.VB2], hi[O.VB2])
            got = ctx.lower_bounds(C, r // 3, items, seg_sweep(C, lo, hi))
            same(got, O.bounds(C, r // 3, items, lo, hi), ("mirror", C, t))
    # 720720 has 240 divisors; windows around c/2 and at the top
    C = 720720
    items = rng.integers(1, C, size=400).astype(np.int32)
    items[:40] = [d for d in range(2, 100000) if C % d == 0][:40]
    for vlo, vhi in ((C // 2 - 200, C // 2 + 200), (C - 300, C)):
        lo = [O.default_range(b, C)[0] for b in range(O.NB)]
        hi = [min(O.default_range(b, C)[1], lo[b] + 99) for b in range(O.NB)]
        lo[O.L2], hi[O.L2] = O.default_range(O.L2, C)
        lo[O.VB2], hi[O.VB2] = vlo, vhi
        say("mirrored VB2 720720", vlo, vhi)
        got = ctx.lower_bounds(C, 100, items, seg_sweep(C, lo, hi))
        same(got, O.bounds(C, 100, items, lo, hi), ("mirror 720720", vlo))
