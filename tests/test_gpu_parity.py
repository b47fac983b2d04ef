"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Integer results, so the bar is equality of every field: each bound, its
smallest maximising parameter, lb, the first bound attaining lb, the verdict.
The single large residual instance (r = 14 000, C = 100 000) is compared
field by field with the oracle's dense record (every parameter of every
range, L2 included, split over a thread pool), and per parameter: copies of
it in one batch, each swept at single parameters or short windows.
Capacities near 2^31 are compared on windows at both ends of every range,
and over full ranges against the oracle's piece-start and event sweeps.
"""
import os
import random
import sys

import numpy as np
import pytest

import oracle as O
import paper_2402_14821_amd as bp
import oracle_par
from golden_io import fig3, hand_bounds
from paper_2402_14821_amd import workloads as W

pytestmark = pytest.mark.gpu
NAME2ID = {n: i for i, n in enumerate(O.NAMES)}


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = bp.Context(0)
    yield c
    c.close()


def same(got, want, what=""):
    assert got["status"] == 0, (what, got)
    assert np.array_equal(got["value"], want["value"]), (what, got["value"], want["value"])
    assert np.array_equal(got["argmax"], want["argmax"]), (what, got["argmax"], want["argmax"])
    assert got["lb"] == want["lb"] and got["lb_arg"] == want["lb_arg"], (what, got, want)
    assert got["verdict"] == want["verdict"], what


def row_dict(row):
    return bp.bounds_to_dict(row)


def rand_instance(rng, cmax=300, nmax=40):
    C = rng.randint(1, cmax)
    n = rng.randint(0, nmax)
    pool = [0, C, C // 2, (C + 1) // 2, 1, C - 1]
    items = [rng.choice(pool) if rng.random() < 0.2 else rng.randint(0, C) for _ in range(n)]
    items = [min(max(w, 0), C) for w in items]
    return C, items


@pytest.fixture(scope="module")
def ctx_pipe():
    # a context whose small checks run the multi-kernel pipeline too
    old = os.environ.get("BP_NO_SMALL_PATH")
    os.environ["BP_NO_SMALL_PATH"] = "1"
    try:
        c = bp.Context(0)
    finally:
        if old is None:
            os.environ.pop("BP_NO_SMALL_PATH", None)
        else:
            os.environ["BP_NO_SMALL_PATH"] = old
    yield c
    c.close()


@pytest.fixture(scope="module")
def ctx_block():
    # a context whose large instances are prepared by one block (LDS sort)
    old = os.environ.get("BP_NO_VALUE_PREP")
    os.environ["BP_NO_VALUE_PREP"] = "1"
    try:
        c = bp.Context(0)
    finally:
        if old is None:
            os.environ.pop("BP_NO_VALUE_PREP", None)
        else:
            os.environ["BP_NO_VALUE_PREP"] = old
    yield c
    c.close()


def test_value_table_prep_matches_block_prep_and_oracle(ctx, ctx_block):
    # large instances (more than 8192 reduced items, c <= 16 r) prepared from
    # value tables over the whole GPU, against the one-block prep and the
    # oracle: both input forms, the segment sums with the mirrored VB2
    # (divisor lattice), the VB2 cut, heavy duplicates, tiny c, the largest r
    g = np.random.default_rng(31)
    cases = [(12000, 9000, 0, 0), (12000, 7000, 3000, bp.BP_SEGMENTS), (5040, 8500, 500, bp.BP_SEGMENTS),
             (16000, 6000, 3000, -1), (2, 9000, 0, 0), (1000, 16384, 0, bp.BP_SEGMENTS), (77, 4000, 5000, 0)]
    for C, n, m, flags in cases:
        unp = g.integers(0, C + 1, size=n).astype(np.int32)
        if m:
            res = g.integers(0, C + 1, size=m).astype(np.int32)
            res[: m // 4] = C  # empty bins
            items = O.residual_reduce(C, res, unp)
            k = m
        else:
            items = list(unp)
            k = int(O.bounds(C, 0, items[:50])["lb"]) + n // 4
        if flags == -1:  # the paper's VB2 cut
            maxw = max(items) if len(items) else 0
            lo, hi = zip(*(O.default_range(b, C, len(items), maxw, clamp_vb2=True) for b in range(O.NB)))
            want = O.bounds(C, k, items, list(lo), list(hi))
        else:
            want = O.bounds(C, k, items)
        for c, name in ((ctx, "value tables"), (ctx_block, "block")):
            say("value prep", C, n, m, flags, name)
            if flags == -1:
                sw = bp.default_sweep(C)
                sw.flags = bp.BP_SWEEP_PAPER_VB2_CLAMP
                got = c.lower_bounds(C, k, np.asarray(items, dtype=np.int32), sw)
            elif m:
                got = c.feasible(C, res, unp, flags=bp.BP_NO_EARLY_EXIT | flags)
            else:
                sw = bp.default_sweep(C)
                sw.flags = bp.BP_SWEEP_SEGMENTS if flags else 0
                got = c.lower_bounds(C, k, unp, sw)
            same(got, want, (name, C, n, m, flags))
            assert got["r"] == len(items)
    # a residual outside [0, c] and a size outside [0, c] in device memory:
    # the device-side range error from both preps, and clean tables after it
    torch = pytest.importorskip("torch")
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev).cuda_stream
    d_out = torch.zeros(bp.BOUNDS_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    C = 20000
    unp = g.integers(0, C + 1, size=9000).astype(np.int32)
    res = g.integers(0, C + 1, size=100).astype(np.int32)
    for bad_res, bad_unp in ((C + 1, None), (None, -3)):
        r2, u2 = res.copy(), unp.copy()
        if bad_res is not None:
            r2[17] = bad_res
        if bad_unp is not None:
            u2[4321] = bad_unp
        d_res, d_unp = torch.from_numpy(r2).to(dev), torch.from_numpy(u2).to(dev)
        for c, name in ((ctx, "value tables"), (ctx_block, "block")):
            say("value prep range error", name, bad_res, bad_unp)
            c.feasible_dev(C, len(r2), d_res.data_ptr(), len(u2), d_unp.data_ptr(), d_out.data_ptr(), stream)
            torch.cuda.synchronize()
            got = row_dict(np.frombuffer(d_out.cpu().numpy().tobytes(), dtype=bp.BOUNDS_DTYPE)[0])
            assert got["status"] == bp.BP_ERR_RANGE, name
    want = O.bounds(C, 100, O.residual_reduce(C, res, unp))
    same(ctx.feasible(C, res, unp, flags=bp.BP_NO_EARLY_EXIT), want, "after the range errors")


@pytest.mark.parametrize("C", [2046, 2047, 2048, 4094, 4095])
def test_value_table_chunk_edges(ctx, C):
    # the tables hold c + 2 values in chunks of 2 048: c + 2 at, just past and
    # just below a chunk boundary, dense and segment form, items and residuals
    g = np.random.default_rng(C)
    n, m = 8600, 600
    unp = g.integers(0, C + 1, size=n).astype(np.int32)
    unp[:40] = C
    unp[40:80] = 0
    res = g.integers(0, C + 1, size=m).astype(np.int32)
    res[:100] = C
    items = O.residual_reduce(C, res, unp)
    want, want_items = O.bounds_many([(C, m, items), (C, m, unp)])
    for flags in (0, bp.BP_SEGMENTS):
        say("value-table chunk edge", C, flags)
        same(ctx.feasible(C, res, unp, flags=bp.BP_NO_EARLY_EXIT | flags), want, ("chunk edge", C, flags))
        sw = bp.default_sweep(C)
        sw.flags = bp.BP_SWEEP_SEGMENTS if flags else 0
        same(ctx.lower_bounds(C, m, unp, sw), want_items, ("chunk edge items", C, flags))


def test_one_multiply_quotient_cuts(ctx):
    # sizes around the limits of the one-multiply quotients: VB2's a <= 2^32 / c (a the size or its complement),
    # CCM1's a <= 2^32 / lambda and BJ1's w <= 2^32 / lambda over the top tiles of their ranges, so that tiles
    # and item chunks straddle every cut; at capacities where the VB2 cut lies below c / 2, dense and segment
    # form, against the oracle's dense record
    insts = []
    for C in (92_682, 100_000, 140_001):
        g = np.random.default_rng(C)
        lv = (1 << 32) // C
        near = g.integers(max(1, lv - 400), min(C // 2, lv + 400), size=150)
        spread = g.integers(1, C, size=250)
        exact = [lv - 1, lv, lv + 1, C - lv - 1, C - lv, C - lv + 1, C // 2, (C + 1) // 2, C - 1, 1, C]
        items = np.concatenate([near, C - near, spread, exact]).astype(np.int32)
        k = int(items.astype(np.int64).sum()) // C + 2
        insts.append((C, k, items))
    wants = O.bounds_many([(C, k, list(map(int, items))) for C, k, items in insts], l2_dense=True)
    for (C, k, items), want in zip(insts, wants):
        for flags in (0, bp.BP_SWEEP_SEGMENTS):
            say("one-multiply cuts", C, flags)
            sw = bp.default_sweep(C)
            sw.flags = flags
            same(ctx.lower_bounds(C, k, items, sw), want, ("quotient cuts", C, flags))


def test_value_table_launch_sequences(ctx):
    # value-table launches of different capacities and instance orders on one
    # context, so that each launch finds its tables where earlier launches of
    # other layouts left theirs (they must be back at zero in between)
    g = np.random.default_rng(33)
    insts = []
    for C, n in ((60000, 9000), (20000, 9500), (45000, 8800)):
        items = g.integers(0, C + 1, size=n).astype(np.int32)
        insts.append((C, int(items.sum()) // C + 2, items))
    want = [oracle_par.dense_record(C, k, items) for C, k, items in insts]
    seq = [[0], [1], [0], [1, 0], [0, 1, 2], [2], [0], [2, 1], [1]]
    for step, ids in enumerate(seq):
        say("value-table sequence", step, ids)
        if len(ids) == 1:
            C, k, items = insts[ids[0]]
            same(ctx.lower_bounds(C, k, items), want[ids[0]], ("sequence", step))
        else:
            out = ctx.lower_bounds_batch([insts[i][0] for i in ids], [insts[i][1] for i in ids],
                                         [insts[i][2] for i in ids])
            for j, i in enumerate(ids):
                same(row_dict(out[j]), want[i], ("sequence batch", step, j))


def test_small_checks_on_both_paths(ctx, ctx_pipe):
    # the one-launch path (instance in the kernel arguments) and the pipeline
    # on the same small checks: random instances with custom ranges and the
    # VB2 cut, and partial packings; every record equal to the oracle's
    rng = random.Random(909)
    for t in range(120):
        C, items = rand_instance(rng, cmax=400, nmax=60)
        k = rng.randint(0, len(items) + 1)
        dlo, dhi = zip(*(O.default_range(b, C) for b in range(O.NB)))
        lo, hi = list(dlo), list(dhi)
        if t % 3 == 1:
            for b in range(1, O.NB):
                if dlo[b] <= dhi[b]:
                    x, y = sorted(rng.randint(dlo[b], dhi[b]) for _ in range(2))
                    lo[b], hi[b] = x, y
        want = O.bounds(C, k, items, lo, hi, l2_dense=True)
        for c, name in ((ctx, "one launch"), (ctx_pipe, "pipeline")):
            say("small both paths", t, name)
            same(c.lower_bounds(C, k, items, bp.make_sweep(lo, hi)), want, (name, C, items, lo, hi))
        if t % 6 == 0:
            maxw = max(items) if items else 0
            clo, chi = zip(*(O.default_range(b, C, len(items), maxw, clamp_vb2=True) for b in range(O.NB)))
            sw = bp.default_sweep(C)
            sw.flags = bp.BP_SWEEP_PAPER_VB2_CLAMP
            wantc = O.bounds(C, k, items, list(clo), list(chi), l2_dense=True)
            for c, name in ((ctx, "one launch"), (ctx_pipe, "pipeline")):
                same(c.lower_bounds(C, k, items, sw), wantc, (name, "clamp", C))
    for seed in range(100, 140):
        C, m, res, unp = W.small_partial_packing(seed)
        want = O.bounds(C, m, O.residual_reduce(C, res, unp))
        for c, name in ((ctx, "one launch"), (ctx_pipe, "pipeline")):
            got = c.feasible(C, res, unp, flags=bp.BP_NO_EARLY_EXIT)
            same(got, want, (name, seed))
            assert got["evals_done"] == got["evals"]
            assert c.feasible(C, res, unp)["verdict"] == want["verdict"]


def test_small_path_at_larger_capacities(ctx, ctx_pipe):
    # the one-launch path takes checks up to 2^26 evaluations: capacities up
    # to 92 500 and up to 960 inputs, in both forms, with one lane or several
    # per parameter and more pairs than one pass of the grid holds
    g = np.random.default_rng(77)
    cases = [(2500, 100, 50), (2500, 900, 60), (10000, 300, 0), (30000, 150, 60), (92500, 150, 60),
             (92500, 30, 10), (15000, 600, 300), (1, 5, 3), (7, 0, 12)]
    for C, n, m in cases:
        unp = np.minimum(C, np.maximum(0, (C * g.uniform(0.0, 0.8, n)).astype(np.int32))).astype(np.int32)
        res = (C * g.uniform(0, 1, m)).astype(np.int32)
        res[: m // 5] = C  # some empty bins
        if m:
            want = O.bounds(C, m, O.residual_reduce(C, res, unp))
            for c, name in ((ctx, "one launch"), (ctx_pipe, "pipeline")):
                say("small path larger", C, n, m, name)
                got = c.feasible(C, res, unp, flags=bp.BP_NO_EARLY_EXIT)
                same(got, want, (name, C, n, m))
                assert got["evals_done"] == got["evals"]
        else:
            k = int(g.integers(0, n + 1))
            want = O.bounds(C, k, list(unp))
            for c, name in ((ctx, "one launch"), (ctx_pipe, "pipeline")):
                say("small path larger items", C, n, name)
                same(c.lower_bounds(C, k, unp, bp.default_sweep(C)), want, (name, C, n))


def test_fig3_worked_example(ctx):
    g = fig3()
    C, k = g["C"][0], g["bins"][0]
    say("fig3 feasible")
    got = ctx.feasible(C, g["residual"], g["unpacked"], flags=bp.BP_NO_EARLY_EXIT)
    assert got["value"].tolist() == g["bounds"]
    assert got["verdict"] == g["verdict_k4"][0] and got["r"] == 6
    got = ctx.lower_bounds(C, k - 1, g["reduced"])
    assert got["verdict"] == g["verdict_k3"][0]
    same(got, O.bounds(C, k - 1, g["reduced"]), "fig3 k=3")


@pytest.mark.parametrize("row", hand_bounds(), ids=lambda r: r[0])
def test_hand_bounds(ctx, row):
    name, C, lam, want, want_l2, items = row
    say("hand", name)
    got = ctx.lower_bounds(C, len(items), items)
    same(got, O.bounds(C, len(items), items), name)
    assert got["value"][O.L2] == want_l2
    if name != "L2ODD":
        assert got["value"][NAME2ID[name]] == want


def test_random_small_instances(ctx):
    rng = random.Random(101)
    for t in range(250):
        C, items = rand_instance(rng)
        k = rng.randint(0, len(items) + 1)
        say("random", t, C, len(items))
        same(ctx.lower_bounds(C, k, items), O.bounds(C, k, items), (C, k, items))


def test_batch_matches_oracle_and_single(ctx):
    rng = random.Random(202)
    insts = [rand_instance(rng, cmax=2000, nmax=300) for _ in range(200)]
    Cs = [c for c, _ in insts]
    ks = [rng.randint(0, len(it) + 1) for _, it in insts]
    say("batch of", len(insts))
    out = ctx.lower_bounds_batch(Cs, ks, [it for _, it in insts])
    want = O.bounds_many([(C, k, it) for (C, it), k in zip(insts, ks)])
    for i in range(len(insts)):
        same(row_dict(out[i]), want[i], ("batch", i))
    for i in range(0, len(insts), 37):
        same(ctx.lower_bounds(Cs[i], ks[i], insts[i][1]), want[i], ("single", i))


def test_small_partial_packings(ctx):
    for seed in range(40):
        C, m, res, unp = W.small_partial_packing(seed)
        say("config-1 seed", seed)
        items = O.residual_reduce(C, res, unp)
        want = O.bounds(C, m, items)
        got = ctx.feasible(C, res, unp, flags=bp.BP_NO_EARLY_EXIT)
        same(got, want, ("cfg1", seed))
        assert got["r"] == len(items)
        assert got["evals_done"] == got["evals"] == len(items) * 563  # P(150) = 563
        early = ctx.feasible(C, res, unp)
        assert early["verdict"] == want["verdict"]
        assert 0 <= early["evals_done"] <= early["evals"]
        if want["verdict"] == 0:
            assert early["lb"] > m


def test_small_partial_packings_tight_bins(ctx):
    # fewer bins than the optimum needs: the check must refute
    for seed in range(20):
        C, m, res, unp = W.small_partial_packing(seed, m=12)
        items = O.residual_reduce(C, res, unp)
        want = O.bounds(C, m, items)
        say("tight config-1 seed", seed)
        got = ctx.feasible(C, res, unp, flags=bp.BP_NO_EARLY_EXIT)
        same(got, want, ("tight", seed))
        early = ctx.feasible(C, res, unp)
        assert early["verdict"] == want["verdict"]
        if early["early_exit"]:
            assert early["evals_done"] < early["evals"]
            if O.l1(C, items) > m:  # refuted before any sweep ran
                assert early["evals_done"] == 0


def test_large_residual_instance_full(ctx):
    # every field of the record against the oracle's dense record (L2 visited
    # at every parameter, every DFF swept over its whole range)
    C, m, res, unp, items, want = oracle_par.large_residual_record(1)
    say("config-2 full size, dense oracle record")
    got = ctx.feasible(C, res, unp, flags=bp.BP_NO_EARLY_EXIT)
    assert got["r"] == len(items) and got["status"] == 0
    same(got, want, "config-2")
    assert got["evals"] == len(items) * 308_433
    early = ctx.feasible(C, res, unp)
    assert early["verdict"] == want["verdict"]
    if want["verdict"] == 1:
        same(early, want, "config-2 early exit, passing")


def _param_sweeps(C, rng, n_points, n_windows):
    """Single-parameter sweeps (every bound but L1 at one parameter each) and
    short windows at random offsets: together they expose each lane's value,
    not only the maximum of a whole range."""
    dlo, dhi = zip(*(O.default_range(b, C) for b in range(O.NB)))
    sweeps = []
    for t in range(n_points + n_windows):
        lo, hi = [1] * O.NB, [0] * O.NB
        for b in range(O.L2, O.NB):
            if dlo[b] > dhi[b]:
                continue
            if t < n_points:
                lam = [dlo[b], dhi[b], dlo[b] + 1, dhi[b] - 1][t] if t < 4 else rng.randint(dlo[b], dhi[b])
                lam = min(max(lam, dlo[b]), dhi[b])
                lo[b], hi[b] = lam, lam
            else:
                w = rng.choice([2, 63, 64, 65, 127, 128, 129, 300])
                a = rng.randint(dlo[b], dhi[b])
                lo[b], hi[b] = a, min(dhi[b], a + w - 1)
        sweeps.append((lo, hi))
    return sweeps


def test_large_residual_per_parameter_values(ctx):
    # the large instance repeated in one batch, each copy with its own short
    # ranges: per-parameter bound values, compared with the oracle
    C, m, res, unp, items, _ = oracle_par.large_residual_record(1)
    rng = random.Random(77)
    sweeps = _param_sweeps(C, rng, 384, 128)
    say("config-2 per-parameter values,", len(sweeps), "copies")
    out = ctx.lower_bounds_batch([C] * len(sweeps), [m] * len(sweeps), [items] * len(sweeps),
                                 [bp.make_sweep(lo, hi) for lo, hi in sweeps])
    want = O.bounds_many([(C, m, items, lo, hi) for lo, hi in sweeps], threads=oracle_par.pool_threads(),
                         l2_dense=True)
    for i in range(len(sweeps)):
        same(row_dict(out[i]), want[i], ("per-parameter", i, sweeps[i]))


def test_sweep_subranges_and_vb2_clamp(ctx):
    rng = random.Random(303)
    for t in range(60):
        C, items = rand_instance(rng, cmax=5000, nmax=60)
        dlo, dhi = zip(*(O.default_range(b, C) for b in range(O.NB)))
        lo, hi = list(dlo), list(dhi)
        for b in range(1, O.NB):
            if dlo[b] <= dhi[b] and rng.random() < 0.7:
                x, y = sorted(rng.randint(dlo[b], dhi[b]) for _ in range(2))
                lo[b], hi[b] = x, y
            elif rng.random() < 0.1:
                lo[b], hi[b] = 1, 0
        say("subrange", t, C)
        got = ctx.lower_bounds(C, 3, items, bp.make_sweep(lo, hi))
        same(got, O.bounds(C, 3, items, lo, hi, l2_dense=True), ("sub", C, items, lo, hi))
    # the paper's VB2 cut
    for t in range(20):
        C, items = rand_instance(rng, cmax=3000, nmax=200)
        say("clamp", t)
        maxw = max(items) if items else 0
        sw = bp.default_sweep(C, len(items), maxw, bp.BP_SWEEP_PAPER_VB2_CLAMP)
        # the oracle's own cut of the VB2 range (pinned by the hand-worked clamp fixture)
        lo, hi = zip(*(O.default_range(b, C, len(items), maxw, clamp_vb2=True) for b in range(O.NB)))
        assert (sw.lo[O.VB2], sw.hi[O.VB2]) == (lo[O.VB2], hi[O.VB2])
        got = ctx.lower_bounds(C, 3, items, sw)
        same(got, O.bounds(C, 3, items, list(lo), list(hi), l2_dense=True), ("clamp", C))
        # the same cut applied on the device from the flag alone (the sizes' maximum known only there)
        full = bp.default_sweep(C)
        full.flags = bp.BP_SWEEP_PAPER_VB2_CLAMP
        same(ctx.lower_bounds(C, 3, items, full), O.bounds(C, 3, items, list(lo), list(hi), l2_dense=True),
             ("clamp on device", C))


def test_huge_capacity_windows(ctx):
    rng = random.Random(404)
    for C in (2**31 - 1, 2**31 - 2, 1_999_999_973, 2**30 + 1, 2**25 + 3, 1_000_000):
        for t in range(3):
            n = rng.randint(1, 50)
            pool = [C, C - 1, C // 2, C // 2 + 1, (C + 1) // 2, 1, C // 3, C // 4 + 1]
            items = [rng.choice(pool) if rng.random() < 0.4 else rng.randint(0, C) for _ in range(n)]
            for side in ("low", "high"):
                lo, hi = [0] * O.NB, [-1] * O.NB
                for b in range(1, O.NB):
                    dlo, dhi = O.default_range(b, C)
                    if b == O.L2:
                        lo[b], hi[b] = dlo, dhi  # exact over the full range (piece starts)
                        continue
                    if dlo > dhi:
                        lo[b], hi[b] = 1, 0
                        continue
                    w = 200
                    lo[b], hi[b] = (dlo, min(dhi, dlo + w - 1)) if side == "low" else (max(dlo, dhi - w + 1), dhi)
                say("huge C", C, t, side, n)
                got = ctx.lower_bounds(C, n, items, bp.make_sweep(lo, hi))
                same(got, O.bounds(C, n, items, lo, hi, l2_dense=False), ("huge", C, side, items))


def _unpairable_instance(seed, C, r):
    # items of 0.55-0.6 c and of 0.46-0.5 c never share a bin, so the DFF
    # bounds beat L1 and their maximisers sit inside the ranges
    g = np.random.default_rng(seed)
    a = g.integers(int(C * 0.55), int(C * 0.6), int(r * 0.4))
    b = g.integers(int(C * 0.46), C // 2, int(r * 0.4))
    c = g.integers(1, C // 20, r - len(a) - len(b))
    return np.concatenate([a, b, c]).astype(np.int32)


def test_huge_capacity_full_ranges(ctx):
    # every parameter of every range at capacities up to 2^31 - 1 (dense and
    # segment form) against the oracle's piece-start and event sweeps; VB2 has
    # no such oracle path: its value only enters lb
    cases = [(1, 2**31 - 1, 700), (2, 1_000_000_007, 900), (3, 123_456_789, 1500)]
    insts = [(C, _unpairable_instance(seed, C, r)) for seed, C, r in cases]
    with oracle_par.ThreadPoolExecutor(max_workers=3) as ex:
        wants = list(ex.map(lambda ci: O.bounds_by_pieces(ci[0], 0, ci[1], threads=6), insts))
    for (C, items), want in zip(insts, wants):
        k = int(want["value"].max())
        for flags in (0, bp.BP_SWEEP_SEGMENTS):
            say("huge C full ranges", C, len(items), flags)
            got = ctx.lower_bounds(C, k, items, bp.default_sweep(C, 0, 0, flags))
            assert got["status"] == 0
            for b in range(O.NB):
                if b == O.VB2:
                    continue
                assert got["value"][b] == want["value"][b], (C, flags, O.NAMES[b], got["value"], want["value"])
                assert got["argmax"][b] == want["argmax"][b], (C, flags, O.NAMES[b], got["argmax"], want["argmax"])
            vals = want["value"].copy()
            vals[O.VB2] = got["value"][O.VB2]
            assert got["lb"] == int(vals.max()) and got["lb_arg"] == int(np.argmax(vals))
            assert got["verdict"] == int(got["lb"] <= k)
            assert got["evals"] == len(items) * sum(
                max(0, hi - lo + 1) for lo, hi in (O.default_range(d, C) for d in O.DFFS))


@pytest.mark.parametrize("C", [1 << 20, 1 << 21])
def test_split_tile_slot_widths(ctx, C):
    # 16 000 big sizes, each range cut to 384 parameters (three tiles) at its
    # top end, so every tile is split into 16 item chunks of 1 000 sizes: at
    # c = 2^20 the chunk sums go through 32-bit slots (1 000 x 2c < 2^31), at
    # 2^21 through 64-bit ones; both against the oracle
    g = np.random.default_rng(C)
    items = g.integers(C // 2, C + 1, size=16000).astype(np.int32)
    lo, hi = [0] * O.NB, [-1] * O.NB
    for b in range(1, O.NB):
        dlo, dhi = O.default_range(b, C)
        lo[b], hi[b] = (max(dlo, dhi - 383), dhi) if dlo <= dhi else (1, 0)
    want = O.bounds(C, 0, items, lo, hi)
    say("split-tile slot widths", C)
    same(ctx.lower_bounds(C, 0, items, bp.make_sweep(lo, hi)), want, ("slots", C))


def test_edge_cases(ctx):
    cases = [
        (1, []), (1, [0]), (1, [1, 1, 0]), (2, [1, 1, 2]), (3, [1, 2, 3, 0]), (7, [7] * 5),
        (10, [0] * 9), (10, [5] * 7), (11, [6, 5, 6, 5]),
    ]
    for C, items in cases:
        for k in (0, len(items)):
            say("edge", C, items, k)
            same(ctx.lower_bounds(C, k, items), O.bounds(C, k, items), (C, items, k))
    # the largest capacity: every range cut to its first 64 parameters (the oracle cannot sweep 2^31)
    C = 2**31 - 1
    lo = [O.default_range(b, C)[0] for b in range(O.NB)]
    hi = [min(O.default_range(b, C)[1], lo[b] + 63) for b in range(O.NB)]
    for items in ([], [C], [C, C, 0], [C // 2 + 1, C // 2, 1]):
        say("edge max C", items)
        same(ctx.lower_bounds(C, 1, items, bp.make_sweep(lo, hi)), O.bounds(C, 1, items, lo, hi), ("maxC", items))
    say("empty residual form")
    got = ctx.feasible(10, [], [], flags=bp.BP_NO_EARLY_EXIT)
    assert got["lb"] == 0 and got["verdict"] == 1 and got["r"] == 0
    got = ctx.feasible(10, [10, 10, 10], [], flags=bp.BP_NO_EARLY_EXIT)
    assert got["r"] == 0 and got["verdict"] == 1


@pytest.mark.parametrize("r", [2048, 2049, 8191, 8192, 8193, 16384])
def test_block_capacity_boundaries(ctx, r):
    rng = np.random.default_rng(r)
    C = 600
    items = rng.integers(0, C + 1, size=r).astype(np.int32)
    say("capacity boundary r =", r)
    same(ctx.lower_bounds(C, r // 2, items), O.bounds(C, r // 2, items), ("cap", r))


def test_more_items_than_one_block_sorts(ctx):
    # past 16 384 reduced items the value tables prepare the instance: both
    # forms against the oracle's record (ranges split over a thread pool)
    g = np.random.default_rng(2024)
    C, n, m = 12000, 30000, 8000
    unp = g.integers(1, C // 2 + 1, size=n).astype(np.int32)
    res = g.integers(C // 3, C + 1, size=m).astype(np.int32)
    items = O.residual_reduce(C, res, unp)
    want = oracle_par.dense_record(C, m, items)
    say("more items", C, n, m, len(items))
    for flags in (0, bp.BP_SEGMENTS):
        got = ctx.feasible(C, res, unp, flags=bp.BP_NO_EARLY_EXIT | flags)
        same(got, want, ("more items", flags))
        assert got["r"] == len(items) > 16384
    items2 = g.integers(0, 700, size=70000).astype(np.int32)
    want2 = oracle_par.dense_record(700, 30000, items2)
    same(ctx.lower_bounds(700, 30000, items2), want2, "items form, 70 000 sizes")


def test_limits_and_range_errors(ctx):
    say("errors")
    # more than 16 384 items need c <= 2^21 and c <= 16 r (value tables)
    for C in (1 << 22, 16 * 16385 + 1):
        with pytest.raises(bp.BpError) as e:
            ctx.lower_bounds(C, 1, np.ones(16385, np.int32))
        assert e.value.status == bp.BP_ERR_LIMIT, C
    with pytest.raises(bp.BpError) as e:
        ctx.lower_bounds(10, 1, np.ones(bp.BP_MAX_ITEMS + 1, np.int32))
    assert e.value.status == bp.BP_ERR_LIMIT
    with pytest.raises(bp.BpError) as e:
        ctx.lower_bounds(10, 1, [3, 11])
    assert e.value.status == bp.BP_ERR_RANGE
    with pytest.raises(bp.BpError) as e:
        ctx.feasible(10, [11], [1])
    assert e.value.status == bp.BP_ERR_RANGE
    with pytest.raises(bp.BpError) as e:
        ctx.lower_bounds(10, 1, [3], bp.make_sweep([0] * 8, [5] * 8))  # MT beyond c/2 ... RAD2 outside its range
    assert e.value.status == bp.BP_ERR_RANGE
    # still usable after errors
    same(ctx.lower_bounds(10, 1, [3, 9]), O.bounds(10, 1, [3, 9]), "after errors")


def test_reductions(ctx):
    rng = random.Random(505)
    for t in range(30):
        C = rng.randint(1, 100)
        m = rng.randint(0, 30)
        res = [rng.randint(0, C) for _ in range(m)]
        unp = [rng.randint(0, C) for _ in range(rng.randint(0, 40))]
        say("residual_reduce", t)
        assert ctx.residual_reduce(C, res, unp).tolist() == O.residual_reduce(C, res, unp).tolist()
    for t in range(30):
        C = rng.randint(1, 100)
        m = rng.randint(1, 10)
        loads = [0] * m
        size, bin_of = [], []
        for _ in range(rng.randint(0, 40)):
            w = rng.randint(0, C)
            j = rng.randint(-1, m - 1)
            if j >= 0 and loads[j] + w > C:
                j = -1
            if j >= 0:
                loads[j] += w
            size.append(w)
            bin_of.append(j)
        say("assignment_reduce", t)
        got_items, got_res = ctx.assignment_reduce(C, m, size, bin_of)
        want_items, want_res = O.assignment_reduce(C, m, size, bin_of)
        assert got_items.tolist() == want_items.tolist()
        assert got_res.tolist() == want_res.tolist()
    with pytest.raises(bp.BpError):
        ctx.assignment_reduce(10, 1, [6, 6], [0, 0])  # bin over capacity


def test_device_pointer_paths(ctx):
    torch = pytest.importorskip("torch")
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev).cuda_stream
    rng = random.Random(606)
    C, items = rand_instance(rng, cmax=1000, nmax=300)
    d_items = torch.tensor(items or [0], dtype=torch.int32, device=dev)
    d_out = torch.zeros(bp.BOUNDS_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    say("lower_bounds_dev")
    ctx.lower_bounds_dev(C, 5, d_items.data_ptr(), len(items), d_out.data_ptr(), stream)
    torch.cuda.synchronize()
    got = row_dict(np.frombuffer(d_out.cpu().numpy().tobytes(), dtype=bp.BOUNDS_DTYPE)[0])
    same(got, O.bounds(C, 5, items), "dev single")
    insts = [rand_instance(rng, cmax=3000, nmax=200) for _ in range(50)]
    off = np.zeros(len(insts) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(it) for _, it in insts])
    flat = np.concatenate([np.asarray(it, np.int32) for _, it in insts] + [np.zeros(1, np.int32)])
    d_flat = torch.from_numpy(flat).to(dev)
    d_outb = torch.zeros(len(insts) * bp.BOUNDS_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    say("lower_bounds_batch_dev")
    ctx.lower_bounds_batch_dev([c for c, _ in insts], [2] * len(insts), off, d_flat.data_ptr(), d_outb.data_ptr(),
                               stream)
    torch.cuda.synchronize()
    rows = np.frombuffer(d_outb.cpu().numpy().tobytes(), dtype=bp.BOUNDS_DTYPE)
    want = O.bounds_many([(c, 2, it) for c, it in insts])
    for i in range(len(insts)):
        same(row_dict(rows[i]), want[i], ("dev batch", i))
    # device-side validation reports a bad size in the record
    bad = torch.tensor([5, 12], dtype=torch.int32, device=dev)
    ctx.lower_bounds_dev(10, 1, bad.data_ptr(), 2, d_out.data_ptr(), stream)
    torch.cuda.synchronize()
    got = row_dict(np.frombuffer(d_out.cpu().numpy().tobytes(), dtype=bp.BOUNDS_DTYPE)[0])
    assert got["status"] == bp.BP_ERR_RANGE


def test_device_call_then_other_calls_without_sync(ctx):
    # A *_dev call of the large instance on a side stream, then, with no
    # synchronisation, a host-memory check, a *_dev check on a second stream
    # and another host-memory check, all on the same context.  Each launch
    # waits for the previous one of the context, so every record is whole.
    torch = pytest.importorskip("torch")
    dev = torch.device("cuda:0")
    C, m, res, unp, items, want_big = oracle_par.large_residual_record(1)
    d_res = torch.from_numpy(res).to(dev)
    d_unp = torch.from_numpy(unp).to(dev)
    d_out1 = torch.zeros(bp.BOUNDS_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    d_out2 = torch.zeros(bp.BOUNDS_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    s1, s2 = torch.cuda.Stream(dev), torch.cuda.Stream(dev)
    rng = random.Random(616)
    C2, items2 = rand_instance(rng, cmax=2000, nmax=200)
    d_items2 = torch.tensor(items2 or [0], dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    for rep in range(3):
        say("dev call then host calls without sync, rep", rep)
        ctx.feasible_dev(C, m, d_res.data_ptr(), len(unp), d_unp.data_ptr(), d_out1.data_ptr(), s1.cuda_stream,
                         flags=bp.BP_NO_EARLY_EXIT)
        small = [W.small_partial_packing(seed=40 + rep)]
        Cs, ms, rs, us = small[0]
        got_host = ctx.feasible(Cs, rs, us, flags=bp.BP_NO_EARLY_EXIT)
        ctx.lower_bounds_dev(C2, 3, d_items2.data_ptr(), len(items2), d_out2.data_ptr(), s2.cuda_stream)
        got_host2 = ctx.lower_bounds(C2, 4, items2)
        torch.cuda.synchronize()
        big = row_dict(np.frombuffer(d_out1.cpu().numpy().tobytes(), dtype=bp.BOUNDS_DTYPE)[0])
        same(big, want_big, ("dev big", rep))
        same(got_host, O.bounds(Cs, ms, O.residual_reduce(Cs, rs, us)), ("host after dev", rep))
        dev2 = row_dict(np.frombuffer(d_out2.cpu().numpy().tobytes(), dtype=bp.BOUNDS_DTYPE)[0])
        same(dev2, O.bounds(C2, 3, items2), ("dev second stream", rep))
        same(got_host2, O.bounds(C2, 4, items2), ("host last", rep))


def test_repeated_calls_reuse_the_graph(ctx):
    rng = random.Random(707)
    insts = [rand_instance(rng, cmax=500, nmax=100) for _ in range(12)]
    want = [O.bounds(C, 4, it) for C, it in insts]
    for rep in range(3):
        for i, (C, it) in enumerate(insts):
            say("replay", rep, i)
            same(ctx.lower_bounds(C, 4, it), want[i], ("replay", rep, i))


def test_feasible_batch(ctx):
    b = W.uneven_batch(2, count=48, capacities=(1_000, 10_000), nmax=800)
    say("feasible_batch")
    v, lb = ctx.feasible_batch(b.C, b.k, [b.instance(i)[2] for i in range(len(b))])
    for i in range(len(b)):
        C, k, items = b.instance(i)
        want = O.bounds(C, k, items)
        assert v[i] == want["verdict"], i
        assert v[i] == (0 if b.expect_fail[i] else 1)
        if v[i] == 0:
            assert lb[i] > k
        else:
            assert lb[i] == want["lb"]


@pytest.mark.parametrize("shape", [(1, 8, 1, 64), (4, 32, 16, 128), (2, 16, 4, 1024), (4, 4, 64, 65536)])
def test_results_do_not_depend_on_the_sweep_shape(ctx, shape):
    rng = random.Random(808)
    insts = [rand_instance(rng, cmax=20000, nmax=700) for _ in range(40)]
    insts.append((100_000, list(W.large_residual(1)[3][:3000])))
    ks = [len(it) // 3 for _, it in insts]
    want = O.bounds_many([(C, k, it) for (C, it), k in zip(insts, ks)])
    old = ctx.get_tuning()
    try:
        ctx.set_tuning(*shape)
        say("shape", shape)
        out = ctx.lower_bounds_batch([c for c, _ in insts], ks, [it for _, it in insts])
        for i in range(len(insts)):
            same(row_dict(out[i]), want[i], ("shape", shape, i))
    finally:
        ctx.set_tuning(**old)


def test_autotuner_cache_and_schedule_order(ctx, tmp_path):
    rng = random.Random(818)
    insts = [rand_instance(rng, cmax=3000, nmax=250) for _ in range(64)]
    Cs = [c for c, _ in insts]
    ks = [rng.randint(0, len(it) + 1) for _, it in insts]
    its = [it for _, it in insts]
    want = O.bounds_many([(C, k, it) for (C, it), k in zip(insts, ks)])
    cache = str(tmp_path / "tuning.txt")
    say("autotuner cache")
    t1, ms1, hit1 = ctx.autotune_batch_cached(Cs, ks, its, cache, reps=1)
    t2, ms2, hit2 = ctx.autotune_batch_cached(Cs, ks, its, cache, reps=1)
    assert not hit1 and hit2 and t1 == t2 and ctx.get_tuning() == t2
    with open(cache) as fh:
        assert len(fh.read().splitlines()) == 1
    # results do not depend on the schedule order; records of the batched check carry the work done
    for order in ([bp.BP_MT, bp.BP_RAD2, bp.BP_FS1, bp.BP_CCM1, bp.BP_VB2, bp.BP_BJ1],
                  [bp.BP_CCM1, bp.BP_MT, bp.BP_BJ1, bp.BP_VB2, bp.BP_FS1, bp.BP_RAD2], None):
        ctx.set_order(order)
        out = ctx.lower_bounds_batch(Cs, ks, its)
        for i in range(len(insts)):
            same(row_dict(out[i]), want[i], ("order", order, i))
        v, lb, rec = ctx.feasible_batch(Cs, ks, its, records=True)
        assert np.array_equal(v, [w["verdict"] for w in want])
        assert (rec["evals_done"] <= rec["evals"]).all()
        assert (rec["evals_done"][rec["early_exit"] == 0] == rec["evals"][rec["early_exit"] == 0]).all()
    with pytest.raises(bp.BpError):
        ctx.set_order([bp.BP_MT] * 6)
    ctx.set_order(None)
    ctx.set_tuning(2, 32, 32, 2048)


def test_autotuner_keeps_results(ctx):
    rng = random.Random(909)
    insts = [rand_instance(rng, cmax=50000, nmax=400) for _ in range(24)]
    ks = [len(it) // 2 for _, it in insts]
    old = ctx.get_tuning()
    try:
        say("autotune")
        best, ms = ctx.autotune_batch([c for c, _ in insts], ks, [it for _, it in insts], reps=1)
        assert best == ctx.get_tuning() and ms > 0
        out = ctx.lower_bounds_batch([c for c, _ in insts], ks, [it for _, it in insts])
        want = O.bounds_many([(C, k, it) for (C, it), k in zip(insts, ks)])
        for i in range(len(insts)):
            same(row_dict(out[i]), want[i], ("tuned", i))
    finally:
        ctx.set_tuning(**old)


def test_stage_timing_averages_every_timed_call(ctx):
    rng = random.Random(1212)
    C, items = rand_instance(rng, cmax=5000, nmax=300)
    ctx.set_timing(True)
    try:
        for _ in range(70):  # more calls than the context keeps event sets for
            ctx.lower_bounds(C, len(items), items)
        ms, runs = ctx.stage_times(with_runs=True)
        assert runs == 70 and all(t > 0 for t in ms)
        ctx.set_timing(True)  # restarts the count
        with pytest.raises(bp.BpError):
            ctx.stage_times()
        ctx.lower_bounds(C, len(items), items)
        assert ctx.stage_times(with_runs=True)[1] == 1
    finally:
        ctx.set_timing(False)


@pytest.mark.parametrize("shape", [(4, 32, 64, 64), (1, 32, 64, 64), (2, 24, 64, 128)])
def test_heavily_split_tiles_repeatably_exact(ctx, shape):
    # tiles cut into many item chunks run by different waves, combined through
    # device-scope atomics: the same exact result on every repetition
    rng = np.random.default_rng(4242)
    C = 20_000
    items = rng.integers(C // 10, C // 2 + 1, size=3000).tolist() + [C - int(x) for x in rng.integers(C // 2, C, 600)]
    want = O.bounds(C, len(items) // 2, items)
    old = ctx.get_tuning()
    try:
        ctx.set_tuning(*shape)
        say("split", shape)
        for rep in range(8):
            same(ctx.lower_bounds(C, len(items) // 2, items), want, ("split", shape, rep))
    finally:
        ctx.set_tuning(**old)
