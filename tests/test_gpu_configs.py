"""GPU parity on the batch workloads: the uneven mixed-capacity batch and the
triplet-tight batch with huge capacities.

Every instance of each batch runs on the GPU in one launch.  Verdicts are
pinned for all of them by construction; full records are compared with the
oracle on seeded samples the oracle finishes in seconds, and the full ranges
of a few triplet instances with the oracle's piece-start and event sweeps.
"""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle as O
import paper_2402_14821_amd as bp
from paper_2402_14821_amd import workloads as W

pytestmark = pytest.mark.gpu

WINDOW = 8192  # parameters kept at each end of a long range


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


def window_sweeps(C):
    """Low-end and high-end windowed sweeps of capacity C: every DFF range
    longer than two windows keeps its first (resp. last) WINDOW parameters,
    shorter ranges and L2 stay whole."""
    sides = []
    for side in (0, 1):
        lo, hi = [0] * O.NB, [-1] * O.NB
        for b in range(1, O.NB):
            dlo, dhi = O.default_range(b, C)
            win = W.windows(dlo, dhi, WINDOW) if dlo <= dhi else [(1, 0)]
            if b == O.L2 or len(win) == 1:
                lo[b], hi[b] = (dlo, dhi) if dlo <= dhi else (1, 0)
            else:
                lo[b], hi[b] = win[side]
        sides.append((lo, hi))
    return sides


def test_uneven_batch_verdicts_and_sample(ctx):
    b = W.uneven_batch(2, count=4096)
    items = [b.instance(i)[2] for i in range(len(b))]
    say("uneven batch 4096")
    out = ctx.lower_bounds_batch(b.C, b.k, items)
    assert (out["status"] == 0).all()
    assert np.array_equal(out["verdict"] == 0, b.expect_fail)
    v, lb = ctx.feasible_batch(b.C, b.k, items)
    assert np.array_equal(v, out["verdict"])
    assert (lb[v == 0] > b.k[v == 0]).all() and np.array_equal(lb[v == 1], out["lb"][v == 1])
    rng = np.random.default_rng(22)
    small = np.flatnonzero(b.C < 1_000_000)
    large = np.flatnonzero(b.C == 1_000_000)
    large = large[np.argsort([len(items[i]) for i in large])][:2]  # the two cheapest for the oracle
    pick = list(rng.choice(small, size=48, replace=False)) + list(large)
    want = O.bounds_many([(int(b.C[i]), int(b.k[i]), items[i]) for i in pick])
    for j, i in enumerate(pick):
        same(bp.bounds_to_dict(out[i]), want[j], ("uneven", int(i), int(b.C[i]), len(items[i])))


def test_triplet_batch_windowed(ctx):
    tb = W.triplet_batch(5, count=1024)
    Cs, ks, its, sweeps, owner = [], [], [], [], []
    for i in range(len(tb)):
        C, k, items = tb.instance(i)
        for lo, hi in window_sweeps(C):
            Cs.append(C)
            ks.append(k)
            its.append(items)
            sweeps.append(bp.make_sweep(lo, hi))
            owner.append(i)
    say("triplet batch", len(tb), "x 2 windows")
    out = ctx.lower_bounds_batch(np.array(Cs), np.array(ks), its, sweeps)
    assert (out["status"] == 0).all()
    for j, i in enumerate(owner):
        C, k, items = tb.instance(i)
        m = len(items) // 3  # the triplets fill exactly m bins: OPT = m = L1
        vals = out["value"][j]
        assert vals[O.L1] == m and (vals <= m).all() and out["lb"][j] == m, (i, vals)
        assert out["verdict"][j] == (0 if tb.expect_fail[i] else 1)
        assert vals[O.L2] == m  # every size is below C/2, so L2 = L1
    rng = np.random.default_rng(55)
    pick = sorted(rng.choice(len(tb), size=4, replace=False))
    cases, rows = [], []
    for i in pick:
        C, k, items = tb.instance(int(i))
        for s, (lo, hi) in enumerate(window_sweeps(C)):
            cases.append((C, k, items, lo, hi))
            rows.append(2 * int(i) + s)
    want = O.bounds_many(cases)
    for j, row in enumerate(rows):
        same(bp.bounds_to_dict(out[row]), want[j], ("triplet", row))


def test_triplet_full_ranges_by_construction(ctx):
    # full parameter ranges (up to 2^31 - 1) on the instances with the largest
    # and the smallest capacities; pinned by the construction alone
    # and every bound but VB2 against the oracle's piece-start and event sweeps
    tb = W.triplet_batch(5, count=1024)
    order = np.argsort(tb.C)
    pick = [int(i) for i in list(order[:3]) + list(order[-2:])]
    with ThreadPoolExecutor(max_workers=5) as ex:
        wants = list(ex.map(lambda i: O.bounds_by_pieces(*tb.instance(i), threads=6), pick))
    for i, want in zip(pick, wants):
        C, k, items = tb.instance(i)
        m = len(items) // 3
        say("triplet full range", i, C, len(items))
        got = ctx.lower_bounds(C, k, items)
        assert got["status"] == 0
        assert got["value"][O.L1] == m and (got["value"] <= m).all() and got["lb"] == m
        assert got["verdict"] == (0 if tb.expect_fail[i] else 1)
        P = sum(max(0, hi - lo + 1) for lo, hi in (O.default_range(d, C) for d in O.DFFS))
        assert got["evals"] == len(items) * P
        keep = [b for b in range(O.NB) if b != O.VB2]
        assert np.array_equal(got["value"][keep], want["value"][keep]), (i, got["value"], want["value"])
        assert np.array_equal(got["argmax"][keep], want["argmax"][keep]), (i, got["argmax"], want["argmax"])
