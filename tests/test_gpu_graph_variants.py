"""Pipeline variants of one context against the oracle.

A launch replays a captured graph that holds the large-instance prep only
when some instance has more than 8 192 reduced items, and the combine kernel
only when some tile is split into chunks; a context caches one graph per
variant.  One context here alternates between the four variants (each call
made twice, so every cached graph is also replayed after the others ran),
and every record must equal the oracle's, field by field.

Which variant a call takes follows from the planner's rules: an instance of
at most 8 192 items with fewer than 512 items splits nothing; one of 3 000
items splits FS1's single tile; one of 9 000 items is large and, with the
default shape, splits its tiles; with chunks of at least 65 536 items and no
FS1 or RAD2 range (the bounds whose few tiles would still be split) it
splits nothing.
"""
import os
import sys

import numpy as np
import pytest

import oracle as O
import paper_2402_14821_amd as bp

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def same(got, want, what=""):
    assert got["status"] == 0, (what, got)
    assert np.array_equal(got["value"], want["value"]), (what, got["value"], want["value"])
    assert np.array_equal(got["argmax"], want["argmax"]), (what, got["argmax"], want["argmax"])
    assert got["lb"] == want["lb"] and got["lb_arg"] == want["lb_arg"], (what, got, want)
    assert got["verdict"] == want["verdict"], what


def _case(name, C, r, seed, drop=()):
    rng = np.random.default_rng(seed)
    items = rng.integers(1, C + 1, size=r).astype(np.int32)
    k = int(-(-int(items.sum()) // C))
    full = bp.default_sweep(C)
    lo = [int(full.lo[b]) for b in range(bp.BP_NB)]
    hi = [int(full.hi[b]) for b in range(bp.BP_NB)]
    for b in drop:
        lo[b], hi[b] = 1, 0
    return {"name": name, "C": C, "k": k, "items": items, "lo": lo, "hi": hi, "drop": tuple(drop)}


def test_variants_alternate_in_one_context():
    cases = {
        "small": _case("small", 150, 40, 11),
        "small_split": _case("small_split", 1000, 3000, 12),
        "large_whole": _case("large_whole", 2000, 9000, 13, drop=(bp.BP_FS1, bp.BP_RAD2)),
        "large_split": _case("large_split", 2000, 9000, 14),
    }
    want = {}
    for name, c in cases.items():
        lo = hi = None
        if c["drop"]:
            lo, hi = c["lo"], c["hi"]
        want[name] = O.bounds(c["C"], c["k"], c["items"], lo, hi)
    # the pipeline itself: small checks would otherwise take the one-launch path
    old = os.environ.get("BP_NO_SMALL_PATH")
    os.environ["BP_NO_SMALL_PATH"] = "1"
    try:
        ctx = bp.Context(0)
    finally:
        if old is None:
            os.environ.pop("BP_NO_SMALL_PATH", None)
        else:
            os.environ["BP_NO_SMALL_PATH"] = old
    with ctx:
        default = ctx.get_tuning()
        for name in ("small", "large_split", "small_split", "large_whole", "small", "large_whole", "large_split",
                     "small_split"):
            c = cases[name]
            if name == "large_whole":
                ctx.set_tuning(default["lanes_params"], default["waves_per_cu"], default["tasks_per_wave"], 65536)
            sweep = bp.make_sweep(c["lo"], c["hi"]) if c["drop"] else None
            for rep in range(2):
                say("graph variant", name, "C", c["C"], "r", len(c["items"]), "rep", rep)
                same(ctx.lower_bounds(c["C"], c["k"], c["items"], sweep), want[name], (name, rep))
            if name == "large_whole":
                ctx.set_tuning(default["lanes_params"], default["waves_per_cu"], default["tasks_per_wave"],
                               default["min_chunk"])
