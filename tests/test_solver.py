"""The propagator and the search around the check (Alg. 1, Sec. 5), on the CPU.

bp_solve takes the check as a caller's function here: the oracle's lower
bound of each node's reduced instance.  The optimum it reports must equal a
brute-force optimum on tiny instances under every combination of the
filtering and dominance rules, every packing it returns must be valid, and
the knapsack test the rules rest on must never claim a gap that a subset
sum falls into.  The GPU tests run the same searches with the library's
check and require the identical trajectory."""
import itertools
import random

import numpy as np
import pytest

import oracle as O
import paper_2402_14821_amd as bp
from paper_2402_14821_amd import workloads as W
from test_oracle_pins import brute_force_opt


def oracle_lb(C, residual, unpacked):
    return O.bounds(C, len(residual), O.residual_reduce(C, residual, unpacked))["lb"]


def oracle_l2_lb(C, residual, unpacked):
    items = O.residual_reduce(C, residual, unpacked)
    lo, hi = [1] * O.NB, [0] * O.NB
    lo[O.L2], hi[O.L2] = O.default_range(O.L2, C)
    return O.bounds(C, len(residual), items, lo, hi, l2_dense=True)["lb"]


def valid_packing(C, sizes, bin_of, bins):
    assert len(bin_of) == len(sizes)
    assert all(0 <= b < bins for b in bin_of)
    load = np.zeros(bins, dtype=np.int64)
    np.add.at(load, np.asarray(bin_of), np.asarray(sizes, dtype=np.int64))
    assert (load <= C).all()


def subset_sums(x):
    sums = {0}
    for v in x:
        sums |= {s + v for s in sums}
    return sums


def test_subset_sum_gap_never_hides_a_sum():
    rng = random.Random(5)
    proved = 0
    for _ in range(3000):
        x = [rng.randint(0, rng.choice((5, 20, 60))) for _ in range(rng.randint(0, 9))]
        sums = subset_sums(x)
        top = sum(x) + 3
        a = rng.randint(-2, top)
        b = a + rng.randint(0, 12)
        g = bp.subset_sum_gap(x, a, b)
        if g is None:
            continue
        proved += 1
        below, above = g
        assert below < a <= b < above, (x, a, b, g)
        assert not any(below < s < above for s in sums), (x, a, b, g)
    assert proved > 300


def test_subset_sum_gap_cases():
    assert bp.subset_sum_gap([7, 3], 4, 6) == (3, 7)      # sums 0 3 7 10
    assert bp.subset_sum_gap([5, 5, 5], 6, 9) == (5, 10)
    assert bp.subset_sum_gap([5, 5, 1], 7, 9) == (6, 10)    # sums 0 1 5 6 10 11
    assert bp.subset_sum_gap([4, 3], 8, 9) == (7, 2**61 - 1)  # above the total
    assert bp.subset_sum_gap([4, 3], 0, 2) is None          # the empty set sums to 0
    assert bp.subset_sum_gap([4, 3, 2, 1], 5, 5) is None    # 4 + 1
    assert bp.subset_sum_gap([], 1, 1) == (0, 2**61 - 1)
    assert bp.load().bp_subset_sum_gap(None, 2, 1, 1, None, None) == bp.BP_ERR_ARG
    x = np.array([1, 2], dtype=np.int32)  # not sorted
    lo, hi = bp._i64(), bp._i64()
    assert bp.load().bp_subset_sum_gap(bp._p32(x), 2, 1, 1, bp.ctypes.byref(lo), bp.ctypes.byref(hi)) == bp.BP_ERR_ARG


RULE_SETS = [0, bp.BP_SOLVE_OFF_KNAPSACK, bp.BP_SOLVE_OFF_SINGLE, bp.BP_SOLVE_OFF_FILL | bp.BP_SOLVE_OFF_SYMMETRY,
             bp.BP_SOLVE_OFF_KNAPSACK | bp.BP_SOLVE_OFF_SINGLE | bp.BP_SOLVE_OFF_FILL | bp.BP_SOLVE_OFF_SYMMETRY]


def test_tiny_instances_reach_the_brute_force_optimum():
    rng = random.Random(41)
    for _ in range(160):
        C = rng.randint(1, 30)
        n = rng.randint(1, 8)
        sizes = [rng.randint(1, C) for _ in range(n)]
        opt = brute_force_opt(C, sizes)
        runs = [(oracle_lb, bp.BP_SOLVE_DFFS, 0), (oracle_l2_lb, bp.BP_SOLVE_L2, 0)]
        runs += [(None, bp.BP_SOLVE_NO_CHECK, d) for d in RULE_SETS]
        for check, mode, disable in runs:
            res, bin_of = bp.solve(C, sizes, mode=mode, check=check, disable=disable)
            assert res["status"] == bp.BP_SOLVE_OPTIMAL, (C, sizes, res)
            assert res["bins"] == opt, (C, sizes, disable, res, opt)
            assert res["lower"] <= opt <= res["upper"]
            valid_packing(C, sizes, bin_of, res["bins"])


def test_tight_instances_reach_the_optimum_under_every_rule_set():
    # instances built from a known perfect packing: the optimum is m bins
    rng = random.Random(7)
    for _ in range(40):
        C = rng.randint(20, 60)
        m = rng.randint(2, 4)
        sizes = []
        for _ in range(m):
            left = C
            while left > 0:
                v = min(left, rng.randint(1, C // 2 + 1))
                sizes.append(v)
                left -= v
        sizes = sizes[:10] if len(sizes) > 10 else sizes
        opt = brute_force_opt(C, sizes)
        for disable in RULE_SETS:
            res, bin_of = bp.solve(C, sizes, mode=bp.BP_SOLVE_NO_CHECK, disable=disable)
            assert res["status"] == bp.BP_SOLVE_OPTIMAL and res["bins"] == opt, (C, sizes, disable, res, opt)
            valid_packing(C, sizes, bin_of, res["bins"])


@pytest.mark.parametrize("shape,sigma,seed", [(2.0, 1.2, 20), (2.5, 1.4, 25), (4.0, 1.2, 40)])
def test_weibull_searches(shape, sigma, seed):
    """Weibull instances of Sec. 5 (n = 100) that need a search: the check
    prunes nodes that filtering alone does not, and every packing is valid."""
    C, sizes = W.weibull_instance(seed=seed, n=100, shape=shape, sigma=sigma)
    a, pa = bp.solve(C, sizes, check=oracle_l2_lb, max_nodes=20_000)
    b, pb = bp.solve(C, sizes, mode=bp.BP_SOLVE_NO_CHECK, max_nodes=20_000)
    assert a["status"] == b["status"] == bp.BP_SOLVE_OPTIMAL
    assert a["bins"] == b["bins"]
    assert a["lower"] >= b["lower"]  # L2 at the root is at least L1
    valid_packing(C, sizes, pa, a["bins"])
    valid_packing(C, sizes, pb, b["bins"])
    assert a["checks"] >= a["nodes"] > 0 and b["checks"] == 0


def test_limits_and_errors():
    C, sizes = W.weibull_instance(seed=20, n=100, shape=2.0, sigma=1.0)
    res, bin_of = bp.solve(C, sizes, mode=bp.BP_SOLVE_NO_CHECK, max_nodes=50)
    assert res["status"] == bp.BP_SOLVE_LIMIT and res["limit_reached"] == 1
    assert res["bins"] == res["upper"]  # first fit decreasing's packing comes back
    valid_packing(C, sizes, bin_of, res["bins"])
    res, _ = bp.solve(C, sizes, mode=bp.BP_SOLVE_NO_CHECK, time_limit_s=0.05)
    assert res["status"] == bp.BP_SOLVE_LIMIT and res["seconds"] < 5
    res, bin_of = bp.solve(C, [], mode=bp.BP_SOLVE_NO_CHECK)
    assert res["bins"] == 0 and res["status"] == bp.BP_SOLVE_OPTIMAL
    with pytest.raises(bp.BpError) as e:
        bp.solve(C, sizes)  # the library's check needs a context
    assert e.value.status == bp.BP_ERR_ARG
    with pytest.raises(bp.BpError) as e:
        bp.solve(10, [11], mode=bp.BP_SOLVE_NO_CHECK)
    assert e.value.status == bp.BP_ERR_RANGE
    with pytest.raises(bp.BpError) as e:
        bp.solve(10, [1], mode=7, check=oracle_lb)
    assert e.value.status == bp.BP_ERR_ARG

    def broken(C_, res_, unp_):
        raise RuntimeError("no check")
    with pytest.raises(bp.BpError) as e:
        bp.solve(C, sizes, check=broken)
    assert e.value.status == bp.BP_ERR_STATE


def test_weibull_generator_follows_the_recipe():
    for shape in (0.5, 1.0, 5.0):
        for sigma in (1.0, 1.2, 2.0):
            C, w = W.weibull_instance(seed=1, n=100, shape=shape, sigma=sigma)
            assert len(w) == 100 and w.min() >= 1 and C == round(sigma * int(w.max()))
            C2, w2 = W.weibull_instance(seed=1, n=100, shape=shape, sigma=sigma)
            assert C2 == C and np.array_equal(w, w2)
