"""Pins of the CPU oracle to facts that do not come from the oracle itself.

Each test checks the oracle against something the paper or the mathematics
fixes: hand-worked values (tests/golden), the brute-force optimum on tiny
instances, dual feasibility by dynamic programming, closed forms and
invariants.  A plausible slip in any oracle function (a dropped term, a wrong
sign, a swapped operand, an off-by-one range) fails at least one of them.
"""
import math
import random

import numpy as np
import pytest

import oracle as O
from golden_io import dff_values, fig3, hand_bounds, param_counts, vb2_clamp
import oracle_par

NAME2ID = {n: i for i, n in enumerate(O.NAMES)}


# --- hand-worked fixtures ---------------------------------------------------

def test_fig3_reduction_and_bounds():
    g = fig3()
    C, k = g["C"][0], g["bins"][0]
    items = O.residual_reduce(C, g["residual"], g["unpacked"])
    assert sorted(items.tolist()) == sorted(g["reduced"])
    assert items.tolist() == g["reduced"]  # unpacked first, then one virtual item per loaded bin
    b = O.bounds(C, k, items, l2_dense=True)
    assert b["value"].tolist() == g["bounds"]
    assert b["verdict"] == g["verdict_k4"][0]
    assert O.bounds(C, k - 1, items)["verdict"] == g["verdict_k3"][0]


def test_fig3_assignment_form():
    # Same partial packing given as the constraint's variables: bin of each item.
    g = fig3()
    sizes = [5, 4, 2, 2, 3, 2, 2, 1]
    bin_of = [0, 1, 1, 2, 2, -1, -1, -1]
    items, residual = O.assignment_reduce(g["C"][0], g["bins"][0], sizes, bin_of)
    assert residual.tolist() == g["residual"]
    assert sorted(items.tolist()) == sorted(g["reduced"])


@pytest.mark.parametrize("row", dff_values(), ids=lambda r: f"{r[0]}-c{r[1]}-w{r[2]}-l{r[3]}")
def test_dff_hand_values(row):
    name, C, w, lam, want, _case = row
    assert O.f(NAME2ID[name], C, w, lam) == want


@pytest.mark.parametrize("row", hand_bounds(), ids=lambda r: r[0])
def test_hand_bounds(row):
    name, C, lam, want, want_l2, items = row
    b = O.bounds(C, len(items), items, l2_dense=True)
    assert b["value"][O.L2] == want_l2
    if name == "L2ODD":
        assert b["value"][O.L2] == want
        assert b["value"][O.MT] == 2  # MT falls short of L2 for odd c
        assert b["value"][O.L1] == 2
        return
    d = NAME2ID[name]
    assert b["value"][d] == want
    assert b["argmax"][d] <= lam
    # the witness parameter reaches the bound on its own
    v, _ = O.dff_bound(d, C, items, lam, lam)
    assert v == want


@pytest.mark.parametrize("row", param_counts(), ids=lambda r: f"c{r[0]}")
def test_parameter_counts(row):
    C, *counts, total = row
    got = []
    for d in O.DFFS:
        lo, hi = O.default_range(d, C)
        got.append(max(0, hi - lo + 1))
    assert got == counts
    assert sum(got) == total


# --- brute force ------------------------------------------------------------

def brute_force_opt(C, items):
    """Minimum number of bins of capacity C holding all items (tiny inputs)."""
    items = sorted((w for w in items if w > 0), reverse=True)
    best = [len(items)]
    loads = []

    def rec(i):
        if len(loads) >= best[0]:
            return
        if i == len(items):
            best[0] = len(loads)
            return
        w = items[i]
        tried = set()
        for j in range(len(loads)):
            if loads[j] + w <= C and loads[j] not in tried:
                tried.add(loads[j])
                loads[j] += w
                rec(i + 1)
                loads[j] -= w
        if len(loads) + 1 < best[0]:
            loads.append(w)
            rec(i + 1)
            loads.pop()

    rec(0)
    return best[0]


def test_brute_force_helper_itself():
    assert brute_force_opt(6, [6, 5, 5, 2, 2, 1]) == 4
    assert brute_force_opt(9, [5, 5, 5]) == 3
    assert brute_force_opt(10, [5, 5, 5, 5]) == 2
    assert brute_force_opt(10, []) == 0
    assert brute_force_opt(24, [18, 13, 8, 5, 2, 2]) == 3


def test_every_bound_at_most_optimum():
    rng = random.Random(20240222)
    seen_gap = 0
    for _ in range(600):
        C = rng.randint(1, 40)
        n = rng.randint(0, 8)
        items = [rng.randint(0, C) for _ in range(n)]
        opt = brute_force_opt(C, items)
        b = O.bounds(C, opt, items, l2_dense=True)
        assert (b["value"] <= opt).all(), (C, items, b["value"], opt)
        assert b["verdict"] == 1  # a packing into opt bins exists, so the check must not refute it
        if opt > 0:
            assert O.bounds(C, opt - 1, items)["verdict"] in (0, 1)
        seen_gap += int(b["lb"] < opt)
    assert seen_gap > 0  # the bounds are not trivially exact on this sample


def test_fail_verdict_is_sound_by_construction():
    # Items that fill m bins exactly need m bins: with m - 1 bins L1 already refutes.
    rng = random.Random(7)
    for _ in range(200):
        C = rng.randint(2, 60)
        m = rng.randint(1, 6)
        items = []
        for _b in range(m):
            left = C
            while left > 0:
                w = rng.randint(1, left)
                items.append(w)
                left -= w
        rng.shuffle(items)
        assert O.bounds(C, m, items)["verdict"] == 1
        b = O.bounds(C, m - 1, items)
        assert b["verdict"] == 0 and b["lb"] == m


# --- dual feasibility by dynamic programming ---------------------------------

@pytest.mark.parametrize("dff", O.DFFS, ids=lambda d: O.NAMES[d])
def test_dual_feasible_by_knapsack_dp(dff):
    """For every multiset of sizes with total <= c: sum f(w) <= f(c)  (c <= 30).

    This is the defining property of a dual feasible function; it is checked
    with an unbounded-knapsack table over the function's values."""
    for C in range(1, 31):
        lo, hi = O.default_range(dff, C)
        for lam in range(lo, hi + 1):
            fv = [O.f(dff, C, w, lam) for w in range(C + 1)]
            assert fv[0] == 0
            assert min(fv) >= 0
            best = [0] * (C + 1)
            for cap in range(1, C + 1):
                b = best[cap - 1]
                for w in range(1, cap + 1):
                    b = max(b, best[cap - w] + fv[w])
                best[cap] = b
            assert best[C] <= fv[C], (O.NAMES[dff], C, lam, best[C], fv[C])
            assert fv[C] >= 1  # the division in the bound is well defined


# --- closed forms and invariants ---------------------------------------------

def _rand_instance(rng, cmax=60, nmax=14):
    C = rng.randint(1, cmax)
    items = [rng.randint(0, C) for _ in range(rng.randint(0, nmax))]
    return C, items


def test_mt_at_zero_and_bj1_at_divisors_are_l1():
    rng = random.Random(3)
    for _ in range(300):
        C, items = _rand_instance(rng)
        l1 = O.l1(C, items)
        assert O.dff_bound(O.MT, C, items, 0, 0)[0] == l1
        for lam in (d for d in range(1, C + 1) if C % d == 0):
            assert O.dff_bound(O.BJ1, C, items, lam, lam)[0] == l1
        # L1 by its own arithmetic on exact rationals
        assert l1 == math.ceil(sum(items) / C) if items else l1 == 0


def test_l1_l2_mt_order_and_even_capacity_equivalence():
    rng = random.Random(11)
    n_even = 0
    for _ in range(400):
        C, items = _rand_instance(rng)
        b = O.bounds(C, 0, items, l2_dense=True)
        v = b["value"]
        assert v[O.L1] <= v[O.L2]
        assert v[O.MT] <= v[O.L2]
        if C % 2 == 0:
            n_even += 1
            assert v[O.MT] == v[O.L2], (C, items, v)
    assert n_even > 50


def test_full_item_adds_one_and_zero_item_adds_nothing():
    rng = random.Random(5)
    for _ in range(150):
        C, items = _rand_instance(rng, cmax=40, nmax=10)
        base = O.bounds(C, 0, items, l2_dense=True)["value"]
        plus_full = O.bounds(C, 0, items + [C], l2_dense=True)["value"]
        plus_zero = O.bounds(C, 0, items + [0, 0], l2_dense=True)["value"]
        # an empty range keeps its bound at 0 whatever the items (Alg. 2 starts L_f at 0)
        for b in range(O.NB):
            lo, hi = O.default_range(b, C) if b != O.L1 else (0, 0)
            if lo > hi:
                assert base[b] == 0 and plus_full[b] == 0
            else:
                assert plus_full[b] == base[b] + 1, (O.NAMES[b], C, items)
        assert (plus_zero == base).all()


def test_vb2_below_scaled_size():
    # f_VB2(w, lambda) <= 2 w lambda / c: each case is at most twice ceil(w lambda / c) - 1 < w lambda / c.
    for C in range(1, 40):
        for lam in range(2, C + 1):
            for w in range(C + 1):
                assert O.f(O.VB2, C, w, lam) * C <= 2 * w * lam


def test_piece_starts_match_every_lambda():
    rng = random.Random(13)
    for t in range(500):
        C, items = _rand_instance(rng, cmax=200 if t < 300 else 3000, nmax=12 if t < 300 else 80)
        for kind in (O.L2, O.MT, O.RAD2):
            lo, hi = O.default_range(kind, C)
            if kind == O.L2:
                dense = O.l2_dense(C, items)
            else:
                dense = O.dff_bound(kind, C, items, lo, hi)
            if lo > hi:
                continue
            assert O.piecewise_bound(kind, C, items) == dense, (O.NAMES[kind], C, items)


def test_event_sweep_matches_every_lambda():
    # the CCM1 / BJ1 event sweep against the per-lambda definition, on full
    # ranges and random sub-ranges, with the boundary sizes over-represented
    rng = random.Random(29)
    for t in range(700):
        C = rng.choice([rng.randint(1, 12), rng.randint(1, 200), rng.randint(1, 2500)])
        pool = [0, 1, C - 1, C, C // 2, (C + 1) // 2, max(0, C // 2 - 1), min(C, C // 2 + 1)]
        items = [rng.choice(pool) if rng.random() < 0.3 else rng.randint(0, C) for _ in range(rng.randint(0, 30))]
        for dff in (O.CCM1, O.BJ1):
            lo, hi = O.default_range(dff, C)
            if t % 2 and hi >= lo:
                lo = rng.randint(lo, hi)
                hi = rng.randint(lo - 1, hi)
            assert O.event_bound(dff, C, items, lo, hi) == O.dff_bound(dff, C, items, lo, hi), (
                O.NAMES[dff], C, lo, hi, items)
    # a medium capacity with many items: long runs of constant quotients
    r2 = np.random.default_rng(31)
    for C in (46_340, 65_536, 99_991):
        items = np.concatenate([r2.integers(C // 10, C // 2, 120), r2.integers(C // 2, C + 1, 40)])
        for dff in (O.CCM1, O.BJ1):
            assert O.event_bound(dff, C, items) == O.dff_bound(dff, C, items), (O.NAMES[dff], C)


def _definition_value(dff, C, items, lam):
    return -(-sum(O.f(dff, C, int(w), lam) for w in items) // O.f(dff, C, C, lam))


def test_event_sweep_at_huge_capacities():
    # where every lambda is out of reach: the reported maximum is attained at
    # the reported parameter, no sampled parameter beats it, none sampled
    # below it reaches it, BJ1 is at least L1 (lambda = c), and an instance
    # scaled by s has at least the bound of the original (f(s w, s lambda) at
    # capacity s c is s f(w, lambda) for BJ1 and f(w, lambda) for CCM1)
    r2 = np.random.default_rng(37)
    for C in (2**31 - 1, 2**30, 1_000_000_007, 2 * 3 * 5 * 7 * 11 * 13 * 17 * 19 * 23):
        items = np.concatenate([r2.integers(C // 3, C // 2 + 2, 25), r2.integers(C // 2, C + 1, 10),
                                r2.integers(0, C // 5, 15), [C // 2, C, 0]])
        for dff in (O.CCM1, O.BJ1):
            v, arg = O.event_bound(dff, C, items)
            lo, hi = O.default_range(dff, C)
            assert lo <= arg <= hi
            assert _definition_value(dff, C, items, arg) == v
            for lam in list(r2.integers(lo, hi + 1, 150)) + list(range(lo, min(hi, lo + 50) + 1)):
                g = _definition_value(dff, C, items, int(lam))
                assert g <= v and (g < v or lam >= arg), (O.NAMES[dff], C, lam)
            if dff == O.BJ1:
                assert v >= O.l1(C, items)
    base_C = 997
    base = [int(x) for x in r2.integers(200, base_C + 1, 40)]
    for s in (3, 1_000_003, 2_000_000):
        for dff in (O.CCM1, O.BJ1):
            v0 = O.dff_bound(dff, base_C, base)[0]
            assert O.event_bound(dff, base_C * s, [w * s for w in base])[0] >= v0


def test_event_sweep_rejects_what_it_cannot_do():
    with pytest.raises(O.OracleError):
        O.event_bound(O.VB2, 10, [3])
    with pytest.raises(O.OracleError):
        O.event_bound(O.BJ1, 10, [3], 0, 5)  # lambda = 0 is outside the definition
    with pytest.raises(O.OracleError):
        O.event_bound(O.BJ1, 10, [3], 1, 11)
    assert O.event_bound(O.BJ1, 10, [3], 5, 4) == (0, -1)
    assert O.event_bound(O.CCM1, 10, [], 1, 5) == (0, 1)


def test_reduction_forms_agree_and_keep_total_size():
    rng = random.Random(17)
    for _ in range(200):
        C = rng.randint(1, 50)
        m = rng.randint(0, 6)
        loads = [0] * m
        sizes, bin_of = [], []
        for _i in range(rng.randint(0, 12)):
            w = rng.randint(0, C)
            j = rng.randint(-1, m - 1)
            if j >= 0 and loads[j] + w <= C:
                loads[j] += w
            else:
                j = -1
            sizes.append(w)
            bin_of.append(j)
        items, residual = O.assignment_reduce(C, m, sizes, bin_of)
        assert sum(items) == sum(sizes)
        assert len(items) == sum(1 for j in bin_of if j < 0) + sum(1 for x in loads if x > 0)
        unpacked = [w for w, j in zip(sizes, bin_of) if j < 0]
        assert sorted(O.residual_reduce(C, residual, unpacked).tolist()) == sorted(items.tolist())


def test_empty_and_degenerate_inputs():
    b = O.bounds(1, 0, [])
    assert b["value"].tolist() == [0] * 8 and b["verdict"] == 1 and b["lb"] == 0
    # C = 1: sizes are 0 or 1, every bound counts the 1s (ranges per param_counts.txt)
    b = O.bounds(1, 3, [1, 1, 1, 0])
    assert b["value"][O.L1] == 3 and b["lb"] == 3 and b["verdict"] == 1
    assert b["value"][O.RAD2] == 0 and b["argmax"][O.RAD2] == -1
    assert O.bounds(1, 2, [1, 1, 1])["verdict"] == 0
    with pytest.raises(O.OracleError):
        O.bounds(5, 1, [6])
    with pytest.raises(O.OracleError):
        O.bounds(5, 1, [-1])
    with pytest.raises(O.OracleError):
        O.residual_reduce(5, [6], [])


def test_large_capacity_products_stay_exact():
    # c near 2^31: products c*lambda reach 2^62; compare with Python's exact integers
    C = 2**31 - 1
    for w, lam in [(C, C), (C - 1, C), (C // 2 + 1, C - 3), (12345, C), (C // 2, C)]:
        got = O.f(O.VB2, C, w, lam)
        if 2 * w > C:
            a, b = -(-C * lam // C) - 1, -(-(C * lam - w * lam) // C) - 1
            want = 2 * max(0, a) - 2 * max(0, b)
        elif 2 * w == C:
            want = max(0, -(-C * lam // C) - 1)
        else:
            want = 2 * max(0, -(-w * lam // C) - 1)
        assert got == want
    for w, lam in [(C, 100), (C - 1, 100), (C // 3, 99)]:
        num = w * (lam + 1)
        want = w * lam if num % C == 0 else (num // C) * C
        assert O.f(O.FS1, C, w, lam) == want


# --- the paper's VB2 cut (Sec. 4, "Implementation details") -------------------


@pytest.mark.parametrize("row", vb2_clamp(), ids=lambda r: f"c{r[0]}-r{r[1]}-w{r[2]}")
def test_vb2_clamp_hand_values(row):
    C, r, maxw, want_hi = row
    assert O.default_range(O.VB2, C, r, maxw, clamp_vb2=True) == (2, want_hi)
    assert O.default_range(O.VB2, C, r, maxw, clamp_vb2=False) == (2, C)
    # the cut touches only VB2
    for b in range(O.NB):
        if b != O.VB2:
            assert O.default_range(b, C, r, maxw, clamp_vb2=True) == O.default_range(b, C)


def test_vb2_clamp_keeps_32_bit_products():
    # Where the cut binds, hi is the largest parameter with r * max w * hi <= 2^32 - 1
    # (the paper's reason for it), checked by that inequality on both sides.
    rng = random.Random(23)
    for _ in range(2000):
        C = rng.randint(1, 2**31 - 1)
        r = rng.randint(0, 20000)
        maxw = rng.randint(0, C)
        lo, hi = O.default_range(O.VB2, C, r, maxw, clamp_vb2=True)
        assert lo == 2 and hi <= C
        d = r * maxw
        if d == 0:
            assert hi == C  # no items: nothing to cut
        elif hi == C:
            assert d * C <= 2**32 - 1  # the cut lies past c
        else:
            assert d * hi <= 2**32 - 1 < d * (hi + 1)


# --- the thread-pool helper used for full-size records --------------------------


def test_pooled_record_equals_single_pass():
    # cutting every range into chunks (down to one parameter) keeps the maximum
    # and the smallest maximiser of one pass over the range
    rng = random.Random(29)
    for t in range(60):
        C, items = _rand_instance(rng, cmax=400, nmax=25)
        k = rng.randint(0, len(items) + 1)
        want = O.bounds(C, k, items, l2_dense=True)
        for chunk in (1, 3, 17, None):
            got = oracle_par.dense_record(C, k, items, threads=4, chunk=chunk)
            for f in ("value", "argmax"):
                assert np.array_equal(got[f], want[f]), (t, chunk, f, got[f], want[f])
            assert (got["lb"], got["lb_arg"], got["verdict"]) == (want["lb"], want["lb_arg"], want["verdict"])
