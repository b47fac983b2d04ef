"""C-ABI boundary on the CPU: the library loads, exports every declared entry
point, and its host-side logic (parameter ranges, argument checks, the
multiply-shift constants of the kernels) behaves as documented.  No device
work is started here."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2402_14821_amd as bp
from golden_io import param_counts

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    with open(os.path.join(ROOT, "include", "bp.h")) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"^\s*(?:const\s+char\s*\*|bp_status|int64_t|int32_t)\s*(bp_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    lib = bp.load()
    decl = declared_symbols()
    assert len(decl) >= 19
    for name in decl:
        assert hasattr(lib, name), name
    assert sorted(decl) == sorted(bp.exported_symbols())


def test_struct_sizes_match_header_layout():
    assert ctypes.sizeof(bp.bp_sweep) == 8 * 8 * 2 + 8
    assert ctypes.sizeof(bp.bp_bounds) == 8 * 8 * 2 + 8 + 4 + 4 + 8 * 3 + 4 + 4 + 8
    assert ctypes.sizeof(bp.bp_batch) == 8 + 4 * 8
    assert bp.BOUNDS_DTYPE.itemsize == ctypes.sizeof(bp.bp_bounds)
    assert ctypes.sizeof(bp.bp_solve_opts) == 4 + 4 + 8 + 8 + 8 + 8 + 4 + 4
    assert ctypes.sizeof(bp.bp_solve_result) == 6 * 4 + 4 * 8 + 2 * 8 + 8


def test_version_and_error_text():
    lib = bp.load()
    assert b"gfx950" in lib.bp_version()
    assert lib.bp_ctx_destroy(None) == bp.BP_ERR_STATE
    assert b"context" in lib.bp_last_error()


@pytest.mark.parametrize("row", param_counts(), ids=lambda r: f"c{r[0]}")
def test_default_sweep_matches_hand_counted_ranges(row):
    C, *counts, total = row
    sw = bp.default_sweep(C)
    got = [max(0, sw.hi[b] - sw.lo[b] + 1) for b in (bp.BP_MT, bp.BP_RAD2, bp.BP_FS1, bp.BP_CCM1, bp.BP_VB2, bp.BP_BJ1)]
    assert got == counts and sum(got) == total
    assert sw.lo[bp.BP_L2] == 0 and sw.hi[bp.BP_L2] == C // 2


def test_default_sweep_vb2_clamp():
    # floor((2^32 - 1) / (r * max w)) as in the paper's overflow note
    sw = bp.default_sweep(100_000, 14_000, 50_000, bp.BP_SWEEP_PAPER_VB2_CLAMP)
    assert sw.hi[bp.BP_VB2] == (2**32 - 1) // (14_000 * 50_000)
    sw = bp.default_sweep(150, 50, 100, bp.BP_SWEEP_PAPER_VB2_CLAMP)
    assert sw.hi[bp.BP_VB2] == 150  # the cut is above c there
    sw = bp.default_sweep(10**9, 3000, 10**9 // 2, bp.BP_SWEEP_PAPER_VB2_CLAMP)
    assert sw.hi[bp.BP_VB2] < sw.lo[bp.BP_VB2]  # empty


def test_argument_errors_without_device():
    lib = bp.load()
    sw = bp.bp_sweep()
    assert lib.bp_default_sweep(0, 0, 0, 0, ctypes.byref(sw)) == bp.BP_ERR_ARG
    assert lib.bp_default_sweep(10, 0, 0, 0x10, ctypes.byref(sw)) == bp.BP_ERR_ARG
    assert lib.bp_default_sweep(10, 0, 0, 0, None) == bp.BP_ERR_ARG
    out = bp.bp_bounds()
    items = np.array([1, 2], dtype=np.int32)
    assert lib.bp_lower_bounds(None, 10, 1, items.ctypes.data_as(bp._P32), 2, None, ctypes.byref(out)) == bp.BP_ERR_STATE
    assert lib.bp_queue_destroy(None) == bp.BP_ERR_STATE
    t = bp.bp_tuning(2, 32, 8, 384)
    assert lib.bp_ctx_set_tuning(None, ctypes.byref(t)) == bp.BP_ERR_STATE
    assert lib.bp_queue_poll(None, None, 0, None, 0) == bp.BP_ERR_STATE


def test_division_constants_small_divisors_exhaustive():
    # floor(n / d) = mulhi(2n, m) >> s for every d < 2^11 and n < 2^13 (plus multiples of d and the top of the range)
    assert bp.selftest_division(1, 2048, 8192, 0) == 0


def test_division_constants_edge_divisors():
    for lo, hi in [(2**15 - 3, 2**15 + 3), (2**16 - 2, 2**16 + 2), (2**20 - 1, 2**20 + 1), (2**30 - 2, 2**30 + 2),
                   (2**31 - 4, 2**31 - 1), (99_999, 100_001), (999_999, 1_000_001)]:
        assert bp.selftest_division(lo, hi, 4096, 0) == 0, (lo, hi)


def test_vb2_reciprocal_exhaustive_small_capacities():
    # ceil(a lambda / c) - 1 for every c <= 160, lambda <= c, a <= c
    assert bp.selftest_division(1, 160, 1 << 20, 1) == 0


def test_vb2_reciprocal_large_capacities():
    for c in (10_000, 100_000, 1_000_000, 2**25, 2**31 - 1, 2**31 - 2, 1_999_999_973):
        assert bp.selftest_division(c, c, 2048, 1) == 0, c


def test_divisibility_test_exhaustive_small_divisors():
    # d | n as n * ceil(2^64 / d) mod 2^64 <= ceil(2^64 / d) - 1, every d < 2^11 and n < 2^13 (plus multiples)
    assert bp.selftest_division(1, 2048, 8192, 2) == 0


def test_divisibility_test_edge_divisors():
    # divisors of the capacities the segment sums meet, powers of two and the top of the int32 range
    for lo, hi in [(2**15 - 3, 2**15 + 3), (2**20 - 1, 2**20 + 1), (2**30 - 2, 2**30 + 2), (2**31 - 4, 2**31 - 1),
                   (3125, 3125), (50_000, 50_000), (99_999, 100_001), (999_999, 1_000_001)]:
        assert bp.selftest_division(lo, hi, 4096, 2) == 0, (lo, hi)


def test_fp64_floor_small_divisors_exhaustive():
    # floor(n / d) = truncation of n * fl(1/d), one correction step: every d < 2^11, n < 2^13, multiples, top
    assert bp.selftest_division(1, 2048, 8192, 3) == 0


def test_fp64_floor_edge_divisors():
    for lo, hi in [(2**15 - 3, 2**15 + 3), (2**20 - 1, 2**20 + 1), (2**30 - 2, 2**30 + 2), (2**31 - 4, 2**31 - 1),
                   (99_999, 100_001), (999_999, 1_000_001), (1_999_999_973, 1_999_999_973)]:
        assert bp.selftest_division(lo, hi, 4096, 3) == 0, (lo, hi)


def test_fp64_floor_vb2_quotient():
    # floor((a lambda - 1) / c) for a, lambda <= c: every c <= 300, and large capacities near the int32 top
    assert bp.selftest_division(1, 300, 1 << 20, 4) == 0
    for c in (10_000, 100_000, 1_000_000, 2**25, 2**31 - 1, 2**31 - 2, 1_999_999_973):
        assert bp.selftest_division(c, c, 4096, 4) == 0, c


def test_short_quotient_small_divisors_exhaustive():
    # floor(n / d) = mulhi(n, ceil(2^32 / d)) wherever n d <= 2^32: every 2 <= d < 2^11, n < 2^13, multiples of d
    # and the limit floor(2^32 / d) itself
    assert bp.selftest_division(1, 2048, 8192, 5) == 0


def test_short_quotient_edge_divisors():
    for lo, hi in [(2**15 - 3, 2**15 + 3), (2**16 - 2, 2**16 + 2), (42_949, 42_951), (50_000, 50_001),
                   (85_898, 85_900), (99_999, 100_001), (2**20 - 1, 2**20 + 1), (2**31 - 4, 2**31 - 1)]:
        assert bp.selftest_division(lo, hi, 4096, 5) == 0, (lo, hi)


def test_vb2_short_form_small_capacities_exhaustive():
    # ceil(a lambda / c) - 1 = mulhi(a, R_hi) for every c <= 160, lambda <= c, a <= c (a c <= 2^32 throughout)
    assert bp.selftest_division(1, 160, 1 << 20, 6) == 0


def test_vb2_short_form_large_capacities():
    # capacities where a c <= 2^32 cuts a below c / 2 (the limit and the a just under it included)
    for c in (65_536, 65_537, 92_681, 92_682, 100_000, 1_000_000, 2**25, 2**31 - 1):
        assert bp.selftest_division(c, c, 2048, 6) == 0, c


def test_selftest_rejects_bad_ranges():
    assert bp.selftest_division(0, 10, 10, 0) == bp.BP_ERR_ARG
    assert bp.selftest_division(10, 5, 10, 0) == bp.BP_ERR_ARG
    assert bp.selftest_division(1, 10, 10, 7) == bp.BP_ERR_ARG


def test_workload_generators_are_seeded_and_shaped():
    from paper_2402_14821_amd import workloads as W
    a = W.small_partial_packing(3)
    b = W.small_partial_packing(3)
    assert all(np.array_equal(x, y) for x, y in zip(a[2:], b[2:]))
    C, m, res, unp = a
    assert C == 150 and m == 20 and len(res) == 20
    assert (unp >= 20).all() and (unp <= 100).all() and (res >= 0).all() and (res <= C).all()
    C, m, res, unp = W.large_residual(1)
    assert len(unp) == 10_000 and unp.min() >= 10_000 and unp.max() <= 50_000
    assert res.min() >= 50_000 and res.max() <= 100_000
    tb = W.triplet_batch(5, count=4)
    for i in range(4):
        C, k, items = tb.instance(i)
        assert len(items) % 3 == 0 and 4 * items.min() > C and 2 * items.max() < C
        assert int(items.astype(np.int64).sum()) == C * (len(items) // 3)
        assert k in (len(items) // 3, len(items) // 3 - 1)
    ub = W.uneven_batch(2, count=32)
    assert len(ub) == 32 and ub.off[-1] == len(ub.items)
    for i in range(32):
        C, k, items = ub.instance(i)
        assert 50 <= len(items) <= 5000 and items.min() >= 1 and items.max() <= C
        total = int(items.astype(np.int64).sum())
        if ub.expect_fail[i]:
            assert k * C < total
        else:
            assert k >= -(-total // C)
