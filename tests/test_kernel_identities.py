"""The per-class arithmetic the sweep kernels evaluate, checked on the CPU
against the oracle's f (Sec. 3.1's definitions).

The kernels never call f: for each DFF they stream the big (c/2 < w < c) and
small (0 < 2w < c) sizes, or every size strictly between 0 and c, through a
rewritten form -- sign-bit masks, threshold counts, a doubled quotient, a
clamp summed by absolute differences.  Each rewrite is an identity per
(size, parameter); these tests put random and edge triples through it with
Python integers and compare with oracle.f, so a wrong sign, term or case
split in a rewrite fails here without a GPU.  (Division by multiplication
is checked separately by bp_selftest_division.)"""
import random

import oracle as O

CAPS = [2, 3, 4, 5, 6, 7, 9, 10, 150, 1_000, 4_096, 65_537, 100_000, 1_000_000, 2**31 - 1]


def cases(rng, lo_of, hi_of, n=1500):
    """(C, lam, w) triples: every capacity of CAPS and random ones, lam in
    [lo_of(C), hi_of(C)] (its ends included), w in (0, C)."""
    out = []
    for C in CAPS + [rng.randint(2, 10**7) for _ in range(20)]:
        lo, hi = lo_of(C), hi_of(C)
        if hi < lo or C < 2:
            continue
        lams = {lo, hi, (lo + hi) // 2} | {rng.randint(lo, hi) for _ in range(8)}
        for lam in lams:
            ws = {1, C - 1, C // 2, (C + 1) // 2, max(1, lam - 1), min(C - 1, lam), min(C - 1, lam + 1),
                  max(1, C - lam), min(C - 1, C - lam + 1)}
            ws |= {rng.randint(1, C - 1) for _ in range(max(1, n // 200))}
            out += [(C, lam, w) for w in ws if 0 < w < C]
    return out


def test_mt_masks():
    # big: w + [c - w < lam] (c - w); small: [w >= lam] w; mid (2w = c): c/2
    rng = random.Random(1)
    for C, lam, w in cases(rng, lambda C: 0, lambda C: C // 2):
        if 2 * w > C:
            want = w + ((C - w) if C - w < lam else 0)
        elif 2 * w < C:
            want = w if w >= lam else 0
        else:
            want = C // 2
        assert O.f(O.MT, C, w, lam) == want, (C, lam, w)


def test_rad2_threshold_counts():
    # c3 = floor(c/3), c2 = floor(c/2); small: c3 [w >= lam] + (c2 - c3) [w > c - 2 lam];
    # big: c2 + (c - c2 - c3) [w >= 2 lam] + c3 [w > c - lam]; mid: c2
    rng = random.Random(2)
    for C, lam, w in cases(rng, lambda C: C // 4 + 1, lambda C: C // 3):
        c3, c2 = C // 3, C // 2
        if 2 * w < C:
            want = c3 * (w >= lam) + (c2 - c3) * (w > C - 2 * lam)
        elif 2 * w > C:
            want = c2 + (C - c2 - c3) * (w >= 2 * lam) + c3 * (w > C - lam)
        else:
            want = c2
        assert O.f(O.RAD2, C, w, lam) == want, (C, lam, w)


def test_fs1_quotient_minus_divisible():
    # f = c floor(w (lam + 1) / c) - w [c | w (lam + 1)]
    rng = random.Random(3)
    for C, lam, w in cases(rng, lambda C: 1, lambda C: 100):
        n = w * (lam + 1)
        want = C * (n // C) - (w if n % C == 0 else 0)
        assert O.f(O.FS1, C, w, lam) == want, (C, lam, w)


def test_ccm1_doubled_quotients():
    # K = floor(c / lam); big 2K - 2 floor((c - w) / lam), mid K, small 2 floor(w / lam)
    rng = random.Random(4)
    for C, lam, w in cases(rng, lambda C: 1, lambda C: C // 2):
        K = C // lam
        if 2 * w > C:
            want = 2 * K - 2 * ((C - w) // lam)
        elif 2 * w < C:
            want = 2 * (w // lam)
        else:
            want = K
        assert O.f(O.CCM1, C, w, lam) == want, (C, lam, w)


def test_vb2_ceiling_terms():
    # h(a) = ceil(a lam / c) - 1; big 2 (lam - 1) - 2 h(c - w), mid lam - 1, small 2 h(w)
    rng = random.Random(5)
    for C, lam, w in cases(rng, lambda C: 2, lambda C: C):
        def h(a):
            return (a * lam + C - 1) // C - 1
        if 2 * w > C:
            want = 2 * (lam - 1) - 2 * h(C - w)
        elif 2 * w < C:
            want = 2 * h(w)
        else:
            want = lam - 1
        assert O.f(O.VB2, C, w, lam) == want, (C, lam, w)


def test_bj1_absolute_difference_form():
    # p = c mod lam, q = floor(w / lam): 2 f = (lam - 2p) q + |w - (q lam + p)| + w - p
    rng = random.Random(6)
    for C, lam, w in cases(rng, lambda C: 1, lambda C: C):
        p, q = C % lam, w // lam
        assert 2 * O.f(O.BJ1, C, w, lam) == (lam - 2 * p) * q + abs(w - (q * lam + p)) + w - p, (C, lam, w)


def test_bj1_clamp_above_half_capacity():
    # lam > c/2: floor(c / lam) = 1, p = c - lam, f = clamp(w - p, 0, 2 lam - c), and
    # 2 f = |w - p| - |w - lam| + 2 lam - c (the two-difference form of the tiles above c/2)
    rng = random.Random(7)
    for C, lam, w in cases(rng, lambda C: C // 2 + 1, lambda C: C):
        p = C - lam
        assert C % lam == p
        fv = O.f(O.BJ1, C, w, lam)
        assert fv == min(max(w - p, 0), 2 * lam - C), (C, lam, w)
        assert 2 * fv == abs(w - p) - abs(w - lam) + 2 * lam - C, (C, lam, w)
