"""CPU pins of the segment forms the GPU's BP_SEGMENTS tiles compute.

The kernels evaluate the BJ1 sum as a telescoping sum of threshold sums and
the MT sum as class prefixes of the sorted sizes.  These identities are
checked here against the oracle's f (the printed DFFs of Sec. 3.1), summed
item by item, on random instances at every parameter -- a mistake in the
identity (a dropped term, an off-by-one threshold) fails here, on the CPU.
"""
import random

import oracle as O


def U(items, t):
    return sum(max(0, w - t) for w in items)


def bj1_segments(C, items, lam):
    # sizes 0 < w < c; K = floor(c / lambda)
    nz = [w for w in items if 0 < w < C]
    K = C // lam
    return sum(U(nz, C - m * lam) for m in range(1, K + 1)) - sum(U(nz, j * lam) for j in range(1, K + 1))


def mt_segments(C, items, lam):
    # small sizes with w >= lambda, big ones with c - w < lambda (their part of the MT sum)
    small = sorted((w for w in items if 0 < 2 * w < C), reverse=True)
    big = sorted((w for w in items if C < 2 * w < 2 * C), reverse=True)
    n_small = sum(1 for w in small if w >= lam)   # a prefix of the decreasing small sizes
    n_big = sum(1 for w in big if w >= C - lam + 1)  # a prefix of the decreasing big sizes
    return sum(small[:n_small]) + sum(C - w for w in big[:n_big])


def test_bj1_telescoping_form():
    rng = random.Random(7)
    for _ in range(400):
        C = rng.randint(1, 120)
        items = [rng.randint(0, C) for _ in range(rng.randint(0, 10))]
        for lam in range(1, C + 1):
            direct = sum(O.f(O.BJ1, C, w, lam) for w in items if 0 < w < C)
            assert bj1_segments(C, items, lam) == direct, (C, items, lam)


def test_mt_class_prefixes():
    rng = random.Random(8)
    for _ in range(400):
        C = rng.randint(1, 120)
        items = [rng.randint(0, C) for _ in range(rng.randint(0, 10))]
        big_full = sum(w for w in items if C < 2 * w < 2 * C)
        mid = sum(1 for w in items if 2 * w == C)
        for lam in range(0, C // 2 + 1):
            direct = sum(O.f(O.MT, C, w, lam) for w in items if 0 < w < C)
            # f_MT = c for big sizes above c - lambda, w otherwise in the big class; the constant part is
            # sum of the big sizes plus c/2 per mid size
            assert big_full + mid * (C // 2) + mt_segments(C, items, lam) == direct, (C, items, lam)


def test_ccm1_threshold_counts():
    # sum_small floor(w / lambda) = sum_q #{small w >= q lambda}; for the big
    # sizes floor((c - w) / lambda) = sum_q #{big w <= c - q lambda}
    rng = random.Random(9)
    for _ in range(300):
        C = rng.randint(2, 120)
        items = [rng.randint(0, C) for _ in range(rng.randint(0, 10))]
        small = [w for w in items if 0 < 2 * w < C]
        big = [w for w in items if C < 2 * w < 2 * C]
        mid = sum(1 for w in items if 2 * w == C)
        for lam in range(1, C // 2 + 1):
            qmax = (C // 2) // lam
            hs = sum(sum(1 for w in small if w >= q * lam) for q in range(1, qmax + 1))
            hb = sum(sum(1 for w in big if w <= C - q * lam) for q in range(1, qmax + 1))
            K = C // lam
            total = 2 * K * len(big) + K * mid + 2 * (hs - hb)
            direct = sum(O.f(O.CCM1, C, w, lam) for w in items if 0 < w < C)
            assert total == direct, (C, items, lam)


def test_vb2_mirror_identity():
    # with h(a, lambda) = ceil(a lambda / c) - 1 for a >= 1:
    #   h(a, c - lambda) = a - 1 - h(a, lambda) - [d | a],  d = c / gcd(c, lambda)
    # checked through the oracle's f_VB2 (small sizes: f = 2 h(w); big sizes:
    # f = 2 (lambda - 1) - 2 h(c - w))
    import math

    rng = random.Random(10)
    for _ in range(300):
        C = rng.randint(5, 150)
        items = [rng.randint(1, C - 1) for _ in range(rng.randint(1, 10))]
        small = [w for w in items if 2 * w < C]
        big = [w for w in items if 2 * w > C]
        for lam in range(2, (C - 1) // 2 + 1):
            d = C // math.gcd(C, lam)
            hs = sum(O.f(O.VB2, C, w, lam) for w in small) // 2
            hb = sum(2 * (lam - 1) - O.f(O.VB2, C, w, lam) for w in big) // 2
            hs2 = sum(w - 1 for w in small) - hs - sum(1 for w in small if w % d == 0)
            hb2 = sum(C - w - 1 for w in big) - hb - sum(1 for w in big if w % d == 0)
            lam2 = C - lam
            assert 2 * hs2 == sum(O.f(O.VB2, C, w, lam2) for w in small), (C, items, lam)
            assert 2 * hb2 == sum(2 * (lam2 - 1) - O.f(O.VB2, C, w, lam2) for w in big), (C, items, lam)
