"""Seeded synthetic inputs for the bin_packing feasibility check.

Shared by the tests, the bench and the oracle's callers; holds none of the
check's arithmetic (no reduction, no bound).  Shapes follow the workloads of
the paper's experiments (Sec. 5: uniform sizes of the Falkenauer 'U' and
Scholl classes, triplet instances of the Falkenauer 'T' class, capacities up
to 10^5 and beyond) at the sizes given by the build's configurations.  No
benchmark file of the paper is used or reproduced.

Every generator returns plain numpy int32 arrays:
  residual form  (C, m, residual[m], unpacked[n])   -- a partial packing
  items form     (C, k, items[r])                   -- an already reduced instance
"""
from __future__ import annotations

import bisect
from dataclasses import dataclass

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ---- configuration 1: small partial packing --------------------------------

def small_partial_packing(seed: int, n: int = 50, m: int = 20, C: int = 150, lo: int = 20, hi: int = 100,
                          frac_packed: float = 0.3):
    """n sizes U[lo, hi]; a seeded 30% of them placed into uniformly random bins
    where they fit (an item that fits nowhere tried stays unpacked)."""
    g = _rng(seed)
    sizes = g.integers(lo, hi + 1, size=n).astype(np.int64)
    k_pack = int(round(frac_packed * n))
    packed_idx = g.choice(n, size=k_pack, replace=False)
    load = np.zeros(m, dtype=np.int64)
    placed = np.zeros(n, dtype=bool)
    for i in packed_idx:
        order = g.permutation(m)
        for j in order:
            if load[j] + sizes[i] <= C:
                load[j] += sizes[i]
                placed[i] = True
                break
    residual = (C - load).astype(np.int32)
    unpacked = sizes[~placed].astype(np.int32)
    return C, m, residual, unpacked


# ---- configuration 2: one large residual instance ----------------------------

def large_residual(seed: int = 1, n: int = 10_000, m: int = 4_000, C: int = 100_000):
    """n sizes U[C/10, C/2], m bins with remaining capacity U[C/2, C]."""
    g = _rng(seed)
    unpacked = g.integers(C // 10, C // 2 + 1, size=n).astype(np.int32)
    residual = g.integers(C // 2, C + 1, size=m).astype(np.int32)
    return C, m, residual, unpacked


# ---- configuration 3: uneven batch ---------------------------------------------

def best_fit_decreasing_bins(C: int, sizes) -> int:
    """Bins used by best-fit decreasing: a feasible packing, so an upper bound."""
    res = []  # sorted remaining capacities
    for w in sorted((int(x) for x in sizes), reverse=True):
        if w == 0:
            continue
        j = bisect.bisect_left(res, w)
        if j < len(res):
            r = res.pop(j) - w
        else:
            r = C - w
        bisect.insort(res, r)
    return len(res)


@dataclass
class Batch:
    C: np.ndarray      # int32 [count]
    k: np.ndarray      # int32 [count]
    off: np.ndarray    # int64 [count + 1]
    items: np.ndarray  # int32 [off[-1]]
    expect_fail: np.ndarray  # bool [count], True when built to fail (None if unknown)

    def instance(self, i: int):
        return int(self.C[i]), int(self.k[i]), self.items[self.off[i]:self.off[i + 1]]

    def __len__(self):
        return len(self.C)

    def subset(self, idx):
        idx = list(idx)
        parts = [self.items[self.off[i]:self.off[i + 1]] for i in idx]
        off = np.zeros(len(idx) + 1, dtype=np.int64)
        off[1:] = np.cumsum([len(p) for p in parts])
        return Batch(self.C[idx].copy(), self.k[idx].copy(), off,
                     np.concatenate(parts) if parts else np.zeros(0, np.int32), self.expect_fail[idx].copy())


def uneven_batch(seed: int = 2, count: int = 4096, median: float = 400.0, sigma: float = 1.0, nmin: int = 50,
                 nmax: int = 5000, capacities=(1_000, 10_000, 1_000_000), frac_fail: float = 0.4) -> Batch:
    """Lognormal item counts (median 400, clipped to [50, 5000]); C drawn per
    instance from `capacities`; sizes U[1, C].  A seeded 40% get
    k = ceil(total / C) - 1 bins, fewer than the total size can fill (built to
    FAIL); the rest get the best-fit-decreasing bin count (built to PASS)."""
    g = _rng(seed)
    ns = np.clip(np.rint(median * np.exp(g.normal(0.0, sigma, size=count))), nmin, nmax).astype(np.int64)
    Cs = np.asarray(capacities, dtype=np.int64)[g.integers(0, len(capacities), size=count)]
    fail = g.random(count) < frac_fail
    off = np.zeros(count + 1, dtype=np.int64)
    off[1:] = np.cumsum(ns)
    items = np.empty(off[-1], dtype=np.int32)
    ks = np.empty(count, dtype=np.int32)
    for i in range(count):
        w = g.integers(1, Cs[i] + 1, size=ns[i])
        items[off[i]:off[i + 1]] = w
        if fail[i]:
            ks[i] = -(-int(w.sum()) // int(Cs[i])) - 1
        else:
            ks[i] = best_fit_decreasing_bins(int(Cs[i]), w)
    return Batch(Cs.astype(np.int32), ks, off, items, fail)


# ---- configuration 5: triplet-tight batch ---------------------------------------

def triplet_batch(seed: int = 5, count: int = 1024, mlo: int = 300, mhi: int = 1000, clo: int = 1_000_000,
                  chi: int = 2**31 - 1) -> Batch:
    """Every bin holds three sizes in (C/4, C/2) summing exactly to C (drawn by
    rejection); n = 3m items shuffled; C ~ U[clo, chi].  A seeded half gets
    m - 1 bins (must FAIL: the sizes fill m bins exactly)."""
    g = _rng(seed)
    parts, Cs, ks, fail = [], [], [], []
    for _ in range(count):
        m = int(g.integers(mlo, mhi + 1))
        C = int(g.integers(clo, chi + 1))
        lo, hi = C // 4 + 1, (C - 1) // 2  # strictly inside (C/4, C/2)
        trip = np.empty((m, 3), dtype=np.int64)
        filled = 0
        while filled < m:
            a = g.integers(lo, hi + 1, size=2 * (m - filled))
            b = g.integers(lo, hi + 1, size=2 * (m - filled))
            c = C - a - b
            ok = (c >= lo) & (c <= hi)
            take = np.flatnonzero(ok)[: m - filled]
            trip[filled:filled + len(take), 0] = a[take]
            trip[filled:filled + len(take), 1] = b[take]
            trip[filled:filled + len(take), 2] = c[take]
            filled += len(take)
        w = trip.reshape(-1)
        g.shuffle(w)
        parts.append(w.astype(np.int32))
        Cs.append(C)
        drop = bool(g.random() < 0.5)
        ks.append(m - 1 if drop else m)
        fail.append(drop)
    off = np.zeros(count + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(p) for p in parts])
    return Batch(np.array(Cs, np.int32), np.array(ks, np.int32), off, np.concatenate(parts), np.array(fail))


def windows(lo: int, hi: int, width: int):
    """The low and high windows [lo, lo+width-1] and [hi-width+1, hi] of a range,
    or the whole range when it is not longer than 2*width."""
    if hi - lo + 1 <= 2 * width:
        return [(lo, hi)]
    return [(lo, lo + width - 1), (hi - width + 1, hi)]


# ---- Weibull instances for the search (Sec. 5) -----------------------------------

def weibull_instance(seed: int, n: int = 100, shape: float = 1.0, sigma: float = 1.4, scale: float = 1000.0):
    """n sizes from a Weibull distribution of the given shape and scale
    (rounded, at least 1) and capacity c = sigma * max size (rounded), as the
    paper's Weibull instances (Sec. 5: n in {100, 200}, shape 0.5 .. 5.0,
    scale 1000, sigma in {1.0, 1.2, .., 2.0}).  Returns (C, sizes)."""
    g = _rng(seed)
    w = np.maximum(1, np.rint(scale * g.weibull(shape, size=n))).astype(np.int64)
    C = int(round(sigma * int(w.max())))
    return C, w.astype(np.int32)


# ---- configuration 4: requests of a simulated depth-first search ---------------

@dataclass
class Request:
    t: float             # arrival time (s)
    C: int
    residual: np.ndarray
    unpacked: np.ndarray
    node: int
    parent: int = -1     # index of the request of the node this one was reached from (-1: a root)
    commits: tuple = ()  # (size, bin) pairs committed since that request


def dfs_requests(seed: int, rate: float, duration: float, C: int = 10_000, nlo: int = 200, nhi: int = 5000,
                 wlo: int | None = None, whi: int | None = None, p_back: float = 0.3, restart_every: int = 64,
                 max_requests: int | None = None, instances: str = "all"):
    """Open-loop request stream of a simulated depth-first search.

    Poisson arrivals at `rate` per second for `duration` seconds.  A root has
    n ~ U[nlo, nhi] sizes U[C/20, C/2] and as many empty bins as best fit
    decreasing needs.  A child commits the 1-3 largest unpacked items, each to
    the bin with the least remaining capacity that holds it (decreasing best
    fit); with probability p_back the search backtracks 1-3 levels instead.
    Every `restart_every` nodes a new root starts.  Each node is one request
    (residual form); a request also names the request of the node it was
    reached from (`parent`, -1 for a root) and the (size, bin) commits since
    that node (none when the search returned to a node it had checked).
    instances="roots" keeps residual and unpacked of the roots only (None for
    the others), for long streams."""
    g = _rng(seed)
    wlo = C // 20 if wlo is None else wlo
    whi = C // 2 if whi is None else whi
    t = 0.0
    out = []
    stack = []  # (residual, unpacked, index of the node's latest request)
    node = 0
    since_root = restart_every
    while True:
        t += g.exponential(1.0 / rate)
        if t > duration or (max_requests is not None and len(out) >= max_requests):
            break
        parent, commits = -1, ()
        if since_root >= restart_every or not stack:
            n0 = int(g.integers(nlo, nhi + 1))
            sizes = np.sort(g.integers(wlo, whi + 1, size=n0))[::-1].astype(np.int32)
            m = best_fit_decreasing_bins(C, sizes)
            stack = [(np.full(m, C, dtype=np.int32), sizes, -1)]
            since_root = 0
        elif g.random() < p_back and len(stack) > 1:
            for _ in range(int(g.integers(1, 4))):
                if len(stack) > 1:
                    stack.pop()
            parent = stack[-1][2]
        else:
            res, unp, idx = stack[-1]
            parent = idx
            res = res.copy()
            k = min(int(g.integers(1, 4)), len(unp))
            ok = True
            placed = []
            for i in range(k):
                w = int(unp[i])
                fits = np.flatnonzero(res >= w)
                if len(fits) == 0:
                    ok = False
                    break
                j = fits[np.argmin(res[fits])]
                res[j] -= w
                placed.append((w, int(j)))
            if ok and k > 0:
                stack.append((res, unp[k:].copy(), idx))
                commits = tuple(placed)
        res, unp, _ = stack[-1]
        if instances == "all" or parent < 0:
            out.append(Request(t, C, res.copy(), unp.copy(), node, parent, commits))
        else:
            out.append(Request(t, C, None, None, node, parent, commits))
        stack[-1] = (res, unp, len(out) - 1)
        node += 1
        since_root += 1
    return out
