"""Full oracle records of large instances on a thread pool (test infrastructure).

Every bound of the collection is a maximum over a parameter range (Sec. 3.1,
Alg. 2).  These helpers cut each range into consecutive chunks, ask the
oracle for the maximum and its smallest maximiser on every chunk (the ctypes
calls release the GIL, so chunks run in parallel), and keep the largest
value, the earliest chunk winning ties.  That is the same maximum and the
same smallest maximiser as one pass over the whole range.  No bound
arithmetic is done here: every value comes from the oracle.
"""
from __future__ import annotations

import functools
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle as O


def pool_threads() -> int:
    # the GPU machine gives one process a share of 16 cores
    return max(1, min(16, os.cpu_count() or 1))


def _chunks(lo: int, hi: int, size: int):
    out = []
    a = lo
    while a <= hi:
        b = min(hi, a + size - 1)
        out.append((a, b))
        a = b + 1
    return out


def dense_record(C: int, k: int, items, lo=None, hi=None, threads: int | None = None, chunk: int | None = None) -> dict:
    """The oracle's record with L2 visited at every parameter (its dense
    definition) and every DFF swept densely, ranges split over a pool."""
    items = np.ascontiguousarray(np.asarray(items, dtype=np.int64))
    threads = threads or pool_threads()
    rlo, rhi = [], []
    for b in range(O.NB):
        if lo is not None and hi is not None:
            rlo.append(int(lo[b]))
            rhi.append(int(hi[b]))
        else:
            a, z = O.default_range(b, C)
            rlo.append(a)
            rhi.append(z)
    total = sum(max(0, rhi[b] - rlo[b] + 1) for b in range(O.L2, O.NB))
    size = chunk or max(1, total // (threads * 8))
    jobs = []
    for b in range(O.L2, O.NB):
        for a, z in _chunks(rlo[b], rhi[b], size):
            jobs.append((b, a, z))
    empty_lo = [1] * O.NB
    empty_hi = [0] * O.NB

    def run(job):
        b, a, z = job
        if b == O.L2:
            lo2, hi2 = list(empty_lo), list(empty_hi)
            lo2[O.L2], hi2[O.L2] = a, z
            rec = O.bounds(C, k, items, lo2, hi2, l2_dense=True)
            return int(rec["value"][O.L2]), int(rec["argmax"][O.L2])
        return O.dff_bound(b, C, items, a, z)

    with ThreadPoolExecutor(max_workers=threads) as ex:
        parts = list(ex.map(run, jobs))
    value = np.zeros(O.NB, dtype=np.int64)
    argmax = np.full(O.NB, -1, dtype=np.int64)
    value[O.L1] = O.l1(C, items)
    seen = [False] * O.NB
    for (b, _, _), (v, arg) in zip(jobs, parts):  # jobs are in increasing parameter order per bound
        if not seen[b] or v > value[b]:
            value[b], argmax[b] = v, arg
            seen[b] = True
    lb = int(value.max())
    lb_arg = int(np.flatnonzero(value == lb)[0])
    return {"value": value, "argmax": argmax, "lb": lb, "lb_arg": lb_arg, "verdict": int(lb <= k), "r": len(items)}


@functools.lru_cache(maxsize=4)
def large_residual_record(seed: int = 1):
    """(C, m, residual, unpacked, items, record) of the single large residual
    instance (n = 10 000, m = 4 000, C = 100 000), the record dense."""
    from paper_2402_14821_amd import workloads as W

    C, m, res, unp = W.large_residual(seed)
    items = O.residual_reduce(C, res, unp)
    return C, m, res, unp, items, dense_record(C, m, items)
