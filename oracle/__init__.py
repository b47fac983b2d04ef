"""CPU oracle for the bin_packing feasibility check (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``bp_oracle.c`` (plain C,
exact int64, written from the paper's definitions) through ctypes and shares
no code with the HIP library in ``paper_2402_14821_amd``.

Paper: Tardivo, Michel, Pontelli, "Constraint Propagation on GPU: A Case Study
for the Bin Packing Constraint" (arXiv 2402.14821).  Each C function cites the
section, equation or algorithm it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bp_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

L1, L2, MT, RAD2, FS1, CCM1, VB2, BJ1 = range(8)
NB = 8
NAMES = ("L1", "L2", "MT", "RAD2", "FS1", "CCM1", "VB2", "BJ1")
DFFS = (MT, RAD2, FS1, CCM1, VB2, BJ1)

_lib = None
_I64 = ctypes.c_int64
_P64 = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = True) -> str:
    """Compile bp_oracle.c into liboracle.so with gcc (plain -O2)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_residual_reduce.argtypes = [_I64, _I64, _P64, _P64, _I64, _P64, _P64]
    lib.oracle_assignment_reduce.argtypes = [_I64, _I64, _P64, _P64, _I64, _P64, _P64, _P64]
    lib.oracle_l1.argtypes = [_I64, _P64, _I64]
    lib.oracle_l1.restype = _I64
    lib.oracle_l2_at.argtypes = [_I64, _P64, _I64, _I64]
    lib.oracle_l2_at.restype = _I64
    lib.oracle_l2_dense.argtypes = [_I64, _P64, _I64, _P64]
    lib.oracle_l2_dense.restype = _I64
    lib.oracle_f.argtypes = [ctypes.c_int, _I64, _I64, _I64]
    lib.oracle_f.restype = _I64
    lib.oracle_default_range.argtypes = [ctypes.c_int, _I64, _I64, _I64, ctypes.c_int, _P64, _P64]
    lib.oracle_dff_bound.argtypes = [ctypes.c_int, _I64, _P64, _I64, _I64, _I64, _P64]
    lib.oracle_dff_bound.restype = _I64
    lib.oracle_piecewise_bound.argtypes = [ctypes.c_int, _I64, _P64, _I64, _I64, _I64, _P64]
    lib.oracle_piecewise_bound.restype = _I64
    lib.oracle_bounds.argtypes = [_I64, _I64, _P64, _I64, _P64, _P64, ctypes.c_int,
                                  _P64, _P64, _P64, _P64, _P64]
    lib.oracle_dff_bound_strided.argtypes = [ctypes.c_int, _I64, _P64, _I64, _I64, _I64, _I64, _P64, _P64]
    lib.oracle_dff_bound_strided.restype = _I64
    lib.oracle_event_bound.argtypes = [ctypes.c_int, _I64, _P64, _I64, _I64, _I64, _P64]
    lib.oracle_event_bound.restype = _I64
    _lib = lib
    return lib


def _arr(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.int64).reshape(-1))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_P64)


class OracleError(ValueError):
    pass


def residual_reduce(C: int, residual, unpacked) -> np.ndarray:
    """Reduced items: unpacked sizes followed by one virtual item per non-empty bin."""
    lib = _load()
    res, unp = _arr(residual), _arr(unpacked)
    out = np.zeros(len(res) + len(unp) + 1, dtype=np.int64)
    r = ctypes.c_int64(0)
    st = lib.oracle_residual_reduce(C, len(res), _ptr(res), _ptr(unp), len(unp), _ptr(out), ctypes.byref(r))
    if st != 0:
        raise OracleError(f"oracle_residual_reduce status {st}")
    return out[: r.value].copy()


def assignment_reduce(C: int, m: int, size, bin_of):
    lib = _load()
    s, b = _arr(size), _arr(bin_of)
    out = np.zeros(len(s) + m + 1, dtype=np.int64)
    res = np.zeros(max(m, 1), dtype=np.int64)
    r = ctypes.c_int64(0)
    st = lib.oracle_assignment_reduce(C, m, _ptr(s), _ptr(b), len(s), _ptr(out), ctypes.byref(r), _ptr(res))
    if st != 0:
        raise OracleError(f"oracle_assignment_reduce status {st}")
    return out[: r.value].copy(), res[:m].copy()


def f(dff: int, C: int, w: int, lam: int) -> int:
    return int(_load().oracle_f(dff, C, w, lam))


def l1(C: int, items) -> int:
    a = _arr(items)
    return int(_load().oracle_l1(C, _ptr(a), len(a)))


def l2_at(C: int, items, lam: int) -> int:
    a = _arr(items)
    return int(_load().oracle_l2_at(C, _ptr(a), len(a), lam))


def l2_dense(C: int, items):
    a = _arr(items)
    arg = ctypes.c_int64(0)
    v = _load().oracle_l2_dense(C, _ptr(a), len(a), ctypes.byref(arg))
    return int(v), int(arg.value)


def default_range(bound: int, C: int, r: int = 0, maxw: int = 0, clamp_vb2: bool = False):
    lo, hi = ctypes.c_int64(0), ctypes.c_int64(0)
    _load().oracle_default_range(bound, C, r, maxw, int(clamp_vb2), ctypes.byref(lo), ctypes.byref(hi))
    return int(lo.value), int(hi.value)


def dff_bound(dff: int, C: int, items, lo: int | None = None, hi: int | None = None):
    a = _arr(items)
    if lo is None or hi is None:
        dlo, dhi = default_range(dff, C)
        lo = dlo if lo is None else lo
        hi = dhi if hi is None else hi
    arg = ctypes.c_int64(0)
    v = _load().oracle_dff_bound(dff, C, _ptr(a), len(a), lo, hi, ctypes.byref(arg))
    return int(v), int(arg.value)


def piecewise_bound(kind: int, C: int, items, lo: int | None = None, hi: int | None = None):
    a = _arr(items)
    dlo, dhi = default_range(kind, C)
    lo = dlo if lo is None else lo
    hi = dhi if hi is None else hi
    arg = ctypes.c_int64(0)
    v = _load().oracle_piecewise_bound(kind, C, _ptr(a), len(a), lo, hi, ctypes.byref(arg))
    if v < 0:
        raise OracleError("allocation failure")
    return int(v), int(arg.value)


def event_bound(dff: int, C: int, items, lo: int | None = None, hi: int | None = None):
    """CCM1 or BJ1 by the event sweep (any capacity): (value, smallest argmax)."""
    a = _arr(items)
    dlo, dhi = default_range(dff, C)
    lo = dlo if lo is None else lo
    hi = dhi if hi is None else hi
    arg = ctypes.c_int64(0)
    v = _load().oracle_event_bound(dff, C, _ptr(a), len(a), lo, hi, ctypes.byref(arg))
    if v < 0:
        raise OracleError("bad argument or allocation failure")
    return int(v), int(arg.value)


def bounds_by_pieces(C: int, k: int, items, threads: int | None = None) -> dict:
    """Every bound over the default ranges without visiting every parameter,
    except VB2 (left out, value and argmax -1): L2, MT and RAD2 at their piece
    starts, CCM1 and BJ1 by the event sweep, FS1 (100 parameters) directly.
    For capacities where the dense loops are out of reach; lb and the verdict
    are over the bounds computed."""
    a = _arr(items)
    jobs = {L2: lambda: piecewise_bound(L2, C, a), MT: lambda: piecewise_bound(MT, C, a),
            RAD2: lambda: piecewise_bound(RAD2, C, a), FS1: lambda: dff_bound(FS1, C, a),
            CCM1: lambda: event_bound(CCM1, C, a), BJ1: lambda: event_bound(BJ1, C, a)}
    with ThreadPoolExecutor(max_workers=threads or len(jobs)) as ex:
        futs = {b: ex.submit(fn) for b, fn in jobs.items()}
        res = {b: f.result() for b, f in futs.items()}
    val = np.full(NB, -1, dtype=np.int64)
    arg = np.full(NB, -1, dtype=np.int64)
    val[L1] = l1(C, a)
    for b, (v, g) in res.items():
        val[b], arg[b] = v, g
    lb = int(val.max())
    lb_arg = int(np.argmax(val))
    return {"value": val, "argmax": arg, "lb": lb, "lb_arg": lb_arg, "verdict": int(lb <= k), "r": len(a)}


def bounds(C: int, k: int, items, lo=None, hi=None, l2_dense: bool = False) -> dict:
    """Every bound of the collection, lb, lb_arg and verdict (1 = PASS)."""
    lib = _load()
    a = _arr(items)
    val = np.zeros(NB, dtype=np.int64)
    arg = np.zeros(NB, dtype=np.int64)
    lb, lba, ver = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    if lo is not None and hi is not None:
        lo_a, hi_a = _arr(lo), _arr(hi)
        plo, phi = _ptr(lo_a), _ptr(hi_a)
    else:
        plo = phi = None
    st = lib.oracle_bounds(C, k, _ptr(a), len(a), plo, phi, int(l2_dense), _ptr(val), _ptr(arg),
                           ctypes.byref(lb), ctypes.byref(lba), ctypes.byref(ver))
    if st != 0:
        raise OracleError(f"oracle_bounds status {st}")
    return {"value": val, "argmax": arg, "lb": int(lb.value), "lb_arg": int(lba.value),
            "verdict": int(ver.value), "r": len(a)}


def bounds_many(instances, threads: int | None = None, l2_dense: bool = False):
    """bounds() over a list of (C, k, items[, lo, hi]) on a thread pool (ctypes drops the GIL)."""
    _load()
    threads = threads or min(16, os.cpu_count() or 1)

    def one(inst):
        if len(inst) == 5:
            C, k, items, lo, hi = inst
            return bounds(C, k, items, lo, hi, l2_dense=l2_dense)
        C, k, items = inst
        return bounds(C, k, items, l2_dense=l2_dense)

    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(one, instances))


def dff_bound_strided(dff: int, C: int, items, lo: int, hi: int, step: int):
    a = _arr(items)
    arg, ev = ctypes.c_int64(0), ctypes.c_int64(0)
    v = _load().oracle_dff_bound_strided(dff, C, _ptr(a), len(a), lo, hi, step, ctypes.byref(arg), ctypes.byref(ev))
    return int(v), int(arg.value), int(ev.value)
