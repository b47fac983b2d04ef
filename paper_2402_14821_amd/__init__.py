"""Python binding of libbp, the gfx950 feasibility check of the bin_packing constraint.

Argument marshalling only: every step of the check runs in the HIP kernels
of ``libbp.so``.  The entry points keep the C names of ``include/bp.h``
(``bp_lower_bounds``, ``bp_feasible``, ...); the ``Context`` class adds
numpy / torch conveniences around them.  There is no fallback: importing a
function when ``libbp.so`` is missing raises ``BpLibraryMissing``.

Method: Tardivo, Michel, Pontelli, "Constraint Propagation on GPU: A Case
Study for the Bin Packing Constraint" (arXiv 2402.14821), Sec. 3-4.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbp.so")

BP_OK, BP_ERR_ARG, BP_ERR_RANGE, BP_ERR_NOMEM, BP_ERR_DEVICE, BP_ERR_AGAIN, BP_ERR_STATE, BP_ERR_LIMIT = (
    0, -1, -2, -3, -4, -5, -6, -7)
BP_L1, BP_L2, BP_MT, BP_RAD2, BP_FS1, BP_CCM1, BP_VB2, BP_BJ1 = range(8)
BP_NB = 8
BOUND_NAMES = ("L1", "L2", "MT", "RAD2", "FS1", "CCM1", "VB2", "BJ1")
BP_SWEEP_PAPER_VB2_CLAMP = 1
BP_SWEEP_SEGMENTS = 2
BP_NO_EARLY_EXIT = 1
BP_SEGMENTS = 2
BP_MAX_ITEMS = 1 << 20
BP_MAX_REDUCE_ITEMS = 1 << 30
BP_NOALLOC_MAX_ITEMS = 1 << 14
BP_NOALLOC_SCRATCH_BYTES = 32 << 20
BP_MAX_BATCH = 1 << 20
BP_MAX_COMMIT = 1024
BP_QUEUE_HISTORY = 65536

_i32, _i64, _u32, _u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
_P32, _P64 = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)


class bp_sweep(ctypes.Structure):
    _fields_ = [("lo", _i64 * BP_NB), ("hi", _i64 * BP_NB), ("flags", _u32), ("reserved", _u32)]


class bp_bounds(ctypes.Structure):
    _fields_ = [("value", _i64 * BP_NB), ("argmax_lambda", _i64 * BP_NB), ("lb", _i64), ("lb_arg", _i32),
                ("verdict", _i32), ("k", _i64), ("r", _i64), ("evals", _i64), ("status", _i32),
                ("early_exit", _i32), ("evals_done", _i64)]


class bp_batch(ctypes.Structure):
    _fields_ = [("count", _i32), ("reserved", _i32), ("off", _P64), ("items", _P32), ("C", _P32), ("k", _P32)]


class bp_commit(ctypes.Structure):
    _fields_ = [("size", _i32), ("bin", _i32)]


class bp_request(ctypes.Structure):
    _fields_ = [("C", _i32), ("m", _i32), ("n", _i64), ("residual", _P32), ("unpacked", _P32), ("tag", _u64),
                ("flags", _u32), ("reserved", _u32), ("parent", _u64), ("commits", ctypes.POINTER(bp_commit)),
                ("ncommit", _i32), ("reserved2", _i32)]


class bp_result(ctypes.Structure):
    _fields_ = [("ticket", _u64), ("tag", _u64), ("status", _i32), ("verdict", _i32), ("lb", _i64),
                ("submit_us", ctypes.c_double), ("start_us", ctypes.c_double), ("done_us", ctypes.c_double),
                ("bounds", bp_bounds), ("from_parent", _i32), ("reserved", _i32)]


class bp_tuning(ctypes.Structure):
    _fields_ = [("lanes_params", _i32), ("waves_per_cu", _i32), ("tasks_per_wave", _i32), ("min_chunk", _i32)]


BP_SOLVE_DFFS, BP_SOLVE_L2, BP_SOLVE_NO_CHECK = 0, 1, 2
BP_SOLVE_LIMIT, BP_SOLVE_OPTIMAL = 0, 1
BP_SOLVE_OFF_KNAPSACK, BP_SOLVE_OFF_FILL, BP_SOLVE_OFF_SINGLE, BP_SOLVE_OFF_SYMMETRY = 1, 2, 4, 8
bp_check_fn = ctypes.CFUNCTYPE(ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, _P32, _P32,
                               ctypes.c_int64, ctypes.POINTER(ctypes.c_int64))


class bp_solve_opts(ctypes.Structure):
    _fields_ = [("mode", _i32), ("check_flags", _u32), ("max_nodes", _i64), ("time_limit_s", ctypes.c_double),
                ("check", bp_check_fn), ("user", ctypes.c_void_p), ("disable", _u32), ("reserved", _i32)]


class bp_solve_result(ctypes.Structure):
    _fields_ = [("status", _i32), ("bins", _i32), ("lower", _i32), ("upper", _i32), ("attempts", _i32),
                ("limit_reached", _i32), ("nodes", _i64), ("fails", _i64), ("checks", _i64),
                ("check_fails", _i64), ("seconds", ctypes.c_double), ("check_seconds", ctypes.c_double),
                ("filter_fails", _i64)]


class bp_queue_stats(ctypes.Structure):
    _fields_ = [("submitted", _u64), ("completed", _u64), ("rejected", _u64), ("batches", _u64),
                ("in_flight", _u64), ("bytes_in_use", _u64), ("bytes_peak", _u64), ("budget", _u64),
                ("busy_us", ctypes.c_double), ("from_parent", _u64), ("full_sweeps", _u64), ("nodes_kept", _u64),
                ("node_evictions", _u64), ("node_bytes", _u64)]


BOUNDS_DTYPE = np.dtype([("value", np.int64, BP_NB), ("argmax_lambda", np.int64, BP_NB), ("lb", np.int64),
                         ("lb_arg", np.int32), ("verdict", np.int32), ("k", np.int64), ("r", np.int64),
                         ("evals", np.int64), ("status", np.int32), ("early_exit", np.int32),
                         ("evals_done", np.int64)])
assert BOUNDS_DTYPE.itemsize == ctypes.sizeof(bp_bounds)


class BpLibraryMissing(RuntimeError):
    pass


class BpError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"bp status {status}: {msg}")
        self.status = status


_VP = ctypes.c_void_p
_SIGNATURES = {
    "bp_version": ([], ctypes.c_char_p),
    "bp_last_error": ([], ctypes.c_char_p),
    "bp_default_sweep": ([_i32, _i64, _i32, _u32, ctypes.POINTER(bp_sweep)], _i32),
    "bp_ctx_create": ([ctypes.c_int, ctypes.POINTER(_VP)], _i32),
    "bp_ctx_destroy": ([_VP], _i32),
    "bp_residual_reduce": ([_VP, _i32, _i32, _P32, _P32, _i64, _P32, _P64], _i32),
    "bp_assignment_reduce": ([_VP, _i32, _i32, _P32, _P32, _i64, _P32, _P64, _P32], _i32),
    "bp_lower_bounds": ([_VP, _i32, _i32, _P32, _i64, ctypes.POINTER(bp_sweep), ctypes.POINTER(bp_bounds)], _i32),
    "bp_lower_bounds_dev": ([_VP, _i32, _i32, _VP, _i64, ctypes.POINTER(bp_sweep), _VP, _VP], _i32),
    "bp_feasible": ([_VP, _i32, _i32, _P32, _P32, _i64, _u32, _P32, _P64, ctypes.POINTER(bp_bounds)], _i32),
    "bp_feasible_dev": ([_VP, _i32, _i32, _VP, _VP, _i64, _u32, _VP, _VP], _i32),
    "bp_feasible_dev_noalloc": ([_i32, _i32, _VP, _VP, _i64, _u32, _VP, _VP], _i32),
    "bp_ctx_set_timing": ([_VP, _i32], _i32),
    "bp_ctx_get_tuning": ([_VP, ctypes.POINTER(bp_tuning)], _i32),
    "bp_ctx_set_tuning": ([_VP, ctypes.POINTER(bp_tuning)], _i32),
    "bp_autotune_batch": ([_VP, ctypes.POINTER(bp_batch), ctypes.POINTER(bp_sweep), _i32,
                           ctypes.POINTER(bp_tuning), ctypes.POINTER(ctypes.c_double)], _i32),
    "bp_autotune_batch_cached": ([_VP, ctypes.POINTER(bp_batch), ctypes.POINTER(bp_sweep), _i32, ctypes.c_char_p,
                                  ctypes.POINTER(bp_tuning), ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_int32)], _i32),
    "bp_ctx_set_order": ([_VP, _P32], _i32),
    "bp_ctx_stage_times": ([_VP, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)], _i32),
    "bp_lower_bounds_batch": ([_VP, ctypes.POINTER(bp_batch), ctypes.POINTER(bp_sweep), _VP], _i32),
    "bp_lower_bounds_batch_dev": ([_VP, ctypes.POINTER(bp_batch), _VP, ctypes.POINTER(bp_sweep), _VP, _VP], _i32),
    "bp_feasible_batch": ([_VP, ctypes.POINTER(bp_batch), _u32, _P32, _P64, _VP], _i32),
    "bp_queue_create": ([_VP, ctypes.c_size_t, _i32, ctypes.POINTER(_VP)], _i32),
    "bp_queue_submit": ([_VP, ctypes.POINTER(bp_request), _i32, ctypes.POINTER(_u64)], _i32),
    "bp_queue_poll": ([_VP, _VP, _i32, _P32, _i32], _i32),
    "bp_queue_stats_get": ([_VP, ctypes.POINTER(bp_queue_stats)], _i32),
    "bp_queue_replay": ([_VP, _VP, _VP, _VP, _i64, _VP, _VP, ctypes.POINTER(ctypes.c_double)], _i32),
    "bp_queue_destroy": ([_VP], _i32),
    "bp_selftest_division": ([_u32, _u32, _u32, _u32], _i64),
    "bp_solve": ([_VP, _i32, _i64, _P32, ctypes.POINTER(bp_solve_opts), _P32, ctypes.POINTER(bp_solve_result)], _i32),
    "bp_subset_sum_gap": ([_P32, _i32, _i64, _i64, ctypes.POINTER(_i64), ctypes.POINTER(_i64)], _i32),
}

_lib = None


def _preload_torch_hip_runtime():
    """Keep one HIP runtime per process.

    PyTorch-ROCm ships its own libamdhip64 with the same soname as the
    system one.  If libbp loaded the system copy first, torch would later load
    its own and see no GPU.  Loading torch's copy first (by path, without
    importing torch) makes libbp and torch share it.
    """
    import importlib.util

    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.submodule_search_locations:
        return
    cand = os.path.join(list(spec.submodule_search_locations)[0], "lib", "libamdhip64.so")
    if os.path.exists(cand):
        ctypes.CDLL(cand, mode=ctypes.RTLD_GLOBAL)


def load(path: str | None = None):
    """Load libbp.so (built in-tree by ``paper_2402_14821_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    _preload_torch_hip_runtime()
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise BpLibraryMissing(f"{p} is not built; run `python -m paper_2402_14821_amd.build`")
    lib = ctypes.CDLL(p)
    for name, (args, res) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def exported_symbols():
    return list(_SIGNATURES)


def _check(st: int):
    if st != BP_OK:
        raise BpError(st, load().bp_last_error().decode(errors="replace"))


def _i32arr(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.int32).reshape(-1))


def _p32(a: np.ndarray):
    return a.ctypes.data_as(_P32)


def bounds_to_dict(b) -> dict:
    if isinstance(b, bp_bounds):
        return {"value": np.array(b.value[:], dtype=np.int64), "argmax": np.array(b.argmax_lambda[:], dtype=np.int64),
                "lb": int(b.lb), "lb_arg": int(b.lb_arg), "verdict": int(b.verdict), "k": int(b.k), "r": int(b.r),
                "evals": int(b.evals), "status": int(b.status), "early_exit": int(b.early_exit),
                "evals_done": int(b.evals_done)}
    return {"value": np.array(b["value"], dtype=np.int64), "argmax": np.array(b["argmax_lambda"], dtype=np.int64),
            "lb": int(b["lb"]), "lb_arg": int(b["lb_arg"]), "verdict": int(b["verdict"]), "k": int(b["k"]),
            "r": int(b["r"]), "evals": int(b["evals"]), "status": int(b["status"]),
            "early_exit": int(b["early_exit"]), "evals_done": int(b["evals_done"])}


def default_sweep(C: int, r: int = 0, max_w: int = 0, flags: int = 0) -> bp_sweep:
    sw = bp_sweep()
    _check(load().bp_default_sweep(C, r, max_w, flags, ctypes.byref(sw)))
    return sw


def make_sweep(lo, hi, flags: int = 0) -> bp_sweep:
    sw = bp_sweep()
    for b in range(BP_NB):
        sw.lo[b] = int(lo[b])
        sw.hi[b] = int(hi[b])
    sw.flags = flags
    return sw


def feasible_dev_noalloc(C: int, m: int, d_residual_ptr: int, n: int, d_unpacked_ptr: int, d_out_ptr: int,
                         stream_ptr: int, flags: int = 0):
    """bp_feasible_dev_noalloc on the current HIP device (no context)."""
    _check(load().bp_feasible_dev_noalloc(C, m, _VP(d_residual_ptr), _VP(d_unpacked_ptr), n, flags,
                                          _VP(d_out_ptr), _VP(stream_ptr)))


def solve(C: int, sizes, ctx: "Context | None" = None, mode: int = BP_SOLVE_DFFS, check_flags: int = 0,
          max_nodes: int = 0, time_limit_s: float = 0.0, check=None, disable: int = 0):
    """bp_solve: (result dict, bin_of).  check(C, residual, unpacked) -> lb
    replaces the library's check (then ctx may be None); disable holds
    BP_SOLVE_OFF_* bits."""
    lib = load()
    w = _i32arr(sizes)
    cb = bp_check_fn()
    if check is not None:
        def _cb(user, C_, m_, pres, punp, n_, plb):
            try:
                res = np.ctypeslib.as_array(pres, shape=(m_,)).copy() if m_ else np.zeros(0, np.int32)
                unp = np.ctypeslib.as_array(punp, shape=(n_,)).copy() if n_ else np.zeros(0, np.int32)
                plb[0] = int(check(C_, res, unp))
                return BP_OK
            except Exception:  # an exception cannot cross the C boundary: stop the search
                return BP_ERR_STATE
        cb = bp_check_fn(_cb)
    opts = bp_solve_opts(mode, check_flags, max_nodes, time_limit_s, cb, None, disable, 0)
    out = bp_solve_result()
    bin_of = np.zeros(max(len(w), 1), dtype=np.int32)
    _check(lib.bp_solve(ctx.handle if ctx is not None else None, C, len(w), _p32(w) if len(w) else None,
                        ctypes.byref(opts), _p32(bin_of), ctypes.byref(out)))
    res = {f: getattr(out, f) for f, _ in bp_solve_result._fields_}
    return res, bin_of[: len(w)].copy()


def subset_sum_gap(sizes, alpha: int, beta: int):
    """bp_subset_sum_gap over sizes (sorted here, largest first): None when
    nothing is proved, else (below, above) with every subset sum <= below or
    >= above."""
    x = np.sort(_i32arr(sizes))[::-1].copy()
    below, above = _i64(), _i64()
    r = load().bp_subset_sum_gap(_p32(x) if len(x) else None, len(x), alpha, beta, ctypes.byref(below),
                                 ctypes.byref(above))
    if r < 0:
        _check(r)
    return (below.value, above.value) if r == 1 else None


def selftest_division(d_lo: int, d_hi: int, n_hi: int, mode: int) -> int:
    return int(load().bp_selftest_division(d_lo, d_hi, n_hi, mode))


class _Batch:
    """Keeps the numpy arrays behind a bp_batch alive."""

    def __init__(self, Cs, ks, items_list=None, off=None, items=None):
        if items_list is not None:
            lens = np.array([len(x) for x in items_list], dtype=np.int64)
            self.off = np.zeros(len(lens) + 1, dtype=np.int64)
            np.cumsum(lens, out=self.off[1:])
            self.items = np.ascontiguousarray(np.concatenate([_i32arr(x) for x in items_list])
                                              if len(items_list) else np.zeros(0, np.int32))
        else:
            self.off = np.ascontiguousarray(np.asarray(off, dtype=np.int64))
            self.items = _i32arr(items) if items is not None else np.zeros(1, np.int32)
        self.C = _i32arr(Cs)
        self.k = _i32arr(ks)
        self.s = bp_batch(len(self.C), 0, self.off.ctypes.data_as(_P64),
                          _p32(self.items) if self.items.size else _p32(np.zeros(1, np.int32)),
                          _p32(self.C), _p32(self.k))


class Context:
    """A bp_ctx on one GPU."""

    def __init__(self, device: int = 0):
        self._lib = load()
        h = _VP()
        _check(self._lib.bp_ctx_create(device, ctypes.byref(h)))
        self.handle = h

    def close(self):
        if self.handle:
            _check(self._lib.bp_ctx_destroy(self.handle))
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- reduction --
    def residual_reduce(self, C: int, residual, unpacked) -> np.ndarray:
        res, unp = _i32arr(residual), _i32arr(unpacked)
        out = np.zeros(len(res) + len(unp) + 1, dtype=np.int32)
        r = _i64(0)
        _check(self._lib.bp_residual_reduce(self.handle, C, len(res), _p32(res), _p32(unp), len(unp), _p32(out),
                                            ctypes.byref(r)))
        return out[: r.value].copy()

    def assignment_reduce(self, C: int, m: int, size, bin_of):
        s, b = _i32arr(size), _i32arr(bin_of)
        out = np.zeros(len(s) + m + 1, dtype=np.int32)
        res = np.zeros(max(m, 1), dtype=np.int32)
        r = _i64(0)
        _check(self._lib.bp_assignment_reduce(self.handle, C, m, _p32(s), _p32(b), len(s), _p32(out),
                                              ctypes.byref(r), _p32(res)))
        return out[: r.value].copy(), res[:m].copy()

    # -- single checks --
    def lower_bounds(self, C: int, k: int, items, sweep: bp_sweep | None = None) -> dict:
        a = _i32arr(items)
        out = bp_bounds()
        _check(self._lib.bp_lower_bounds(self.handle, C, k, _p32(a), len(a),
                                         ctypes.byref(sweep) if sweep is not None else None, ctypes.byref(out)))
        return bounds_to_dict(out)

    def lower_bounds_dev(self, C: int, k: int, d_items_ptr: int, r: int, d_out_ptr: int, stream_ptr: int,
                         sweep: bp_sweep | None = None):
        _check(self._lib.bp_lower_bounds_dev(self.handle, C, k, _VP(d_items_ptr), r,
                                             ctypes.byref(sweep) if sweep is not None else None,
                                             _VP(d_out_ptr), _VP(stream_ptr)))

    def feasible(self, C: int, residual, unpacked, flags: int = 0) -> dict:
        res, unp = _i32arr(residual), _i32arr(unpacked)
        v, lb, out = _i32(0), _i64(0), bp_bounds()
        _check(self._lib.bp_feasible(self.handle, C, len(res), _p32(res), _p32(unp), len(unp), flags,
                                     ctypes.byref(v), ctypes.byref(lb), ctypes.byref(out)))
        d = bounds_to_dict(out)
        assert d["verdict"] == v.value and d["lb"] == lb.value
        return d

    def feasible_dev(self, C: int, m: int, d_residual_ptr: int, n: int, d_unpacked_ptr: int, d_out_ptr: int,
                     stream_ptr: int, flags: int = 0):
        _check(self._lib.bp_feasible_dev(self.handle, C, m, _VP(d_residual_ptr), _VP(d_unpacked_ptr), n, flags,
                                         _VP(d_out_ptr), _VP(stream_ptr)))

    def set_timing(self, enable: bool):
        _check(self._lib.bp_ctx_set_timing(self.handle, int(enable)))

    def get_tuning(self) -> dict:
        t = bp_tuning()
        _check(self._lib.bp_ctx_get_tuning(self.handle, ctypes.byref(t)))
        return {f: getattr(t, f) for f, _ in bp_tuning._fields_}

    def set_tuning(self, lanes_params: int, waves_per_cu: int, tasks_per_wave: int, min_chunk: int):
        t = bp_tuning(lanes_params, waves_per_cu, tasks_per_wave, min_chunk)
        _check(self._lib.bp_ctx_set_tuning(self.handle, ctypes.byref(t)))

    def autotune_batch(self, Cs, ks, items_list, reps: int = 2, sweeps=None):
        """Pick the fastest sweep shape for this batch; returns (tuning dict, sweep ms)."""
        b = _Batch(Cs, ks, items_list)
        sw = None
        if sweeps is not None:
            arr = (bp_sweep * len(sweeps))(*sweeps)
            sw = ctypes.cast(arr, ctypes.POINTER(bp_sweep))
        t = bp_tuning()
        ms = ctypes.c_double(0)
        _check(self._lib.bp_autotune_batch(self.handle, ctypes.byref(b.s), sw, reps, ctypes.byref(t), ctypes.byref(ms)))
        return {f: getattr(t, f) for f, _ in bp_tuning._fields_}, ms.value

    def autotune_batch_cached(self, Cs, ks, items_list, cache_path: str | None, reps: int = 1, sweeps=None):
        """The autotuner through a cache file: (tuning dict, sweep ms, from_cache)."""
        b = _Batch(Cs, ks, items_list)
        sw = None
        if sweeps is not None:
            arr = (bp_sweep * len(sweeps))(*sweeps)
            sw = ctypes.cast(arr, ctypes.POINTER(bp_sweep))
        t = bp_tuning()
        ms = ctypes.c_double(0)
        fc = ctypes.c_int32(0)
        _check(self._lib.bp_autotune_batch_cached(self.handle, ctypes.byref(b.s), sw, reps,
                                                  cache_path.encode() if cache_path else None, ctypes.byref(t),
                                                  ctypes.byref(ms), ctypes.byref(fc)))
        return {f: getattr(t, f) for f, _ in bp_tuning._fields_}, ms.value, bool(fc.value)

    def set_order(self, order=None):
        """Schedule the six functions' tiles in this order (None: longest first)."""
        if order is None:
            _check(self._lib.bp_ctx_set_order(self.handle, None))
        else:
            arr = _i32arr(order)
            _check(self._lib.bp_ctx_set_order(self.handle, _p32(arr)))

    def stage_times(self, with_runs: bool = False):
        """Mean durations (ms) of prep, sweep and finalize over the calls made
        since timing was switched on; with_runs also returns how many."""
        ms = (ctypes.c_double * 3)()
        runs = ctypes.c_int64(0)
        _check(self._lib.bp_ctx_stage_times(self.handle, ms, ctypes.byref(runs)))
        return (list(ms), runs.value) if with_runs else list(ms)

    # -- batches --
    def lower_bounds_batch(self, Cs, ks, items_list, sweeps=None) -> np.ndarray:
        b = _Batch(Cs, ks, items_list)
        out = np.zeros(len(b.C), dtype=BOUNDS_DTYPE)
        sw = None
        if sweeps is not None:
            arr = (bp_sweep * len(sweeps))(*sweeps)
            sw = ctypes.cast(arr, ctypes.POINTER(bp_sweep))
        _check(self._lib.bp_lower_bounds_batch(self.handle, ctypes.byref(b.s), sw, out.ctypes.data_as(_VP)))
        return out

    def lower_bounds_batch_dev(self, Cs, ks, off, d_items_ptr: int, d_out_ptr: int, stream_ptr: int, sweeps=None):
        b = _Batch(Cs, ks, off=off)
        sw = None
        if sweeps is not None:
            arr = (bp_sweep * len(sweeps))(*sweeps)
            sw = ctypes.cast(arr, ctypes.POINTER(bp_sweep))
        _check(self._lib.bp_lower_bounds_batch_dev(self.handle, ctypes.byref(b.s), _VP(d_items_ptr), sw,
                                                   _VP(d_out_ptr), _VP(stream_ptr)))

    def feasible_batch(self, Cs, ks, items_list, flags: int = 0, records: bool = False):
        """(verdict, lb), plus the records when records=True."""
        b = _Batch(Cs, ks, items_list)
        v = np.zeros(len(b.C), dtype=np.int32)
        lb = np.zeros(len(b.C), dtype=np.int64)
        rec = np.zeros(len(b.C), dtype=BOUNDS_DTYPE) if records else None
        _check(self._lib.bp_feasible_batch(self.handle, ctypes.byref(b.s), flags, _p32(v), lb.ctypes.data_as(_P64),
                                           rec.ctypes.data_as(_VP) if records else None))
        return (v, lb, rec) if records else (v, lb)


class Queue:
    """A bp_queue: continuous batching of feasibility checks on one context."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int, max_slots: int):
        self._lib = ctx._lib
        self.ctx = ctx
        h = _VP()
        _check(self._lib.bp_queue_create(ctx.handle, hbm_budget_bytes, max_slots, ctypes.byref(h)))
        self.handle = h

    def submit(self, C: int, residual, unpacked, tag: int = 0, flags: int = 0, blocking: bool = True) -> int:
        res, unp = _i32arr(residual), _i32arr(unpacked)
        req = bp_request(C, len(res), len(unp), _p32(res), _p32(unp), tag, flags, 0, 0, None, 0, 0)
        t = _u64(0)
        _check(self._lib.bp_queue_submit(self.handle, ctypes.byref(req), int(blocking), ctypes.byref(t)))
        return int(t.value)

    def submit_child(self, C: int, m: int, parent: int, commits, tag: int = 0, flags: int = 0,
                     blocking: bool = True, residual=None, unpacked=None) -> int:
        """A node reached from request `parent` by committing (size, bin) pairs;
        its instance may be given too (used only when the parent is gone)."""
        arr = (bp_commit * max(len(commits), 1))(*[bp_commit(int(w), int(b)) for w, b in commits])
        if residual is not None:
            res, unp = _i32arr(residual), _i32arr(unpacked)
            pr, pu, n = _p32(res), _p32(unp), len(unp)
        else:
            pr = pu = None
            n = 0
        req = bp_request(C, m, n, pr, pu, tag, flags, 0, parent, arr, len(commits), 0)
        t = _u64(0)
        _check(self._lib.bp_queue_submit(self.handle, ctypes.byref(req), int(blocking), ctypes.byref(t)))
        return int(t.value)

    def try_submit(self, C: int, residual, unpacked, tag: int = 0, flags: int = 0):
        """Non-blocking submit: ticket, or None when the queue is full (BP_ERR_AGAIN)."""
        res, unp = _i32arr(residual), _i32arr(unpacked)
        req = bp_request(C, len(res), len(unp), _p32(res), _p32(unp), tag, flags, 0, 0, None, 0, 0)
        t = _u64(0)
        st = self._lib.bp_queue_submit(self.handle, ctypes.byref(req), 0, ctypes.byref(t))
        if st == BP_ERR_AGAIN:
            return None
        _check(st)
        return int(t.value)

    def poll(self, max_results: int = 256, timeout_us: int = 0):
        arr = (bp_result * max_results)()
        got = _i32(0)
        _check(self._lib.bp_queue_poll(self.handle, ctypes.cast(arr, _VP), max_results, ctypes.byref(got),
                                       timeout_us))
        return [arr[i] for i in range(got.value)]

    def stats(self) -> dict:
        s = bp_queue_stats()
        _check(self._lib.bp_queue_stats_get(self.handle, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in bp_queue_stats._fields_}

    def close(self):
        if self.handle:
            _check(self._lib.bp_queue_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
