"""Thin Python binding of the HIP PDHG library (libscylla_pdhg.so).

Argument marshalling only: every step of the solve runs in the library's
kernels.  Names follow the C ABI in include/scylla_pdhg.h.  The binding
raises if the library has not been built; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libscylla_pdhg.so")

FP64, FP32 = 0, 1
RUNNING, OPTIMAL, ITERATION_LIMIT, TIME_LIMIT, NUMERICAL_ERROR, PRIMAL_INFEASIBLE, DUAL_INFEASIBLE = 0, 1, 2, 3, 4, 5, 6
STALLED = 7
FORMATS = {0: "packed-int", 1: "bf16", 2: "fp32", 3: "fp64"}

EXPORTS = [
    "scylla_params_default", "scylla_last_error", "scylla_validate_lp", "scylla_pdhg_solve",
    "scylla_batch_create", "scylla_batch_destroy", "scylla_batch_set_objective",
    "scylla_batch_set_blend", "scylla_batch_set_start", "scylla_batch_solve",
    "scylla_batch_get_solution", "scylla_batch_get_x_all", "scylla_batch_device_iterates",
    "scylla_batch_get_info", "scylla_batch_time_passes", "scylla_batch_set_layout",
    "scylla_batch_set_cached_loads",
    "scylla_fix_propagate", "scylla_batch_pump",
    "scylla_pump_params_default", "scylla_batch_pump_ex", "scylla_batch_set_quadratic",
    "scylla_batch_mip_feasible", "scylla_batch_fix_propagate", "scylla_batch_mip_feasible_static",
    "scylla_batch_set_start_device", "scylla_batch_get_average",
]


class ScyllaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"scylla error {code}: {msg}")
        self.code = code


class CSR(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class LPDesc(ctypes.Structure):
    _fields_ = [("A", CSR), ("c", ctypes.c_void_p), ("b", ctypes.c_void_p),
                ("senses", ctypes.c_void_p), ("l", ctypes.c_void_p), ("u", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("iter_limit", ctypes.c_int64),
                ("precision", ctypes.c_int32), ("check_period", ctypes.c_int32),
                ("restarts", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("eta", ctypes.c_double), ("time_limit_s", ctypes.c_double),
                ("fused_window", ctypes.c_int32), ("adaptive", ctypes.c_int32),
                ("infeas_tol", ctypes.c_double), ("stall_tol", ctypes.c_double),
                ("stall_checks", ctypes.c_int32), ("restart_avg", ctypes.c_int32),
                ("compact", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("iterations", ctypes.c_int64), ("rel_kkt", ctypes.c_double),
                ("rho_primal", ctypes.c_double), ("rho_dual", ctypes.c_double),
                ("rho_gap", ctypes.c_double), ("primal_obj", ctypes.c_double),
                ("dual_obj", ctypes.c_double), ("omega", ctypes.c_double),
                ("solve_seconds", ctypes.c_double), ("setup_seconds", ctypes.c_double),
                ("tune_seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BatchInfo(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("format", ctypes.c_int32), ("fused_eligible", ctypes.c_int32),
                ("m_total", ctypes.c_int64), ("n_total", ctypes.c_int64),
                ("nnz_total", ctypes.c_int64), ("row_chunk", ctypes.c_int32),
                ("col_chunk", ctypes.c_int32), ("long_rows", ctypes.c_int32),
                ("long_cols", ctypes.c_int32), ("row_blocks", ctypes.c_int32),
                ("col_blocks", ctypes.c_int32), ("row_staged_nnz", ctypes.c_int32),
                ("col_staged_nnz", ctypes.c_int32), ("row_staged_variant", ctypes.c_int32),
                ("col_staged_variant", ctypes.c_int32), ("row_sliced", ctypes.c_int32),
                ("col_sliced", ctypes.c_int32), ("row_slices", ctypes.c_int32), ("col_slices", ctypes.c_int32),
                ("row_half_lds", ctypes.c_int32), ("col_half_lds", ctypes.c_int32),
                ("row_tile_threads", ctypes.c_int32), ("col_tile_threads", ctypes.c_int32),
                ("row_direct", ctypes.c_int32), ("col_direct", ctypes.c_int32),
                ("row_cached", ctypes.c_int32), ("col_cached", ctypes.c_int32)]


_lib = None


def lib():
    """Loads the built library (raises if it is missing: no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
        sig = {
            "scylla_params_default": ([ctypes.POINTER(Params)], ctypes.c_int),
            "scylla_last_error": ([], ctypes.c_char_p),
            "scylla_validate_lp": ([ctypes.POINTER(LPDesc)], ctypes.c_int),
            "scylla_pdhg_solve": ([ctypes.POINTER(CSR), vp, vp, vp, vp, vp, ctypes.POINTER(Params),
                                   vp, vp, vp, vp, ctypes.POINTER(Result)], ctypes.c_int),
            "scylla_batch_create": ([ctypes.POINTER(LPDesc), i32, i32, vp, ctypes.POINTER(vp)], ctypes.c_int),
            "scylla_batch_destroy": ([vp], None),
            "scylla_batch_set_objective": ([vp, i32, vp], ctypes.c_int),
            "scylla_batch_set_blend": ([vp, i32, vp, vp, dbl, dbl], ctypes.c_int),
            "scylla_batch_set_quadratic": ([vp, i32, vp], ctypes.c_int),
            "scylla_batch_set_start": ([vp, i32, vp, vp, dbl], ctypes.c_int),
            "scylla_batch_set_start_device": ([vp, vp, vp, vp], ctypes.c_int),
            "scylla_batch_solve": ([vp, ctypes.POINTER(Params), i32, ctypes.POINTER(Result)], ctypes.c_int),
            "scylla_batch_get_solution": ([vp, i32, vp, vp], ctypes.c_int),
            "scylla_batch_get_average": ([vp, i32, vp, vp], ctypes.c_int),
            "scylla_batch_get_x_all": ([vp, vp], ctypes.c_int),
            "scylla_batch_device_iterates": ([vp, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                              ctypes.POINTER(i32)], ctypes.c_int),
            "scylla_batch_get_info": ([vp, ctypes.POINTER(BatchInfo)], ctypes.c_int),
            "scylla_batch_time_passes": ([vp, i32, ctypes.POINTER(dbl), ctypes.POINTER(dbl)], ctypes.c_int),
            "scylla_batch_set_layout": ([vp, i32, i32, i32, i32], ctypes.c_int),
            "scylla_batch_set_cached_loads": ([vp, i32, i32], ctypes.c_int),
            "scylla_fix_propagate": ([ctypes.POINTER(LPDesc), vp, vp, vp, vp], ctypes.c_int),
            "scylla_batch_pump": ([vp, ctypes.POINTER(Params), vp, i32, dbl, i32, ctypes.POINTER(PumpRecord), vp],
                                  ctypes.c_int),
            "scylla_pump_params_default": ([ctypes.POINTER(PumpParams)], ctypes.c_int),
            "scylla_batch_mip_feasible": ([vp, vp, dbl, vp], ctypes.c_int),
            "scylla_batch_mip_feasible_static": ([vp, vp, dbl, vp], ctypes.c_int),
            "scylla_batch_fix_propagate": ([vp, vp, vp, i32, i32, vp, vp, vp], ctypes.c_int),
            "scylla_batch_pump_ex": ([vp, ctypes.POINTER(Params), vp, ctypes.POINTER(PumpParams),
                                      ctypes.POINTER(PumpRecord), ctypes.POINTER(PumpOutcome), vp], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise ScyllaError(rc, lib().scylla_last_error().decode())


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def params(**kw) -> Params:
    p = Params()
    _check(lib().scylla_params_default(ctypes.byref(p)))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k}")
        setattr(p, k, v)
    return p


class PumpRecord(ctypes.Structure):
    _fields_ = [("round", ctypes.c_int32), ("status", ctypes.c_int32), ("iterations", ctypes.c_int64),
                ("rel_kkt", ctypes.c_double), ("lp_feasible", ctypes.c_int32),
                ("xhat_feasible", ctypes.c_int32), ("ignored_rows", ctypes.c_int32),
                ("perturbed", ctypes.c_int32), ("xhat_obj", ctypes.c_double),
                ("solve_seconds", ctypes.c_double), ("round_seconds", ctypes.c_double),
                ("tune_seconds", ctypes.c_double), ("rounding_seconds", ctypes.c_double),
                ("group", ctypes.c_int32), ("pad", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class PumpParams(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("eps_schedule", ctypes.c_int32), ("eps1", ctypes.c_double),
                ("beta", ctypes.c_double), ("eps_floor", ctypes.c_double), ("alpha", ctypes.c_double),
                ("total_iter_limit", ctypes.c_int64), ("early_exit", ctypes.c_int32),
                ("perturb", ctypes.c_int32), ("seed", ctypes.c_uint64), ("threads", ctypes.c_int32),
                ("distance", ctypes.c_int32), ("pipeline", ctypes.c_int32),
                ("fp_batch", ctypes.c_int32), ("fp_max_rounds", ctypes.c_int32)]


class PumpOutcome(ctypes.Structure):
    _fields_ = [("found_kind", ctypes.c_int32), ("found_round", ctypes.c_int32),
                ("rounds_run", ctypes.c_int32), ("perturbations", ctypes.c_int32),
                ("iterations", ctypes.c_int64), ("obj", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def pump_params(**kw) -> PumpParams:
    o = PumpParams()
    _check(lib().scylla_pump_params_default(ctypes.byref(o)))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown pump parameter {k}")
        setattr(o, k, v)
    return o


class _LPArrays:
    """Contiguous host copies of one LP kept alive for the duration of a call."""

    def __init__(self, lp, c=None):
        self.row_ptr = np.ascontiguousarray(lp.row_ptr, dtype=np.int64)
        self.col_idx = np.ascontiguousarray(lp.col_idx, dtype=np.int32)
        self.val = np.ascontiguousarray(lp.val, dtype=np.float64)
        self.c = np.ascontiguousarray(lp.c if c is None else c, dtype=np.float64)
        self.b = np.ascontiguousarray(lp.b, dtype=np.float64)
        self.senses = np.ascontiguousarray(lp.senses, dtype=np.uint8)
        self.l = np.ascontiguousarray(lp.l, dtype=np.float64)
        self.u = np.ascontiguousarray(lp.u, dtype=np.float64)
        self.csr = CSR(lp.m, lp.n, int(self.row_ptr[-1]) if self.row_ptr.size else 0,
                       _ptr(self.row_ptr), _ptr(self.col_idx), _ptr(self.val))
        self.desc = LPDesc(self.csr, _ptr(self.c), _ptr(self.b), _ptr(self.senses), _ptr(self.l),
                           _ptr(self.u))


def validate(lp) -> None:
    a = _LPArrays(lp)
    _check(lib().scylla_validate_lp(ctypes.byref(a.desc)))


def fix_propagate(lp, x_ref, is_int=None):
    """Host fix-and-propagate rounding (library implementation).  Returns
    (x_hat, feasible, ignored_rows)."""
    a = _LPArrays(lp)
    ii = np.ascontiguousarray(lp.is_int if is_int is None else is_int, dtype=np.uint8)
    xr = np.ascontiguousarray(x_ref, dtype=np.float64)
    xh = np.empty(lp.n)
    info = np.zeros(2, dtype=np.int32)
    _check(lib().scylla_fix_propagate(ctypes.byref(a.desc), _ptr(ii), _ptr(xr), _ptr(xh), _ptr(info)))
    return xh, bool(info[0]), int(info[1])


@dataclass
class Solution:
    x: np.ndarray
    y: np.ndarray
    result: dict


def solve(lp, x0=None, y0=None, **kw) -> Solution:
    """One-shot solve (scylla_pdhg_solve) of an LP with host arrays."""
    a = _LPArrays(lp)
    p = params(**kw)
    x = np.empty(lp.n)
    y = np.empty(max(lp.m, 1))
    x0a = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
    y0a = None if y0 is None else np.ascontiguousarray(y0, dtype=np.float64)
    r = Result()
    _check(lib().scylla_pdhg_solve(ctypes.byref(a.csr), _ptr(a.c), _ptr(a.b), _ptr(a.senses), _ptr(a.l),
                                   _ptr(a.u), ctypes.byref(p), _ptr(x0a), _ptr(y0a), _ptr(x), _ptr(y),
                                   ctypes.byref(r)))
    return Solution(x, y[: lp.m], r.as_dict())


class Batch:
    """Device-resident batch of LPs (scylla_batch_*)."""

    def __init__(self, lps: Sequence, precision: int = FP32, stream=None):
        self._arrays = [_LPArrays(lp) for lp in lps]
        descs = (LPDesc * len(lps))(*[a.desc for a in self._arrays])
        h = ctypes.c_void_p()
        s = None if stream is None else ctypes.c_void_p(stream)
        _check(lib().scylla_batch_create(descs, len(lps), precision, s, ctypes.byref(h)))
        self._h = h
        self.count = len(lps)
        self.precision = precision
        self.m = [lp.m for lp in lps]
        self.n = [lp.n for lp in lps]
        self._arrays = None  # data is on the device now

    def close(self):
        if getattr(self, "_h", None):
            lib().scylla_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def info(self) -> dict:
        inf = BatchInfo()
        _check(lib().scylla_batch_get_info(self._h, ctypes.byref(inf)))
        d = {k: getattr(inf, k) for k, _ in inf._fields_}
        d["format_name"] = FORMATS.get(d["format"], "?")
        return d

    def solve(self, warm: bool = False, **kw) -> List[dict]:
        p = params(precision=self.precision, **kw)
        res = (Result * self.count)()
        _check(lib().scylla_batch_solve(self._h, ctypes.byref(p), int(warm), res))
        return [r.as_dict() for r in res]

    def solution(self, inst: int = 0):
        x = np.empty(self.n[inst])
        y = np.empty(max(self.m[inst], 1))
        _check(lib().scylla_batch_get_solution(self._h, inst, _ptr(x), _ptr(y)))
        return x, y[: self.m[inst]]

    def average(self, inst: int = 0):
        """Running means of x and y since instance `inst`'s last restart
        (solves with restart_avg=1)."""
        x = np.empty(self.n[inst])
        y = np.empty(max(self.m[inst], 1))
        _check(lib().scylla_batch_get_average(self._h, inst, _ptr(x), _ptr(y)))
        return x, y[: self.m[inst]]

    def x_all(self) -> np.ndarray:
        x = np.empty(sum(self.n))
        _check(lib().scylla_batch_get_x_all(self._h, _ptr(x)))
        return x

    def set_objective(self, inst: int, c_hat) -> None:
        c = np.ascontiguousarray(c_hat, dtype=np.float64)
        assert c.size == self.n[inst]
        _check(lib().scylla_batch_set_objective(self._h, inst, _ptr(c)))

    def set_blend(self, inst: int, xhat_up: np.ndarray, a: float, kappa: float, is_int=None) -> None:
        """xhat_up[j] = True where the rounded value sits at the upper bound."""
        bits = np.packbits(np.asarray(xhat_up, dtype=bool), bitorder="little")
        ib = None if is_int is None else np.packbits(np.asarray(is_int, dtype=bool), bitorder="little")
        _check(lib().scylla_batch_set_blend(self._h, inst, _ptr(bits), _ptr(ib), a, kappa))

    def set_start(self, inst: int, x0=None, y0=None, omega0: float = 0.0) -> None:
        x = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
        y = None if y0 is None else np.ascontiguousarray(y0, dtype=np.float64)
        _check(lib().scylla_batch_set_start(self._h, inst, _ptr(x), _ptr(y), omega0))

    def set_start_device(self, x0_ptr: int | None, y0_ptr: int | None, omega0=None) -> None:
        """Warm start of every instance from device FP64 buffers (raw device
        pointers to the concatenated x0 [n_total] / y0 [m_total], or None)."""
        om = None if omega0 is None else np.ascontiguousarray(omega0, dtype=np.float64)
        _check(lib().scylla_batch_set_start_device(self._h, x0_ptr, y0_ptr, _ptr(om)))

    def pump(self, rounds: int = 20, alpha: float = 0.9, is_int=None, threads: int = 0, **kw):
        """Native pump loop; returns (records [rounds][count] as dicts, x_hat_all)."""
        p = params(precision=self.precision, **kw)
        recs = (PumpRecord * (rounds * self.count))()
        ii = None if is_int is None else np.ascontiguousarray(is_int, dtype=np.uint8)
        xh = np.empty(sum(self.n))
        _check(lib().scylla_batch_pump(self._h, ctypes.byref(p), _ptr(ii), rounds, alpha, threads, recs, _ptr(xh)))
        out = [[recs[k * self.count + q].as_dict() for q in range(self.count)] for k in range(rounds)]
        return out, xh

    def mip_feasible(self, is_int=None, tol: float = 1e-6) -> np.ndarray:
        """Device MIP-feasibility of every instance's current x: [count] 0/1."""
        ii = None if is_int is None else np.ascontiguousarray(is_int, dtype=np.uint8)
        out = np.zeros(self.count, dtype=np.int32)
        _check(lib().scylla_batch_mip_feasible(self._h, _ptr(ii), tol, _ptr(out)))
        return out

    def mip_feasible_static(self, is_int=None, tol: float = 1e-6) -> np.ndarray:
        """mip_feasible through the allocation-free entry point
        (scylla_batch_mip_feasible_static)."""
        ii = None if is_int is None else np.ascontiguousarray(is_int, dtype=np.uint8)
        out = np.zeros(self.count, dtype=np.int32)
        _check(lib().scylla_batch_mip_feasible_static(self._h, _ptr(ii), tol, _ptr(out)))
        return out

    def fix_propagate(self, K: int, max_rounds: int = 1000, is_int=None, xbar=None):
        """Batched fix-and-propagate of every instance on the device
        (scylla_batch_fix_propagate), rounding `xbar` (all instances
        concatenated) or, if None, the current iterates.  Returns (x_hat,
        feasible [count] bool, ignored rows [count], ignored mask [m_total])."""
        ii = None if is_int is None else np.ascontiguousarray(is_int, dtype=np.uint8)
        xb = None if xbar is None else np.ascontiguousarray(xbar, dtype=np.float64)
        xh = np.empty(sum(self.n))
        info = np.zeros(2 * self.count, dtype=np.int32)
        mask = np.zeros(max(1, sum(self.m)), dtype=np.uint8)
        _check(lib().scylla_batch_fix_propagate(self._h, _ptr(ii), _ptr(xb), K, max_rounds, _ptr(xh),
                                                _ptr(info), _ptr(mask)))
        return xh, info[0::2].astype(bool), info[1::2].copy(), mask[: sum(self.m)].astype(bool)

    def set_quadratic(self, inst: int, q):
        """Diagonal Hessian (>= 0) of instance `inst`'s objective, or None."""
        qa = None if q is None else np.ascontiguousarray(q, dtype=np.float64)
        _check(lib().scylla_batch_set_quadratic(self._h, inst, _ptr(qa)))

    def pump_ex(self, is_int=None, pump: dict | None = None, **kw):
        """Complete Algorithm 1 loop (scylla_batch_pump_ex).  `pump` holds
        scylla_pump_params fields, `kw` scylla_params fields.  Returns
        (records [rounds][count] as dicts, outcomes [count] as dicts, x_out)."""
        p = params(precision=self.precision, **kw)
        o = pump_params(**(pump or {}))
        recs = (PumpRecord * (o.rounds * self.count))()
        outs = (PumpOutcome * self.count)()
        ii = None if is_int is None else np.ascontiguousarray(is_int, dtype=np.uint8)
        xo = np.empty(sum(self.n))
        _check(lib().scylla_batch_pump_ex(self._h, ctypes.byref(p), _ptr(ii), ctypes.byref(o), recs, outs,
                                          _ptr(xo)))
        out = [[recs[k * self.count + q].as_dict() for q in range(self.count)] for k in range(o.rounds)]
        return out, [outs[q].as_dict() for q in range(self.count)], xo

    def set_layout(self, row_blocks: int = 0, row_ept: int = 8, col_blocks: int = 0, col_ept: int = 8):
        """Pin the tile plan (-6 / -7 / -8 direct staged with at least 1 / 4 / 8 lanes per row,
        -3 as -2 in half the LDS, -2 LDS-staged + sliced, -1 LDS-staged, 0 normal,
        2 / 4 / 8 gather blocks; 2 / 4 / 8 / 16 nonzeros per thread, or -8 / -16 on
        1024-thread workgroups)."""
        _check(lib().scylla_batch_set_layout(self._h, row_blocks, row_ept, col_blocks, col_ept))

    def set_cached_loads(self, row: int = 1, col: int = 1):
        """Matrix load policy of the iteration passes: plain (cacheable)
        loads (1) or non-temporal ones (0)."""
        _check(lib().scylla_batch_set_cached_loads(self._h, row, col))

    def time_passes(self, reps: int = 20):
        """Average ms of one launch of the row pass and of the column pass."""
        a, b = ctypes.c_double(), ctypes.c_double()
        _check(lib().scylla_batch_time_passes(self._h, reps, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def device_iterates(self):
        x, y, eb = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_int32()
        _check(lib().scylla_batch_device_iterates(self._h, ctypes.byref(x), ctypes.byref(y), ctypes.byref(eb)))
        return x.value, y.value, eb.value
