"""Plain FP64 CPU oracle for the Scylla LP hot path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg may import this package; the HIP library and its Python binding
never do.  The heavy loops (PDHG, KKT, fix-and-propagate) are plain C in
``scylla_oracle.c``; the pump objective update (Algorithm 1, objective update
step; Section 2.4) and the tolerance schedule (Section 2.2) are written here
with numpy.

Parity status of each function (pins live in tests/test_oracle_*.py):
  precondition, pdhg, kkt       pinned (brute force, closed forms, HiGHS,
                                independent KKT, invariants, fixed point,
                                nonexpansiveness, ||A~|| <= 1); the restart
                                rule, the cold-start primal weight and its
                                update, and the adaptive step rule are
                                restated from snapshot iterates with
                                independently computed norms
                                (tests/test_oracle_steps.py)
  fix_propagate                 pinned (integrality/bounds, identity on
                                feasible integral input, set-cover success,
                                brute-force propagation soundness)
  fix_propagate_batched         pinned (hand-worked round cap, conflict and
                                tolerance cases, plain rounding without
                                rows, fixpoint at x_hat, equal to
                                fix_propagate for K = 1 where neither
                                ignores a row)
  objective_update(_l2),        pinned (closed forms / norm identities,
  eps_schedule                  the QP form equals the L2 distance up to a
                                constant)
  pump, scylla                  parity unpinned: the round of first success
                                depends on rounding choices the paper leaves
                                open; only invariants are checked (early
                                exit, schedule, budget, perturbation rule).
  splitmix64                    pinned (published reference outputs)
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np
from typing import Optional

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "scylla_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OPTIMAL, ITERATION_LIMIT, NUMERICAL_ERROR, PRIMAL_INFEASIBLE, DUAL_INFEASIBLE = 1, 2, 4, 5, 6
STALLED = 7


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain -O2, no vectorisation tricks)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _LPStruct(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("n", ctypes.c_int32),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("val", ctypes.c_void_p), ("c", ctypes.c_void_p), ("b", ctypes.c_void_p),
                ("sense", ctypes.c_void_p), ("l", ctypes.c_void_p), ("u", ctypes.c_void_p),
                ("q", ctypes.c_void_p)]


class _Params(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("iter_limit", ctypes.c_int64),
                ("check_period", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("eta", ctypes.c_double), ("ruiz_iters", ctypes.c_int32),
                ("pock_chambolle", ctypes.c_int32), ("omega0", ctypes.c_double),
                ("adaptive", ctypes.c_int32), ("infeas_tol", ctypes.c_double),
                ("stall_tol", ctypes.c_double), ("stall_checks", ctypes.c_int32),
                ("restart_avg", ctypes.c_int32)]


class _Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("iterations", ctypes.c_int64), ("rel_kkt", ctypes.c_double),
                ("rho_p", ctypes.c_double), ("rho_d", ctypes.c_double),
                ("rho_g", ctypes.c_double), ("pobj", ctypes.c_double),
                ("dobj", ctypes.c_double), ("omega", ctypes.c_double), ("eta", ctypes.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        for fn in ("orc_precondition", "orc_kkt", "orc_pdhg", "orc_pdhg_avg", "orc_fix_propagate", "orc_ray",
                   "orc_fix_propagate_batched"):
            getattr(lib, fn).restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


class _Pinned:
    """Keeps contiguous numpy copies alive while C uses them."""

    def __init__(self, lp, c=None, q=None):
        self.row_ptr = np.ascontiguousarray(lp.row_ptr, dtype=np.int64)
        self.col_idx = np.ascontiguousarray(lp.col_idx, dtype=np.int32)
        self.val = np.ascontiguousarray(lp.val, dtype=np.float64)
        self.c = np.ascontiguousarray(lp.c if c is None else c, dtype=np.float64)
        self.b = np.ascontiguousarray(lp.b, dtype=np.float64)
        self.sense = np.ascontiguousarray(lp.senses, dtype=np.uint8)
        self.l = np.ascontiguousarray(lp.l, dtype=np.float64)
        self.u = np.ascontiguousarray(lp.u, dtype=np.float64)
        self.q = None if q is None else np.ascontiguousarray(q, dtype=np.float64)
        if self.q is not None and (self.q.shape != (lp.n,) or np.any(~(self.q >= 0))):
            raise ValueError("q must be a nonnegative [n] vector")
        self.s = _LPStruct(lp.m, lp.n, _p(self.row_ptr), _p(self.col_idx), _p(self.val),
                           _p(self.c), _p(self.b), _p(self.sense), _p(self.l), _p(self.u), _p(self.q))


@dataclass
class PDHGResult:
    x: np.ndarray
    y: np.ndarray
    status: int
    iterations: int
    restarts: int
    rel_kkt: float
    rho_p: float
    rho_d: float
    rho_g: float
    pobj: float
    dobj: float
    omega: float
    eta: float
    x_avg: Optional[np.ndarray] = None  # running means (restart_avg) at the stop
    y_avg: Optional[np.ndarray] = None


def precondition(lp, ruiz_iters: int = 10, pock_chambolle: bool = True):
    """Diagonal preconditioner (d_r, d_c); A~ = diag(d_r) A diag(d_c)."""
    pin = _Pinned(lp)
    dr = np.empty(lp.m)
    dc = np.empty(lp.n)
    rc = _load().orc_precondition(ctypes.byref(pin.s), ruiz_iters, int(pock_chambolle), _p(dr), _p(dc))
    assert rc == 0
    return dr, dc


def kkt(lp, x, y, c=None, q=None):
    """Relative KKT of (x, y): dict with rel, rho_p, rho_d, rho_g, pobj, dobj
    (with a diagonal Hessian q: of the QP min c^T x + x^T diag(q) x / 2)."""
    pin = _Pinned(lp, c, q)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    out = np.zeros(8)
    rc = _load().orc_kkt(ctypes.byref(pin.s), _p(x), _p(y), _p(out))
    assert rc == 0
    return dict(rel=out[0], rho_p=out[1], rho_d=out[2], rho_g=out[3], pobj=out[4],
                dobj=out[5], bnorm=out[6], cnorm=out[7])


def pdhg(lp, tol: float = 1e-4, iter_limit: int = 100_000, check_period: int = 64,
         restarts: bool = True, eta: float = 0.99, x0=None, y0=None, omega0: float = 0.0,
         c=None, ruiz_iters: int = 10, pock_chambolle: bool = True,
         adaptive: bool = False, q=None, infeas_tol: float = 1e-8, stall_tol: float = 0.0,
         stall_checks: int = 3, restart_avg: bool = False) -> PDHGResult:
    """FP64 PDHG solve of the LP relaxation (Algorithm 1 inner loop); with
    `adaptive` the step size follows PDLP's adaptive rule (no retries),
    starting at `eta`.  `q`: diagonal Hessian (>= 0) of a QP objective
    c^T x + x^T diag(q) x / 2, or None.  infeas_tol > 0: stop with
    PRIMAL_INFEASIBLE / DUAL_INFEASIBLE when the moves between two checks
    certify it to that relative accuracy (0: off).  stall_tol > 0: stop with
    STALLED when neither objective bound moved by more than
    stall_tol (1 + |value|) at stall_checks consecutive checks.
    restart_avg: the running mean of the iterates since the last restart is
    a candidate at every check (the lower relative KKT error wins: the
    termination test, the restart rule and the returned point use the
    winner); the result's x_avg / y_avg hold that mean at the stop."""
    pin = _Pinned(lp, c, q)
    x = np.empty(lp.n)
    y = np.empty(lp.m)
    x0a = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
    y0a = None if y0 is None else np.ascontiguousarray(y0, dtype=np.float64)
    prm = _Params(tol, iter_limit, check_period, int(restarts), eta, ruiz_iters,
                  int(pock_chambolle), omega0, int(adaptive), infeas_tol, stall_tol, stall_checks,
                  int(restart_avg))
    res = _Result()
    xa = np.zeros(lp.n)
    ya = np.zeros(lp.m)
    rc = _load().orc_pdhg_avg(ctypes.byref(pin.s), ctypes.byref(prm), _p(x0a), _p(y0a), _p(x), _p(y),
                              _p(xa), _p(ya), ctypes.byref(res))
    assert rc == 0
    out = PDHGResult(x, y, res.status, res.iterations, res.restarts, res.rel_kkt, res.rho_p,
                     res.rho_d, res.rho_g, res.pobj, res.dobj, res.omega, res.eta)
    if restart_avg:
        out.x_avg, out.y_avg = xa, ya
    return out


def ray(lp, x, y, xp, yp, q=None):
    """Certificate quantities of the moves d = x - xp, v = y - yp:
    (rho, dual-ray residual, c^T d, primal-ray violation)."""
    pin = _Pinned(lp, None, q)
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (x, y, xp, yp)]
    out = np.zeros(4)
    rc = _load().orc_ray(ctypes.byref(pin.s), *[_p(a) for a in arrs], _p(out))
    assert rc == 0
    return tuple(out)


def fix_propagate(lp, xbar, is_int=None):
    """Fix-and-propagate rounding (Section 2.3).  Returns (x_hat, feasible,
    ignored_rows)."""
    pin = _Pinned(lp)
    is_int = np.ascontiguousarray(lp.is_int if is_int is None else is_int, dtype=np.uint8)
    xb = np.ascontiguousarray(xbar, dtype=np.float64)
    xhat = np.empty(lp.n)
    info = np.zeros(2, dtype=np.int32)
    rc = _load().orc_fix_propagate(ctypes.byref(pin.s), _p(is_int), _p(xb), _p(xhat), _p(info))
    assert rc == 0
    return xhat, bool(info[0]), int(info[1])


FP_MAX_ROUNDS = 1000


def fix_propagate_batched(lp, xbar, K: int, max_rounds: int = FP_MAX_ROUNDS, is_int=None):
    """Batched fix-and-propagate (a parallel form of Section 2.3): the next K
    unfixed integer variables of the fixing order are fixed together, then
    synchronous propagation rounds (at most max_rounds per batch) combine the
    rows' derived bounds by max / min; rows behind an empty combined domain
    are ignored.  Returns (x_hat, feasible, ignored_rows, ignored_mask)."""
    pin = _Pinned(lp)
    is_int = np.ascontiguousarray(lp.is_int if is_int is None else is_int, dtype=np.uint8)
    xb = np.ascontiguousarray(xbar, dtype=np.float64)
    xhat = np.empty(lp.n)
    info = np.zeros(2, dtype=np.int32)
    mask = np.zeros(max(lp.m, 1), dtype=np.uint8)
    rc = _load().orc_fix_propagate_batched(ctypes.byref(pin.s), _p(is_int), _p(xb), ctypes.c_int32(K),
                                           ctypes.c_int32(max_rounds), _p(xhat), _p(info), _p(mask))
    assert rc == 0
    return xhat, bool(info[0]), int(info[1]), mask[: lp.m].astype(bool)


# ------------------------------------------------ objective update (O3)
ALPHA = 0.9


def distance_gradient(xhat, l, u, is_int):
    """Coefficients g of the L1 distance Delta(x, x_hat) on binary variables:
    Delta = g^T x + sum_j x_hat_j for x in [0,1]^n, with g_j = +1 where x_hat_j
    sits at its lower bound and -1 where it sits at its upper bound; 0 on
    continuous variables.  General integers strictly inside their bounds
    would need auxiliary variables (Section 4) and are rejected."""
    g = np.zeros(len(xhat))
    ii = is_int.astype(bool)
    at_l = ii & (xhat == l)
    at_u = ii & (xhat == u) & ~at_l
    if np.any(ii & ~at_l & ~at_u):
        raise ValueError("general-integer distance needs auxiliary variables")
    g[at_l] = 1.0
    g[at_u] = -1.0
    return g


def objective_update(c, xhat, l, u, is_int, K: int, alpha: float = ALPHA):
    """Algorithm 1 objective update after the K-th rounding:
    c_hat = alpha^K * (sqrt(|I|) / ||c||_2) * c + (1 - alpha^K) * grad Delta."""
    a = alpha ** K
    nI = int(np.count_nonzero(is_int))
    cn = float(np.linalg.norm(c))
    g = distance_gradient(xhat, l, u, is_int)
    scaled = (np.sqrt(nI) / cn) * c if cn > 0 else np.zeros_like(c)
    return a * scaled + (1.0 - a) * g


def objective_update_l2(c, xhat, is_int, K: int, alpha: float = ALPHA):
    """The objective update with the L2 distance Section 5 proposes (no
    auxiliary variables for general integers): alpha^K (sqrt(|I|)/||c||) c^T x
    + (1 - alpha^K) sum_{j in I} (x_j - x_hat_j)^2, written as the QP
    objective c_hat^T x + x^T diag(q) x / 2 plus a constant: q_j =
    2 (1 - alpha^K) and c_hat_j = alpha^K kappa c_j - 2 (1 - alpha^K) x_hat_j
    on I; q_j = 0 and c_hat_j = alpha^K kappa c_j elsewhere.  Returns (c_hat, q)."""
    a = alpha ** K
    ii = is_int.astype(bool)
    nI = int(np.count_nonzero(ii))
    cn = float(np.linalg.norm(c))
    scaled = (np.sqrt(nI) / cn) * c if cn > 0 else np.zeros_like(c)
    c_hat = a * scaled - np.where(ii, 2.0 * (1.0 - a) * xhat, 0.0)
    q = np.where(ii, 2.0 * (1.0 - a), 0.0)
    return c_hat, q


def eps_schedule(K: int, eps1: float = 0.01, beta: float = 0.98, floor: float = 1e-8) -> float:
    """Section 2.2: eps(1) = 0.01, eps(K+1) = max(beta eps(K), 1e-8)."""
    e = eps1
    for _ in range(K - 1):
        e = max(beta * e, floor)
    return e


def mip_feasible(lp, x, tol: float = 1e-6) -> bool:
    """Rows within tol (1 + |b_i|), bounds within tol, integrality within tol."""
    rows = lp.row_of_entry()
    ax = np.bincount(rows, weights=lp.val * x[lp.col_idx], minlength=lp.m)
    t = tol * (1.0 + np.abs(lp.b))
    s = lp.senses
    ok = np.where(s == ord("G"), ax >= lp.b - t,
                  np.where(s == ord("L"), ax <= lp.b + t, np.abs(ax - lp.b) <= t))
    ii = lp.is_int.astype(bool)
    return bool(ok.all() and np.all(x >= lp.l - tol) and np.all(x <= lp.u + tol)
                and np.all(np.abs(x[ii] - np.round(x[ii])) <= tol))


def pump(lp, rounds: int = 20, tol: float = 1e-4, iter_limit: int = 20_000,
         xhat_sequence=None, **kw):
    """Warm-started pump rounds on one instance (Algorithm 1 outer loop with
    cycle perturbation off, every round run).  Round 1 solves with c; round
    K >= 2 solves with the blend built from the (K-1)-th rounding.  If
    ``xhat_sequence`` is given, those roundings are used instead of the
    oracle's own (open-loop replay).  Returns per-round records."""
    c_hat = lp.c.copy()
    x = y = None
    omega = 0.0
    out = []
    for K in range(1, rounds + 1):
        r = pdhg(lp, tol=tol, iter_limit=iter_limit, x0=x, y0=y, omega0=omega, c=c_hat, **kw)
        x, y, omega = r.x, r.y, r.omega
        xhat, feas, ign = fix_propagate(lp, r.x)
        if xhat_sequence is not None:
            xhat = xhat_sequence[K - 1]
            feas = mip_feasible(lp, xhat)
        out.append(dict(K=K, status=r.status, iterations=r.iterations, rel_kkt=r.rel_kkt,
                        x=r.x, y=r.y, omega=r.omega, lp_mip_feasible=mip_feasible(lp, r.x),
                        xhat=xhat, xhat_feasible=feas, ignored=ign,
                        obj=float(lp.c @ xhat)))
        c_hat = objective_update(lp.c, xhat, lp.l, lp.u, lp.is_int, K)
    return out


# ------------------------------------------------- Algorithm 1 outer loop
_MASK64 = (1 << 64) - 1


def splitmix64(seed: int, counter: int) -> int:
    """SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the output for the
    state seed + (counter + 1) * golden gamma.  The perturbation draws its
    random numbers from this counter-based generator so that independent
    implementations draw the same numbers."""
    z = (seed + (counter + 1) * 0x9E3779B97F4A7C15) & _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def perturb_count(seed: int, instance: int, K: int) -> int:
    """Number of variables the K-th perturbation of an instance flips:
    T = 10 + (splitmix64(seed, instance * 2^20 + K) mod 21), in [10, 30]."""
    return 10 + splitmix64(seed, instance * 1048576 + K) % 21


def perturb(lp, xbar, xhat, T):
    """Cycle perturbation (Algorithm 1; Section 2.3 following the 2005
    feasibility pump): flip the T binary variables with the largest
    |x_bar_j - x_hat_j| (ties by index) to their other bound."""
    ii = np.flatnonzero(lp.is_int.astype(bool))
    if np.any((lp.u[ii] - lp.l[ii]) != 1.0):
        raise ValueError("perturbation is defined here for binary variables only")
    d = np.abs(xbar[ii] - xhat[ii])
    order = np.lexsort((ii, -d))[: min(T, ii.size)]
    out = xhat.copy()
    j = ii[order]
    out[j] = np.where(out[j] == lp.l[j], lp.u[j], lp.l[j])
    return out


def scylla(lp, rounds: int = 20, eps_sched: bool = True, tol: float = 1e-4, iter_limit: int = 100_000,
           total_iter_limit: int = 0, early_exit: bool = True, cycle_perturb: bool = True, seed: int = 0,
           instance: int = 0, alpha: float = ALPHA, distance: str = "l1", fp_batch: int = 0,
           fp_max_rounds: int = FP_MAX_ROUNDS, **kw):
    """Algorithm 1 on one instance.  Round K solves the LP relaxation with the
    current objective to tolerance eps(K) (Section 2.2; `tol` if eps_sched
    is off), warm-started from the previous round, with at most iter_limit
    iterations and, if total_iter_limit > 0, at most what remains of the
    cumulative budget (no budget left: the loop ends).  The first round whose
    PDHG iterate, else whose rounding, is MIP-feasible is the find; with
    early_exit the loop returns there.  A rounding equal to an earlier one
    (history of roundings as used, i.e. after perturbation) is perturbed; the
    objective is then updated with alpha^K from the rounding as used, with
    the L1 distance, or with distance="l2" the L2 distance (a QP solve from
    round 2 on).  Rounding: fix_propagate, or with fp_batch = K > 0
    fix_propagate_batched(K, fp_max_rounds).
    Returns (found_kind, found_round, point, records): found_kind 0 (none),
    1 (PDHG iterate), 2 (rounding); point is the find, else the last
    rounding before perturbation (None if no round ran)."""
    if distance not in ("l1", "l2"):
        raise ValueError("distance must be 'l1' or 'l2'")
    c_hat = lp.c.copy()
    q_hat = None
    x = y = None
    omega = 0.0
    history = []
    used = 0
    recs = []
    kind, found_K, point = 0, 0, None
    for K in range(1, rounds + 1):
        lim = iter_limit
        if total_iter_limit > 0:
            lim = min(lim, total_iter_limit - used)
        if lim <= 0:
            break
        tk = eps_schedule(K) if eps_sched else tol
        r = pdhg(lp, tol=tk, iter_limit=lim, x0=x, y0=y, omega0=omega, c=c_hat, q=q_hat, **kw)
        used += r.iterations
        x, y, omega = r.x, r.y, r.omega
        rec = dict(K=K, tol=tk, status=r.status, iterations=r.iterations, rel_kkt=r.rel_kkt,
                   lp_mip_feasible=mip_feasible(lp, r.x), perturbed=False, x=r.x)
        recs.append(rec)
        if rec["lp_mip_feasible"] and not kind:
            kind, found_K, point = 1, K, r.x
            if early_exit:
                break
        if fp_batch > 0:
            xhat, feas, ign, _ = fix_propagate_batched(lp, r.x, fp_batch, fp_max_rounds)
        else:
            xhat, feas, ign = fix_propagate(lp, r.x)
        rec.update(xhat=xhat, xhat_feasible=feas, ignored=ign, obj=float(lp.c @ xhat))
        if not kind:
            point = xhat
            if feas:
                kind, found_K = 2, K
                if early_exit:
                    break
        if cycle_perturb:
            if any(np.array_equal(xhat, h) for h in history):
                xhat = perturb(lp, r.x, xhat, perturb_count(seed, instance, K))
                rec["perturbed"] = True
            history.append(xhat)
        rec["xhat_used"] = xhat
        if K < rounds:
            if distance == "l1":
                c_hat = objective_update(lp.c, xhat, lp.l, lp.u, lp.is_int, K, alpha)
            else:
                c_hat, q_hat = objective_update_l2(lp.c, xhat, lp.is_int, K, alpha)
    return kind, found_K, point, recs
