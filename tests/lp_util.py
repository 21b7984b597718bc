"""Test-side helpers: dense <-> CSR, brute-force vertex enumeration, HiGHS
reference solves and an independent (vectorised) KKT evaluator.  None of this
is used by the library."""
from __future__ import annotations

import itertools
import json
import os

import numpy as np
import scipy.sparse as sps
from scipy.optimize import linprog

from paper_2307_03466_amd.instances import LP

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def lp_from_dense(A, b, senses, c, l, u, is_int=None, name="dense"):
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    rows, cols = np.nonzero(A)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=m), out=row_ptr[1:])
    if isinstance(senses, str):
        senses = np.frombuffer(senses.encode(), dtype=np.uint8).copy()
    return LP(m=m, n=n, row_ptr=row_ptr, col_idx=cols.astype(np.int32),
              val=A[rows, cols].astype(np.float64), c=np.asarray(c, dtype=np.float64),
              b=np.asarray(b, dtype=np.float64), senses=np.asarray(senses, dtype=np.uint8),
              l=np.asarray(l, dtype=np.float64), u=np.asarray(u, dtype=np.float64),
              is_int=np.zeros(n, dtype=np.uint8) if is_int is None else np.asarray(is_int, np.uint8),
              name=name)


def dense(lp):
    return sps.csr_matrix((lp.val, lp.col_idx, lp.row_ptr), shape=(lp.m, lp.n)).toarray()


def csr(lp):
    return sps.csr_matrix((lp.val, lp.col_idx, lp.row_ptr), shape=(lp.m, lp.n))


def load_wyndor():
    with open(os.path.join(GOLDEN, "wyndor_lp.json")) as f:
        d = json.load(f)
    A = np.zeros((d["m"], d["n"]))
    for i, row in enumerate(d["rows"]):
        for j, v in row:
            A[i, j] = v
    u = [float(v) for v in d["u"]]
    return lp_from_dense(A, d["b"], d["senses"], d["c"], d["l"], u, name="wyndor"), d


def highs(lp, c=None):
    """Optimal value (and solution) of the LP by scipy's HiGHS."""
    A = csr(lp)
    s = lp.senses
    G, L, E = A[s == ord("G")], A[s == ord("L")], A[s == ord("E")]
    Aub = sps.vstack([-G, L]).tocsr()
    bub = np.concatenate([-lp.b[s == ord("G")], lp.b[s == ord("L")]])
    kw = {}
    if Aub.shape[0]:
        kw.update(A_ub=Aub, b_ub=bub)
    if E.shape[0]:
        kw.update(A_eq=E, b_eq=lp.b[s == ord("E")])
    bounds = [(None if np.isinf(a) else a, None if np.isinf(b_) else b_) for a, b_ in zip(lp.l, lp.u)]
    r = linprog(lp.c if c is None else c, bounds=bounds, method="highs", **kw)
    assert r.status == 0, r.message
    return r


def brute_force_lp(lp):
    """Minimum of c^T x over the vertices of {rows, l <= x <= u} (all bounds
    finite): every choice of n constraints (rows or bounds) taken as active,
    solved as a square system; singular or infeasible choices are skipped.
    A bounded nonempty polyhedron attains its minimum at such a vertex."""
    A = dense(lp)
    m, n = A.shape
    assert np.all(np.isfinite(lp.l)) and np.all(np.isfinite(lp.u))
    cons = []  # (row vector, rhs, kind)
    for i in range(m):
        cons.append((A[i], lp.b[i], chr(lp.senses[i])))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        cons.append((e, lp.l[j], "lb"))
        cons.append((e, lp.u[j], "ub"))
    best, best_x = np.inf, None
    for idx in itertools.combinations(range(len(cons)), n):
        M = np.array([cons[k][0] for k in idx])
        r = np.array([cons[k][1] for k in idx])
        if abs(np.linalg.det(M)) < 1e-9:
            continue
        x = np.linalg.solve(M, r)
        ax = A @ x
        tol = 1e-9
        ok = np.all(x >= lp.l - tol) and np.all(x <= lp.u + tol)
        s = lp.senses
        ok = ok and np.all(np.where(s == ord("G"), ax >= lp.b - tol,
                                    np.where(s == ord("L"), ax <= lp.b + tol,
                                             np.abs(ax - lp.b) <= tol)))
        if ok:
            v = lp.c @ x
            if v < best:
                best, best_x = v, x
    return best, best_x


def kkt_numpy(lp, x, y, c=None, q=None):
    """Relative KKT errors from the formulas, vectorised with scipy.sparse
    (independent of the C oracle); q: diagonal Hessian of a QP objective
    c^T x + x^T diag(q) x / 2 (its dual objective at the same x subtracts
    x^T diag(q) x / 2)."""
    c = lp.c if c is None else c
    qx = np.zeros(lp.n) if q is None else np.asarray(q) * x
    A = csr(lp)
    ax = A @ x
    aty = A.T @ y
    s = lp.senses
    rp = np.where(s == ord("G"), np.maximum(lp.b - ax, 0),
                  np.where(s == ord("L"), np.maximum(ax - lp.b, 0), lp.b - ax))
    g = c + qx - aty
    lf, uf = np.isfinite(lp.l), np.isfinite(lp.u)
    lam = np.where(lf & uf, g, np.where(lf, np.maximum(g, 0), np.where(uf, np.minimum(g, 0), 0.0)))
    rd = g - lam
    P = c @ x + 0.5 * (qx @ x)
    D = lp.b @ y + np.sum(np.where(lf, lp.l, 0) * np.maximum(lam, 0)) \
        - np.sum(np.where(uf, lp.u, 0) * np.maximum(-lam, 0)) - 0.5 * (qx @ x)
    rho_p = np.linalg.norm(rp) / (1 + np.linalg.norm(lp.b))
    rho_d = np.linalg.norm(rd) / (1 + np.linalg.norm(c))
    rho_g = abs(P - D) / (1 + abs(P) + abs(D))
    return dict(rel=max(rho_p, rho_d, rho_g), rho_p=rho_p, rho_d=rho_d, rho_g=rho_g, pobj=P, dobj=D)


def rel_err(a, ref):
    return float(np.linalg.norm(np.asarray(a, np.float64) - ref) / max(1.0, np.linalg.norm(ref)))


def elem_err(a, ref):
    """Largest per-entry error max_i |a_i - ref_i| / (1 + |ref_i|) (0 for empty vectors)."""
    a = np.asarray(a, np.float64)
    ref = np.asarray(ref, np.float64)
    if ref.size == 0:
        return 0.0
    return float(np.max(np.abs(a - ref) / (1.0 + np.abs(ref))))


def parity_err(x, y, ref_x, ref_y):
    """Larger of the vector error rel_err and the per-entry error elem_err
    over both iterates: a fixed-iteration parity bar applies to both."""
    return max(rel_err(x, ref_x), rel_err(y, ref_y), elem_err(x, ref_x), elem_err(y, ref_y))
