"""Seeded synthetic LP / MIP instances.

This module only draws random instances; it contains none of the solver's
arithmetic (no preconditioning, no PDHG step, no residuals).  Both the HIP
path and the plain CPU checker consume its output, which keeps the two
implementations independent of each other.

The paper evaluates on MIPLIB 2017 and the Fischetti-Salvagnin 2009 set
(Section 3); those instances are not available here, so five synthetic
families of the same problem form (Algorithm 1 input: min c^T x subject to
row constraints, box bounds and integrality) stand in for them:

* ``set_cover``      - 0/1 covering rows  ``A x >= 1``, binary variables.
* ``general_lp``     - integer coefficients in [-20, 20] \\ {0}, geometric row
                       lengths, mixed >= / = rows, feasible by construction.
* ``skewed_lp``      - power-law row lengths (exponent 1.8, max 50 000), 70 %
                       0/1 rows and 30 % rows with integers in [-127, 127].
* ``cover_knapsack`` - binary problems mixing covering rows and knapsack rows
                       (weights 1..100, capacity 0.3 x row sum).

Every instance carries a feasibility certificate ``x_star``.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

SEED_BASE = 2307034660


@dataclasses.dataclass
class LP:
    """An LP relaxation in CSR form: min c^T x, A x (sense) b, l <= x <= u."""

    m: int
    n: int
    row_ptr: np.ndarray  # int64 [m+1]
    col_idx: np.ndarray  # int32 [nnz], strictly increasing within each row
    val: np.ndarray      # float64 [nnz]
    c: np.ndarray        # float64 [n]
    b: np.ndarray        # float64 [m]
    senses: np.ndarray   # uint8 [m] of ord('G'), ord('L'), ord('E')
    l: np.ndarray        # float64 [n]
    u: np.ndarray        # float64 [n]
    is_int: np.ndarray   # uint8 [n]
    x_star: Optional[np.ndarray] = None  # a feasible point (certificate)
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def row_of_entry(self) -> np.ndarray:
        return np.repeat(np.arange(self.m, dtype=np.int64), np.diff(self.row_ptr))


def config_seed(k: int) -> int:
    """Seed of workload family k (1-based numbering of the five workloads)."""
    return SEED_BASE + k


def _csr_from_pairs(m: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray):
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    counts = np.bincount(rows, minlength=m)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return row_ptr, cols.astype(np.int32), vals.astype(np.float64)


def _distinct_per_group(rng, group_len: np.ndarray, universe: int) -> tuple:
    """For each group g draw group_len[g] distinct uniform integers in
    [0, universe).  Returns (group_id, value) sorted by (group, value)."""
    group_len = np.asarray(group_len, dtype=np.int64)
    if np.any(group_len > universe):
        raise ValueError("group longer than universe")
    dense = np.flatnonzero(group_len * 8 > universe)
    if dense.size:
        # long groups: draw without replacement directly
        light = group_len.copy()
        light[dense] = 0
        g0, v0 = _distinct_per_group(rng, light, universe)
        gd = [np.full(group_len[d], d, dtype=np.int64) for d in dense]
        vd = [np.sort(rng.choice(universe, size=int(group_len[d]), replace=False)) for d in dense]
        gid = np.concatenate([g0] + gd)
        val = np.concatenate([v0] + vd)
        order = np.lexsort((val, gid))
        return gid[order], val[order]
    gid = np.repeat(np.arange(group_len.size, dtype=np.int64), group_len)
    val = rng.integers(0, universe, size=gid.size, dtype=np.int64)
    for _ in range(200):
        key = gid * universe + val
        order = np.argsort(key, kind="stable")
        key_s = key[order]
        dup = np.zeros(key_s.size, dtype=bool)
        dup[1:] = key_s[1:] == key_s[:-1]
        if not dup.any():
            return gid[order], val[order]
        gid_s = gid[order]
        val_s = val[order]
        keep = ~dup
        missing = np.bincount(gid_s[dup], minlength=group_len.size)
        new_gid = np.repeat(np.arange(group_len.size, dtype=np.int64), missing)
        new_val = rng.integers(0, universe, size=new_gid.size, dtype=np.int64)
        gid = np.concatenate([gid_s[keep], new_gid])
        val = np.concatenate([val_s[keep], new_val])
    raise RuntimeError("could not draw distinct entries")


# ---------------------------------------------------------------- set cover
def set_cover(m: int = 200, n: int = 500, seed: int | np.random.SeedSequence = None,
              name: str = "set_cover") -> LP:
    """Covering LP: every column hits U{3..8} distinct uniform rows with
    coefficient 1; c_j ~ U{1..100}; A x >= 1; 0 <= x <= 1; all integer.
    Rows left empty get one random column (otherwise infeasible)."""
    rng = np.random.default_rng(config_seed(1) if seed is None else seed)
    deg = rng.integers(3, 9, size=n)
    deg = np.minimum(deg, m)
    col, row = _distinct_per_group(rng, deg, m)
    hit = np.bincount(row, minlength=m)
    empty = np.flatnonzero(hit == 0)
    if empty.size:
        extra = rng.integers(0, n, size=empty.size)
        row = np.concatenate([row, empty])
        col = np.concatenate([col, extra])
    vals = np.ones(row.size)
    row_ptr, col_idx, val = _csr_from_pairs(m, row, col, vals)
    c = rng.integers(1, 101, size=n).astype(np.float64)
    return LP(m=m, n=n, row_ptr=row_ptr, col_idx=col_idx, val=val, c=c,
              b=np.ones(m), senses=np.full(m, ord("G"), dtype=np.uint8),
              l=np.zeros(n), u=np.ones(n), is_int=np.ones(n, dtype=np.uint8),
              x_star=np.ones(n), name=name)


# ------------------------------------------------------ general / skewed LP
def _bounds_and_point(rng, n):
    code = rng.integers(0, 3, size=n)
    u = np.where(code == 0, 1.0, np.where(code == 1, 10.0, np.inf))
    l = np.zeros(n)
    x_star = rng.random(n) * np.where(np.isinf(u), 10.0, u)
    return l, u, x_star


def _rhs(rng, row_ptr, col_idx, val, x_star, senses):
    m = row_ptr.size - 1
    rows = np.repeat(np.arange(m), np.diff(row_ptr))
    ax = np.bincount(rows, weights=val * x_star[col_idx], minlength=m)
    slack = rng.exponential(1.0, size=m)
    b = ax.copy()
    g = senses == ord("G")
    lt = senses == ord("L")
    b[g] -= slack[g]
    b[lt] += slack[lt]
    return b


def general_lp(m: int = 1_000_000, n: int = 2_000_000,
               seed: int | np.random.SeedSequence = None, name: str = "general_lp") -> LP:
    """General LP: geometric(p=0.1) row lengths (mean 10), distinct uniform
    columns, a_ij uniform on {-20..20}\\{0}; l = 0, u in {1, 10, inf}
    (1/3 each); x* ~ U[0, u] (U[0, 10] for u = inf); 20 % equality rows
    b = A x*, 80 % >= rows b = A x* - s, s ~ Exp(1); c ~ N(0, 1) with
    c_j := |c_j| on columns without upper bound (keeps the LP bounded)."""
    rng = np.random.default_rng(config_seed(2) if seed is None else seed)
    lens = np.minimum(rng.geometric(0.1, size=m), n)
    row, col = _distinct_per_group(rng, lens, n)
    mag = rng.integers(1, 21, size=row.size)
    sign = np.where(rng.random(row.size) < 0.5, -1, 1)
    vals = (mag * sign).astype(np.float64)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(row, minlength=m), out=row_ptr[1:])
    col_idx = col.astype(np.int32)
    l, u, x_star = _bounds_and_point(rng, n)
    senses = np.where(rng.random(m) < 0.2, ord("E"), ord("G")).astype(np.uint8)
    b = _rhs(rng, row_ptr, col_idx, vals, x_star, senses)
    c = rng.standard_normal(n)
    c = np.where(np.isinf(u), np.abs(c), c)
    return LP(m=m, n=n, row_ptr=row_ptr, col_idx=col_idx, val=vals, c=c, b=b,
              senses=senses, l=l, u=u, is_int=np.zeros(n, dtype=np.uint8),
              x_star=x_star, name=name)


def powerlaw_lengths(rng, m: int, nnz: int, alpha: float = 1.8, kmax: int = 50_000) -> np.ndarray:
    """Row lengths with P(k) ~ k^-alpha on [1, kmax], rescaled to sum to nnz
    exactly (stochastic rounding, clamp, then +-1 fix-ups on random rows)."""
    k = np.arange(1, kmax + 1, dtype=np.float64)
    p = k ** (-alpha)
    p /= p.sum()
    raw = rng.choice(kmax, size=m, p=p).astype(np.float64) + 1.0
    scaled = raw * (nnz / raw.sum())
    lo = np.floor(scaled)
    lens = lo + (rng.random(m) < (scaled - lo))
    lens = np.clip(lens, 1, kmax).astype(np.int64)
    diff = int(nnz - lens.sum())
    while diff != 0:
        if diff > 0:
            cand = np.flatnonzero(lens < kmax)
            pick = rng.choice(cand, size=min(diff, cand.size), replace=False)
            lens[pick] += 1
        else:
            cand = np.flatnonzero(lens > 1)
            pick = rng.choice(cand, size=min(-diff, cand.size), replace=False)
            lens[pick] -= 1
        diff = int(nnz - lens.sum())
    return lens


def skewed_lp(m: int = 500_000, n: int = 1_000_000, nnz: int = 20_000_000,
              seed: int | np.random.SeedSequence = None, kmax: int = 50_000,
              name: str = "skewed_lp") -> LP:
    """Skewed LP: power-law row lengths (alpha 1.8, max kmax), distinct uniform
    columns; 70 % of rows 0/1 pattern rows, 30 % integers uniform on
    [-127, 127]\\{0}; senses 40 % >=, 40 % <=, 20 % =; bounds, x*, b, c as in
    ``general_lp`` (<= rows: b = A x* + s)."""
    rng = np.random.default_rng(config_seed(3) if seed is None else seed)
    kmax = min(kmax, n)
    lens = powerlaw_lengths(rng, m, nnz, kmax=kmax)
    row, col = _distinct_per_group(rng, lens, n)
    pattern_row = rng.random(m) < 0.7
    mag = rng.integers(1, 128, size=row.size)
    sign = np.where(rng.random(row.size) < 0.5, -1, 1)
    vals = np.where(pattern_row[row], 1, mag * sign).astype(np.float64)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(lens, out=row_ptr[1:])
    col_idx = col.astype(np.int32)
    l, u, x_star = _bounds_and_point(rng, n)
    r = rng.random(m)
    senses = np.where(r < 0.4, ord("G"), np.where(r < 0.8, ord("L"), ord("E"))).astype(np.uint8)
    b = _rhs(rng, row_ptr, col_idx, vals, x_star, senses)
    c = rng.standard_normal(n)
    c = np.where(np.isinf(u), np.abs(c), c)
    return LP(m=m, n=n, row_ptr=row_ptr, col_idx=col_idx, val=vals, c=c, b=b,
              senses=senses, l=l, u=u, is_int=np.zeros(n, dtype=np.uint8),
              x_star=x_star, name=name)


# ------------------------------------------------------ cover / knapsack
def cover_knapsack(m: int, n: Optional[int] = None, seed=None,
                   name: str = "cover_knapsack", umax: int = 1) -> LP:
    """Binary MIP relaxation: each column hits U{3..8} distinct rows; each row
    is a covering row (p = 1/2; coefficients 1, A_i x >= 1) or a knapsack row
    (weights U{1..100}, A_i x <= 0.3 * sum_j a_ij); c_j ~ U{1..100};
    0 <= x <= 1, all integer.  Covering rows with fewer than 4 entries get
    extra random columns, so x = 0.3 * 1 is feasible."""
    n = 2 * m if n is None else n
    rng = np.random.default_rng(seed)
    deg = np.minimum(rng.integers(3, 9, size=n), m)
    col, row = _distinct_per_group(rng, deg, m)
    cover = rng.random(m) < 0.5
    cnt = np.bincount(row, minlength=m)
    short = np.flatnonzero(cover & (cnt < 4))
    if short.size:
        need = 4 - cnt[short]
        # draw replacement sets of 4 distinct columns, keep those not present
        add_rows, add_cols = [], []
        present = set(zip(row[np.isin(row, short)].tolist(), col[np.isin(row, short)].tolist()))
        for r_, k_ in zip(short.tolist(), need.tolist()):
            got = 0
            while got < k_:
                cc = int(rng.integers(0, n))
                if (r_, cc) not in present:
                    present.add((r_, cc))
                    add_rows.append(r_)
                    add_cols.append(cc)
                    got += 1
        row = np.concatenate([row, np.array(add_rows, dtype=np.int64)])
        col = np.concatenate([col, np.array(add_cols, dtype=np.int64)])
    weights = rng.integers(1, 101, size=row.size).astype(np.float64)
    vals = np.where(cover[row], 1.0, weights)
    row_ptr, col_idx, val = _csr_from_pairs(m, row, col, vals)
    rows = np.repeat(np.arange(m), np.diff(row_ptr))
    rowsum = np.bincount(rows, weights=val, minlength=m)
    b = np.where(cover, 1.0, 0.3 * rowsum)
    senses = np.where(cover, ord("G"), ord("L")).astype(np.uint8)
    c = rng.integers(1, 101, size=n).astype(np.float64)
    u = np.ones(n)
    if umax > 1:  # general integers (int_cover_knapsack)
        u = rng.integers(2, umax + 1, size=n).astype(np.float64)
        usum = np.bincount(rows, weights=u[col_idx], minlength=m)
        wusum = np.bincount(rows, weights=val * u[col_idx], minlength=m)
        b = np.where(cover, np.maximum(1.0, np.floor(0.3 * usum)), 0.3 * wusum)
    return LP(m=m, n=n, row_ptr=row_ptr, col_idx=col_idx, val=val, c=c, b=b,
              senses=senses, l=np.zeros(n), u=u,
              is_int=np.ones(n, dtype=np.uint8), x_star=0.3 * u, name=name)


def int_cover_knapsack(m: int, n: Optional[int] = None, seed=None, umax: int = 5,
                       name: str = "int_cover_knapsack") -> LP:
    """General-integer version of cover_knapsack: x_j in {0..u_j},
    u_j ~ U{2..umax}; covering rows sum_j x_j >= max(1, floor(0.3 sum_j u_j)),
    knapsack rows sum_j w_j x_j <= 0.3 sum_j w_j u_j; x = 0.3 u is feasible."""
    return cover_knapsack(m, n, seed=seed, name=name, umax=umax)


def int_pump_batch(count: int = 64, m: int = 5_000, n: int = 10_000, seed=None) -> List[LP]:
    """Batch of general-integer cover/knapsack instances (L2-distance loop)."""
    s = config_seed(6) if seed is None else seed
    kids = np.random.SeedSequence(s).spawn(count)
    return [int_cover_knapsack(m, n, seed=kids[i], name=f"ipump{i}") for i in range(count)]


def set_partition(m: int = 30, n: int = 120, seed=None, name: str = "set_partition") -> LP:
    """Set-partitioning MIP (A x = 1, x binary), the equality-constrained
    class on which rounding-based heuristics cycle.  A planted partition of
    the rows into blocks of U{1..4} rows, one column per block, keeps it
    feasible; the other columns hit U{2..8} distinct uniform rows; the
    columns are shuffled; c_j ~ U{1..19}."""
    rng = np.random.default_rng(config_seed(6) if seed is None else seed)
    perm = rng.permutation(m)
    sizes = []
    while sum(sizes) < m:
        sizes.append(int(min(rng.integers(1, 5), m - sum(sizes))))
    planted = np.split(perm, np.cumsum(sizes)[:-1])
    if len(planted) > n:
        raise ValueError("n is too small for the planted partition")
    cols = [np.sort(g) for g in planted]
    for _ in range(n - len(planted)):
        cols.append(np.sort(rng.choice(m, size=int(min(rng.integers(2, 9), m)), replace=False)))
    order = rng.permutation(n)
    cols = [cols[j] for j in order]
    col = np.concatenate([np.full(len(r), j) for j, r in enumerate(cols)])
    row = np.concatenate(cols)
    row_ptr, col_idx, val = _csr_from_pairs(m, row, col, np.ones(row.size))
    x_star = np.zeros(n)
    x_star[np.argsort(order)[: len(planted)]] = 1.0
    return LP(m=m, n=n, row_ptr=row_ptr, col_idx=col_idx, val=val,
              c=rng.integers(1, 20, size=n).astype(np.float64), b=np.ones(m),
              senses=np.full(m, ord("E"), dtype=np.uint8), l=np.zeros(n), u=np.ones(n),
              is_int=np.ones(n, dtype=np.uint8), x_star=x_star, name=name)


def batch_sizes(count: int = 256, lo: int = 1_000, hi: int = 50_000, seed=None) -> np.ndarray:
    """Row counts m_i = round(exp(U[ln lo, ln hi]))."""
    rng = np.random.default_rng(config_seed(4) if seed is None else seed)
    return np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), size=count))).astype(np.int64)


def uneven_batch(count: int = 256, lo: int = 1_000, hi: int = 50_000, seed=None) -> List[LP]:
    """Batch of cover/knapsack LPs with log-uniform row counts, n_i = 2 m_i."""
    s = config_seed(4) if seed is None else seed
    ms = batch_sizes(count, lo, hi, seed=s)
    kids = np.random.SeedSequence(s).spawn(count)
    return [cover_knapsack(int(mi), seed=kids[i], name=f"batch{i}") for i, mi in enumerate(ms)]


def pump_batch(count: int = 64, m: int = 20_000, n: int = 40_000, seed=None) -> List[LP]:
    """Batch of equal-size cover/knapsack instances for the pump re-solve loop."""
    s = config_seed(5) if seed is None else seed
    kids = np.random.SeedSequence(s).spawn(count)
    return [cover_knapsack(m, n, seed=kids[i], name=f"pump{i}") for i in range(count)]


def tiny_lp(rng, m: int, n: int, density: float = 0.6, lo: int = -5, hi: int = 5,
            bounded: bool = True) -> LP:
    """Small random LP with integer data, feasible by construction (used for
    brute-force checks).  Senses are mixed; bounds finite when ``bounded``."""
    mask = rng.random((m, n)) < density
    vals = rng.integers(lo, hi + 1, size=(m, n)) * mask
    rows, cols = np.nonzero(vals)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=m), out=row_ptr[1:])
    l = -rng.integers(0, 3, size=n).astype(np.float64)
    u = l + rng.integers(1, 4, size=n)
    kind = rng.random(n) if not bounded else np.ones(n)
    # unbounded variants: 30 % no upper bound, 20 % no lower bound, 10 % free
    no_u = kind < 0.3
    no_l = (kind >= 0.3) & (kind < 0.5)
    free = (kind >= 0.5) & (kind < 0.6)
    x_star = l + rng.random(n) * (u - l)
    u = np.where(no_u | free, np.inf, u)
    l = np.where(no_l | free, -np.inf, l)
    senses = rng.choice(np.array([ord("G"), ord("L"), ord("E")], dtype=np.uint8), size=m,
                        p=[0.45, 0.35, 0.2])
    ax = vals @ x_star
    slack = rng.integers(0, 3, size=m).astype(np.float64)
    b = np.where(senses == ord("G"), np.floor(ax) - slack,
                 np.where(senses == ord("L"), np.ceil(ax) + slack, ax))
    c = rng.integers(-6, 7, size=n).astype(np.float64)
    if not bounded:
        # keep the LP bounded below: c >= 1 where only l is finite, c <= -1
        # where only u is finite, c = 0 on free variables
        c = np.where(no_u, np.abs(c) + 1, np.where(no_l, -np.abs(c) - 1, np.where(free, 0.0, c)))
    return LP(m=m, n=n, row_ptr=row_ptr, col_idx=cols.astype(np.int32),
              val=vals[rows, cols].astype(np.float64), c=c, b=b, senses=senses, l=l, u=u,
              is_int=np.zeros(n, dtype=np.uint8), x_star=x_star, name="tiny")


def workload(k: int, scale: float = 1.0):
    """Workload k (1..5) at full size (scale = 1) or scaled down.  Returns an
    LP (k = 1, 2, 3) or a list of LPs (k = 4, 5)."""
    if k == 1:
        return set_cover(200, 500, seed=config_seed(1), name="set_cover_200x500")
    if k == 2:
        m = max(8, int(round(1_000_000 * scale)))
        return general_lp(m, 2 * m, seed=config_seed(2), name=f"general_lp_{m}x{2*m}")
    if k == 3:
        m = max(8, int(round(500_000 * scale)))
        nnz = max(4 * m, int(round(20_000_000 * scale)))
        kmax = max(2, min(50_000, int(round(50_000 * min(1.0, scale * 20)))))
        return skewed_lp(m, 2 * m, nnz, seed=config_seed(3), kmax=kmax,
                         name=f"skewed_lp_{m}x{2*m}")
    if k == 4:
        count = max(1, int(round(256 * min(1.0, scale * 4))))
        hi = max(1_000, int(round(50_000 * min(1.0, scale))))
        lo = min(1_000, hi)
        return uneven_batch(count, lo, hi, seed=config_seed(4))
    if k == 5:
        count = max(1, int(round(64 * min(1.0, scale * 4))))
        m = max(100, int(round(20_000 * scale)))
        return pump_batch(count, m, 2 * m, seed=config_seed(5))
    raise ValueError(k)
