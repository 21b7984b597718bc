"""Edge cases of the device path against the oracle: no constraints, empty
rows and columns, one variable, rows whose lengths sit exactly on tile and
segment boundaries (every layout), instances without rows inside a batch,
free variables, equality-only LPs."""
import numpy as np
import pytest

import oracle
from paper_2307_03466_amd import instances as I
from lp_util import lp_from_dense, parity_err, rel_err

pytestmark = pytest.mark.gpu
pdhg = pytest.importorskip("paper_2307_03466_amd.pdhg")

LAYOUTS = [(0, 4, 0, 4), (0, 16, 0, 16), (4, 8, 8, 4), (2, 8, 2, 16), (-1, 8, -1, 8), (0, -16, 4, -16)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    pdhg.lib()


def _lp_rows(lengths, n, seed, sense="G"):
    """LP whose row i has exactly lengths[i] nonzeros (distinct columns),
    integer coefficients, feasible at x* = 0.5."""
    rng = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    for i, k in enumerate(lengths):
        c = np.sort(rng.choice(n, size=k, replace=False))
        rows += [i] * k
        cols += c.tolist()
        vals += rng.integers(1, 5, size=k).tolist()
    m = len(lengths)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(np.array(rows, dtype=np.int64), minlength=m), out=row_ptr[1:])
    val = np.array(vals, dtype=np.float64)
    col = np.array(cols, dtype=np.int32)
    ax = np.bincount(np.array(rows), weights=val * 0.5, minlength=m)
    b = ax - 1.0 if sense == "G" else ax + 1.0
    return I.LP(m=m, n=n, row_ptr=row_ptr, col_idx=col, val=val, c=rng.integers(1, 9, size=n).astype(float),
                b=b, senses=np.full(m, ord(sense), dtype=np.uint8), l=np.zeros(n), u=np.ones(n),
                is_int=np.zeros(n, dtype=np.uint8))


def _check100(lp, prec, layout=None, fused=1):
    ref = oracle.pdhg(lp, tol=-1.0, iter_limit=100, restarts=False)
    with pdhg.Batch([lp], precision=prec) as b:
        if layout:
            b.set_layout(*layout)
        r = b.solve(tol=1e-300, iter_limit=100, restarts=0, fused_window=fused, autotune=0)[0]
        x, y = b.solution(0)
    bar = 1e-10 if prec == 0 else 1e-4
    assert r["iterations"] == 100
    assert parity_err(x, y, ref.x, ref.y) <= bar
    k = oracle.kkt(lp, x, y)
    assert abs(r["rel_kkt"] - k["rel"]) <= 1e-9 * max(1, k["rel"])


@pytest.mark.parametrize("prec", [0, 1])
def test_no_constraints(prec):
    n = 37
    rng = np.random.default_rng(1)
    c = rng.normal(size=n)
    l, u = -rng.random(n), rng.random(n) + 0.2
    lp = lp_from_dense(np.zeros((0, n)), [], "", c, l, u)
    s = pdhg.solve(lp, tol=1e-9, iter_limit=100_000, precision=prec)
    assert s.result["status"] == pdhg.OPTIMAL
    np.testing.assert_allclose(s.x, np.where(c > 0, l, u), atol=1e-6)
    assert s.y.size == 0


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("fused", [1, 0])
def test_empty_rows_and_columns(prec, fused):
    A = np.zeros((6, 9))
    A[1, [0, 2, 5]] = [1, 2, 3]
    A[4, [2, 3]] = [1, -1]
    lp = lp_from_dense(A, [-1, 1.0, 0, -2, 0.5, 3], "GGLGEL", np.arange(9) - 4.0, -np.ones(9), 2 * np.ones(9))
    _check100(lp, prec, fused=fused)
    s = pdhg.solve(lp, tol=1e-8, iter_limit=500_000, precision=prec, fused_window=fused)
    assert oracle.kkt(lp, s.x, s.y)["rel"] <= 1e-8 * 1.0001


@pytest.mark.parametrize("prec", [0, 1])
def test_single_variable(prec):
    lp = lp_from_dense(np.array([[2.0], [1.0]]), [1.0, 3.0], "GL", [1.0], [0.0], [10.0])
    tol = 1e-9 if prec == 0 else 1e-6  # FP32 iterates carry ~1e-7 rounding
    s = pdhg.solve(lp, tol=tol, iter_limit=200_000, precision=prec)
    assert s.result["status"] == pdhg.OPTIMAL
    assert abs(s.x[0] - 0.5) < 10 * tol


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("prec", [0, 1])
def test_rows_on_tile_boundaries(layout, prec):
    """Row lengths at 1, chunk - 1, chunk, chunk + 1 and multiples of the
    tile sizes 1024 / 2048 / 4096 / 8192 (segmented long rows)."""
    lengths = [1, 1023, 1024, 1025, 2047, 2048, 2049, 4095, 4096, 4097, 8192, 8193, 12288, 3, 0, 7]
    lp = _lp_rows(lengths, 20_000, seed=3)
    _check100(lp, prec, layout=layout, fused=0)


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_with_rowless_and_empty_instances(prec):
    n = 12
    rowless = lp_from_dense(np.zeros((0, n)), [], "", np.linspace(-1, 1, n), np.zeros(n), np.ones(n))
    emptyrows = lp_from_dense(np.zeros((3, 5)), [-1.0, 0.0, 2.0], "GEL", [1.0, -1, 0, 2, -3], -np.ones(5), np.ones(5))
    lps = [I.set_cover(50, 90, seed=1), rowless, emptyrows, I.cover_knapsack(300, seed=2)]
    for fused in (1, 0):
        with pdhg.Batch(lps, precision=prec) as b:
            res = b.solve(tol=1e-300, iter_limit=100, restarts=0, fused_window=fused, autotune=0)
            sols = [b.solution(i) for i in range(len(lps))]
        bar = 1e-10 if prec == 0 else 1e-4
        for i, lp in enumerate(lps):
            # same tolerance on both sides: an instance may reach KKT = 0 exactly
            ref = oracle.pdhg(lp, tol=1e-300, iter_limit=100, restarts=False)
            assert res[i]["iterations"] == ref.iterations
            assert parity_err(sols[i][0], sols[i][1], ref.x, ref.y) <= bar, (fused, i)


@pytest.mark.parametrize("prec", [0, 1])
def test_free_variables_and_equalities(prec):
    rng = np.random.default_rng(4)
    lp = I.tiny_lp(rng, 30, 45, bounded=False)
    lp.senses[:] = ord("E")
    A = np.zeros((30, 45))
    rows = np.repeat(np.arange(30), np.diff(lp.row_ptr))
    A[rows, lp.col_idx] = lp.val
    lp.b = A @ lp.x_star
    _check100(lp, prec)


@pytest.mark.parametrize("prec", [0, 1])
def test_staged_tile_with_many_sub_tiles(prec):
    """An LDS-staged tile keeps the descriptors of its first 64 sub-tiles in
    LDS and reads the others from memory: 400k rows, almost all empty, put
    about a hundred sub-tiles of up to 4096 rows into one tile of the row
    pass, so both paths run."""
    m, n = 400_000, 3000
    full = np.zeros(m, dtype=np.int64)
    full[::997] = 3
    full[-1] = 5
    nz = np.flatnonzero(full)
    dense_rows = _lp_rows(full[nz].tolist(), n, seed=11)  # the non-empty rows
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(full, out=row_ptr[1:])
    b = np.full(m, -1.0)
    b[nz] = dense_rows.b
    lp = I.LP(m=m, n=n, row_ptr=row_ptr, col_idx=dense_rows.col_idx, val=dense_rows.val, c=dense_rows.c, b=b,
              senses=np.full(m, ord("G"), dtype=np.uint8), l=np.zeros(n), u=np.ones(n),
              is_int=np.zeros(n, dtype=np.uint8))
    _check100(lp, prec, layout=(-1, 8, -1, 8), fused=0)
    with pdhg.Batch([lp], precision=prec) as b:
        b.set_layout(-1, 8, -1, 8)
        info = b.info()
    assert info["row_blocks"] == -1
