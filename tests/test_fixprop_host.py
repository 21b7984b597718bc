"""The library's host fix-and-propagate (the rounding step of the pump loop,
Section 2.3) against the oracle's independent implementation of the same
reading: the rounding decides integers, so the two must agree bit for bit."""
import numpy as np
import pytest

import oracle
from paper_2307_03466_amd import instances as I
from paper_2307_03466_amd import pdhg


@pytest.fixture(scope="module", autouse=True)
def _lib():
    import os
    if not os.path.exists(pdhg.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    pdhg.lib()


def _cases():
    out = []
    for s in range(4):
        out.append(("cover", I.set_cover(200, 500, seed=100 + s)))
    for s in range(6):
        out.append(("cover_knapsack", I.cover_knapsack(400 + 150 * s, seed=200 + s)))
    rng = np.random.default_rng(9)
    for s in range(6):
        lp = I.tiny_lp(rng, 12, 20, bounded=(s % 2 == 0))
        lp.is_int = (rng.random(lp.n) < 0.6).astype(np.uint8)
        out.append(("mixed", lp))
    # all-integer data: the library's incremental-activity path
    for s in range(3):
        out.append(("int_cover_knapsack", I.int_cover_knapsack(300 + 200 * s, seed=300 + s)))
    for s in range(3):
        out.append(("set_partition", I.set_partition(30, 90, seed=400 + s)))
    for s in range(4):
        lp = I.tiny_lp(rng, 10, 16)
        lp.is_int = np.ones(lp.n, dtype=np.uint8)
        lp.l, lp.u = -np.floor(rng.random(lp.n) * 4), np.floor(rng.random(lp.n) * 6)
        out.append(("int_tiny", lp))
    return out


N_CASES = 26


def test_case_count():
    assert len(_cases()) == N_CASES


@pytest.mark.parametrize("k", range(N_CASES))
def test_rounding_bit_identical_to_oracle(k):
    name, lp = _cases()[k]
    rng = np.random.default_rng(k)
    for trial in range(5):
        lo = np.where(np.isfinite(lp.l), lp.l, -5.0)
        hi = np.where(np.isfinite(lp.u), lp.u, lo + 5.0)
        xref = lo + rng.random(lp.n) * (hi - lo)
        if trial == 1:  # exact halves and integers: tie handling
            xref = np.round(xref * 2) / 2
        if trial == 2:
            xref = oracle.pdhg(lp, tol=1e-3, iter_limit=20_000).x
        a = oracle.fix_propagate(lp, xref)
        b = pdhg.fix_propagate(lp, xref)
        np.testing.assert_array_equal(a[0], b[0])
        assert a[1] == b[1] and a[2] == b[2], (name, trial, a[1:], b[1:])


def test_rounding_rejects_bad_input():
    lp = I.workload(1)
    with pytest.raises(pdhg.ScyllaError):
        pdhg.fix_propagate(lp, np.full(lp.n, np.nan))
