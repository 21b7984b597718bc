"""The allocation-free MIP-feasibility test (scylla_batch_mip_feasible_static,
flags in a static device array) against the allocating entry point
(scylla_batch_mip_feasible), through the C ABI.  The flags are integer
decisions taken by the same kernels on the same iterates, so they must be
identical; two calls in a row share the static array, the second on a
smaller batch, so a flag left over from the first call would show."""
import numpy as np
import pytest

import oracle
from paper_2307_03466_amd import instances as I

pytestmark = pytest.mark.gpu
pdhg = pytest.importorskip("paper_2307_03466_amd.pdhg")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    pdhg.lib()


def _big():
    return [I.cover_knapsack(3000, seed=1), I.set_cover(400, 1000, seed=2), I.set_partition(60, 200, seed=3),
            I.cover_knapsack(500, seed=4), I.int_cover_knapsack(300, seed=5)]


def _small():
    return [I.set_cover(120, 300, seed=6), I.cover_knapsack(200, seed=7)]


def _candidates(lp, rng, k):
    """Both outcomes: the certificate point rounded or not, the oracle's
    rounding of it, random points, all ones."""
    lo = np.where(np.isfinite(lp.l), lp.l, -3.0)
    hi = np.where(np.isfinite(lp.u), lp.u, lo + 3.0)
    xs = np.clip(lp.x_star, lo, hi)
    ii = lp.is_int.astype(bool)
    pts = [xs, np.where(ii, np.round(xs), xs), oracle.fix_propagate(lp, xs)[0], lo + rng.random(lp.n) * (hi - lo),
           np.ones(lp.n), np.where(ii, np.floor(xs), xs)]
    return pts[k % len(pts)]


def _plant(b, lps, rng, k):
    for q, lp in enumerate(lps):
        b.set_start(q, x0=_candidates(lp, rng, k + q))


@pytest.mark.parametrize("prec", [0, 1])
def test_static_flags_equal_the_allocating_entry_point(prec):
    rng = np.random.default_rng(3 + prec)
    big, small = _big(), _small()
    seen = set()
    with pdhg.Batch(big, precision=prec) as bb, pdhg.Batch(small, precision=prec) as bs:
        ii_big = np.concatenate([lp.is_int for lp in big])
        ii_small = np.concatenate([lp.is_int for lp in small])
        ii_small_relaxed = ii_small.copy()
        ii_small_relaxed[: small[0].n] = 0
        for k in range(6):
            _plant(bb, big, rng, k)
            _plant(bs, small, rng, k + 1)
            for ib, is_ in ((None, None), (ii_big, ii_small), (ii_big, ii_small_relaxed)):
                for tol in (1e-6, 1e-12):
                    # two calls in a row on the static array, the second smaller
                    a_big = bb.mip_feasible_static(ib, tol=tol)
                    a_small = bs.mip_feasible_static(is_, tol=tol)
                    r_big = bb.mip_feasible(ib, tol=tol)
                    r_small = bs.mip_feasible(is_, tol=tol)
                    np.testing.assert_array_equal(a_big, r_big)
                    np.testing.assert_array_equal(a_small, r_small)
                    # and the smaller batch first, then the larger one
                    np.testing.assert_array_equal(bs.mip_feasible_static(is_, tol=tol), r_small)
                    np.testing.assert_array_equal(bb.mip_feasible_static(ib, tol=tol), r_big)
                    seen.update(r_big.tolist() + r_small.tolist())
    assert seen == {0, 1}


def test_static_entry_point_allocates_no_device_memory():
    """After the first call on the GPU (which maps the static array), calls
    on a fresh batch leave the device's free memory unchanged."""
    import torch
    with pdhg.Batch(_small(), precision=1) as b0:
        b0.mip_feasible_static()
    lps = _big()
    with pdhg.Batch(lps, precision=1) as b:
        b.solve(tol=1e-4, iter_limit=3000)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        a = [b.mip_feasible_static() for _ in range(3)]
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        r = b.mip_feasible()
    assert free1 == free0
    for x in a:
        np.testing.assert_array_equal(x, r)


def test_static_entry_point_rejects_a_batch_beyond_its_array():
    """2 n + m (+ count) flag bytes beyond 16 MiB: -EINVAL, nothing written,
    while the allocating entry point handles the same batch."""
    n = 8_400_000
    lp = I.set_cover(1, 10, seed=9)
    wide = I.LP(m=1, n=n, row_ptr=np.array([0, 3], np.int64), col_idx=np.array([0, 5, n - 1], np.int32),
                val=np.ones(3), c=np.ones(n), b=np.ones(1), senses=np.array([ord("G")], np.uint8),
                l=np.zeros(n), u=np.ones(n), is_int=np.ones(n, np.uint8), name="wide")
    with pdhg.Batch([lp, wide], precision=1) as b:
        out = np.full(2, 7, dtype=np.int32)
        rc = pdhg.lib().scylla_batch_mip_feasible_static(b._h, None, 1e-6, pdhg._ptr(out))
        assert rc == -22
        assert b"static scratch" in pdhg.lib().scylla_last_error()
        assert np.all(out == 7)
        assert b.mip_feasible().tolist() == [0, 0]  # x = 0 violates both covering rows


def test_static_entry_point_bad_arguments():
    with pdhg.Batch(_small(), precision=1) as b:
        for tol in (0.0, -1.0, float("nan"), float("inf")):
            with pytest.raises(pdhg.ScyllaError):
                b.mip_feasible_static(tol=tol)
        assert pdhg.lib().scylla_batch_mip_feasible_static(None, None, 1e-6, None) == -22
