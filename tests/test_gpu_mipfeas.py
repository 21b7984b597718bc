"""GPU tests of the device MIP-feasibility test of the PDHG iterate
(Algorithm 1 returns the iterate itself when it is feasible for the MIP,
Section 2.1) through the C ABI (scylla_batch_mip_feasible).

The flag decides an integer from floating point, so both sides take the
decision in FP64 on the same values: the iterate as the device stores it
(read back), rows as FP64 activities.  The oracle's mip_feasible is the
reference, instance by instance; every case set must contain both
outcomes."""
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


def _mixed_lp(seed):
    """Tiny LP with mixed senses, some continuous columns, integer data."""
    rng = np.random.default_rng(seed)
    lp = I.tiny_lp(rng, 14, 22)
    lp.is_int = (rng.random(lp.n) < 0.6).astype(np.uint8)
    return lp


def _family():
    return [I.set_cover(120, 300, seed=3), I.cover_knapsack(400, seed=4), I.set_partition(40, 140, seed=5),
            _mixed_lp(6), I.int_cover_knapsack(300, seed=7), _mixed_lp(8)]


def _candidates(lp, rng):
    """Points spanning both outcomes: planted / rounded / perturbed."""
    lo = np.where(np.isfinite(lp.l), lp.l, -3.0)
    hi = np.where(np.isfinite(lp.u), lp.u, lo + 3.0)
    x_star = np.clip(lp.x_star, lo, hi)
    ii = lp.is_int.astype(bool)
    out = [x_star, np.where(ii, np.round(x_star), x_star), np.where(ii, np.floor(x_star), x_star),
           lo + rng.random(lp.n) * (hi - lo)]
    xh, feas, _ = oracle.fix_propagate(lp, x_star)
    out.append(xh)
    out.append(np.clip(xh + np.where(ii, 3e-7, 0.0) * rng.standard_normal(lp.n), lo, hi))  # inside tol
    out.append(np.clip(xh + np.where(ii, 5e-5, 0.0) * rng.standard_normal(lp.n), lo, hi))  # outside tol
    if lp.name == "set_cover":
        out.append(np.ones(lp.n))
    return out


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("tol", [1e-6, 1e-12])
def test_device_flags_match_oracle(prec, tol):
    lps = _family()
    rng = np.random.default_rng(11)
    cands = [_candidates(lp, rng) for lp in lps]
    is_int = np.concatenate([lp.is_int for lp in lps])
    off = np.cumsum([0] + [lp.n for lp in lps])
    seen = set()
    with pdhg.Batch(lps, precision=prec) as b:
        for k in range(max(len(c) for c in cands)):
            for q, lp in enumerate(lps):
                b.set_start(q, x0=cands[q][k % len(cands[q])])
            got = b.mip_feasible(is_int, tol=tol)
            xd = b.x_all()  # the values the device tested
            for q, lp in enumerate(lps):
                ref = oracle.mip_feasible(lp, xd[off[q]:off[q + 1]], tol=tol)
                assert bool(got[q]) == ref, (prec, tol, k, lp.name)
                seen.add(ref)
    assert seen == {True, False}


@pytest.mark.parametrize("prec", [0, 1])
def test_after_solve_and_integer_flags(prec):
    """After a real solve, and with the integer flags changing the answer:
    the planted fractional point 0.3 * 1 satisfies every row, so it is
    MIP-feasible exactly when no column of it is integer."""
    lp = I.cover_knapsack(600, seed=21)
    cover = I.set_cover(100, 250, seed=22)
    with pdhg.Batch([lp, cover], precision=prec) as b:
        b.solve(tol=1e-4, iter_limit=20_000)
        xd = b.x_all()
        got = b.mip_feasible()
        assert bool(got[0]) == oracle.mip_feasible(lp, xd[:lp.n])
        assert bool(got[1]) == oracle.mip_feasible(cover, xd[lp.n:])
        b.set_start(0, x0=lp.x_star)
        xs = b.x_all()[:lp.n]
        relaxed = I.cover_knapsack(600, seed=21)
        relaxed.is_int = np.zeros(lp.n, dtype=np.uint8)
        ii = np.concatenate([np.zeros(lp.n, np.uint8), np.ones(cover.n, np.uint8)])
        assert int(b.mip_feasible(ii)[0]) == int(oracle.mip_feasible(relaxed, xs)) == 1
        assert int(b.mip_feasible()[0]) == int(oracle.mip_feasible(lp, xs)) == 0


def test_bad_arguments():
    lp = I.set_cover(50, 120, seed=1)
    with pdhg.Batch([lp], precision=1) as b:
        for tol in (0.0, -1.0, float("nan"), float("inf")):
            with pytest.raises(pdhg.ScyllaError):
                b.mip_feasible(tol=tol)
