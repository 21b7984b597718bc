"""GPU parity of the batched fix-and-propagate on the device
(scylla_batch_fix_propagate) with the oracle's batched procedure, instance
by instance.  Rounding is exact work (FP64 in a fixed order, decisions on
integers and bounds), so the roundings, the feasibility flags, the ignored
counts and the ignored-row masks must be identical (zeros compare by value:
the sign of a zero bound is not part of the result)."""
import numpy as np
import pytest

import oracle
from paper_2307_03466_amd import instances as I
from lp_util import csr

pytestmark = pytest.mark.gpu
pdhg = pytest.importorskip("paper_2307_03466_amd.pdhg")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    pdhg.lib()


def _mixed_lp(seed, m=14, n=22, bounded=True):
    """Tiny LP with mixed senses, continuous columns and (unbounded=False)
    infinite bounds."""
    rng = np.random.default_rng(seed)
    lp = I.tiny_lp(rng, m, n, bounded=bounded)
    lp.is_int = (rng.random(lp.n) < 0.6).astype(np.uint8)
    return lp


def _family():
    return [I.set_cover(120, 300, seed=3), I.cover_knapsack(400, seed=4), I.set_partition(40, 140, seed=5),
            _mixed_lp(6), I.int_cover_knapsack(300, seed=7), _mixed_lp(8, 30, 50, bounded=False),
            I.cover_knapsack(3000, seed=9), _mixed_lp(10, 1, 3)]


def _references(lps, rng):
    """Reference values with ties in the fixing order: a quarter exact
    integers, a quarter on .25 / .5 / .75, the rest uniform on the domain."""
    out = []
    for lp in lps:
        lo = np.where(np.isfinite(lp.l), lp.l, -4.0)
        hi = np.where(np.isfinite(lp.u), lp.u, lo + 4.0)
        x = lo + rng.random(lp.n) * (hi - lo)
        k = rng.random(lp.n)
        x = np.where(k < 0.25, np.round(x), x)
        x = np.where((k >= 0.25) & (k < 0.5), np.clip(np.floor(x) + rng.choice([0.25, 0.5, 0.75], lp.n), lo, hi), x)
        out.append(x)
    return out


def _check(lps, xbars, res, K, max_rounds):
    xh, feas, nign, mask = res
    c0 = r0 = 0
    for q, (lp, xb) in enumerate(zip(lps, xbars)):
        ex, eok, en, emask = oracle.fix_propagate_batched(lp, xb, K=K, max_rounds=max_rounds)
        got = xh[c0:c0 + lp.n]
        assert np.array_equal(got, ex), (q, lp.name, K, max_rounds, np.flatnonzero(got != ex)[:8])
        assert feas[q] == eok and nign[q] == en, (q, lp.name, K, max_rounds)
        assert np.array_equal(mask[r0:r0 + lp.m], emask), (q, lp.name, K, max_rounds)
        c0 += lp.n
        r0 += lp.m


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("K,max_rounds", [(1, 1000), (3, 1000), (64, 1000), (10 ** 6, 1000), (1, 1), (16, 2)])
def test_device_rounding_equals_the_oracle(prec, K, max_rounds):
    lps = _family()
    rng = np.random.default_rng(11 + K + max_rounds)
    xbars = _references(lps, rng)
    print(f"fix-propagate parity prec={prec} K={K} max_rounds={max_rounds}", flush=True)
    with pdhg.Batch(lps, precision=prec) as b:
        for rep in range(2):  # the device copies and work arrays are reused
            res = b.fix_propagate(K, max_rounds, is_int=np.concatenate([lp.is_int for lp in lps]),
                                  xbar=np.concatenate(xbars))
            _check(lps, xbars, res, K, max_rounds)
            xbars = _references(lps, rng)


def test_hand_worked_cases_on_the_device():
    """The round cap and the conflict rule of the oracle's pins, in one
    batch: a chain that needs four rounds, and two rows that derive y >= 3
    and y <= 1 in the same round."""
    from tests.test_oracle_fixprop_batched import _chain, _lp
    chain = _chain()
    conflict = _lp([{0: -3, 1: 1}, {0: 3, 1: 1}], "GL", [0, 4], [0, 0], [1, 5], [1, 1], 2)
    lps = [chain, conflict]
    xb = np.array([1.0, 0.4, 0.4, 0.4, 0.4, 1.0, 2.3])
    with pdhg.Batch(lps, precision=1) as b:
        xh, feas, nign, mask = b.fix_propagate(1, 1000, xbar=xb)
        assert xh.tolist() == [1, 1, 1, 1, 1, 1, 2] and feas.tolist() == [True, False]
        assert nign.tolist() == [0, 2] and mask.tolist() == [False] * 4 + [True, True]
        xh, feas, nign, mask = b.fix_propagate(1, 2, xbar=xb)
        assert xh[:5].tolist() == [1, 1, 1, 0, 0] and nign.tolist() == [1, 2]


@pytest.mark.parametrize("prec", [0, 1])
def test_rounding_of_the_iterate(prec):
    """xbar = NULL rounds every instance's current iterate (path precision
    widened to FP64): the same as rounding the iterate read back."""
    lps = I.pump_batch(6, 600, 1200, seed=21)
    with pdhg.Batch(lps, precision=prec) as b:
        b.solve(tol=1e-3, iter_limit=400)
        x = b.x_all()
        xbars, c0 = [], 0
        for lp in lps:
            xbars.append(x[c0:c0 + lp.n])
            c0 += lp.n
        for K in (1, 32):
            _check(lps, xbars, b.fix_propagate(K), K, 1000)


def test_full_size_pump_instances():
    """Eight 20k x 40k cover/knapsack instances (the shape of the pump
    workload) at their PDHG iterate after 300 iterations, K = 64."""
    lps = I.pump_batch(8, 20_000, 40_000, seed=5)
    with pdhg.Batch(lps, precision=1) as b:
        b.solve(tol=1e-4, iter_limit=300)
        x = b.x_all()
        xbars, c0 = [], 0
        for lp in lps:
            xbars.append(x[c0:c0 + lp.n])
            c0 += lp.n
        _check(lps, xbars, b.fix_propagate(64), 64, 1000)


def test_bad_arguments():
    lps = [I.set_cover(20, 40, seed=1)]
    with pdhg.Batch(lps, precision=1) as b:
        for K, mr in [(0, 10), (1, 0)]:
            with pytest.raises(pdhg.ScyllaError) as e:
                b.fix_propagate(K, mr)
            assert e.value.code == -22
        bad = np.zeros(40)
        bad[3] = np.nan
        with pytest.raises(pdhg.ScyllaError):
            b.fix_propagate(4, xbar=bad)


def test_pump_with_device_rounding():
    """One round of the complete loop with the device rounding: every
    instance whose iterate is not MIP-feasible returns the device rounding of
    that iterate (its x_out), equal to the oracle's batched rounding of the
    iterate read back."""
    lps = I.pump_batch(6, 800, 1600, seed=31)
    with pdhg.Batch(lps, precision=1) as b:
        recs, outs, xo = b.pump_ex(pump=dict(rounds=1, fp_batch=16, perturb=0, eps_schedule=0),
                                   tol=1e-3, iter_limit=500)
        x = b.x_all()
        c0 = 0
        for q, lp in enumerate(lps):
            xb = x[c0:c0 + lp.n]
            ex, eok, en, _ = oracle.fix_propagate_batched(lp, xb, K=16)
            r = recs[0][q]
            if outs[q]["found_kind"] != 1:
                assert np.array_equal(xo[c0:c0 + lp.n], ex), q
                assert r["xhat_feasible"] == eok and r["ignored_rows"] == en, q
            c0 += lp.n
        with pytest.raises(pdhg.ScyllaError):
            b.pump_ex(pump=dict(rounds=1, fp_batch=4, pipeline=1))


def test_edge_instances_and_many_workgroups():
    """Row-less instances, rows without nonzeros, an instance without
    integer columns, long rows (more nonzeros than a thread group) and 300
    small instances in one batch (more workgroups than CUs)."""
    from tests.lp_util import lp_from_dense
    n = 12
    rowless = lp_from_dense(np.zeros((0, n)), [], "", np.linspace(-1, 1, n), np.zeros(n), np.full(n, 3.0),
                            is_int=np.ones(n))
    emptyrows = lp_from_dense(np.zeros((3, 5)), [-1.0, 0.0, 2.0], "GEL", [1.0, -1, 0, 2, -3], -np.ones(5),
                              np.ones(5), is_int=np.array([1, 0, 1, 0, 1]))
    cont = _mixed_lp(40, 20, 30, bounded=False)
    cont.is_int[:] = 0
    rng = np.random.default_rng(3)
    wide = lp_from_dense(rng.integers(0, 2, size=(4, 3000)).astype(float), [1500, 1400, 10, 1600], "LLGG",
                         np.ones(3000), np.zeros(3000), np.ones(3000), is_int=np.ones(3000))
    lps = [rowless, emptyrows, cont, wide] + [I.set_cover(12, 30, seed=s) for s in range(300)]
    xbars = _references(lps, np.random.default_rng(5))
    with pdhg.Batch(lps, precision=1) as b:
        for K in (1, 7):
            res = b.fix_propagate(K, 1000, is_int=np.concatenate([lp.is_int for lp in lps]),
                                  xbar=np.concatenate(xbars))
            _check(lps, xbars, res, K, 1000)


@pytest.mark.parametrize("K", [1, 64])
def test_feasible_integral_reference_comes_back(K):
    """Soundness on the device: planted set partitions (equality rows) and
    a set cover at all ones are returned unchanged, no row ignored."""
    lps = [I.set_partition(30, 120, seed=s) for s in range(8)] + [I.set_cover(120, 300, seed=3)]
    xbars = [lp.x_star for lp in lps]
    with pdhg.Batch(lps, precision=1) as b:
        xh, feas, nign, mask = b.fix_propagate(K, xbar=np.concatenate(xbars))
    assert np.array_equal(xh, np.concatenate(xbars)) and feas.all() and not nign.any() and not mask.any()


def test_device_rounding_of_a_failed_iterate():
    """An instance whose solve ended with NUMERICAL_ERROR has a non-finite
    iterate: its integer variables are still rounded to integers inside
    their bounds (non-finite entries last in the fixing order, at the lower
    end of the domain), continuous ones keep the non-finite value, and a
    row with a non-finite activity counts as violated -- the flag agrees
    with an independent row check of the returned point."""
    good = I.cover_knapsack(400, seed=4)
    bad = I.cover_knapsack(400, seed=4)
    bad.c = bad.c * 1e60  # FP32: c -> inf and t -> 0, so the first window yields NaN
    cover_bad = I.set_cover(120, 300, seed=3)
    cover_bad.c = cover_bad.c * 1e60
    lps = [good, bad, cover_bad]
    is_int = np.ones(sum(lp.n for lp in lps), np.uint8)
    is_int[good.n + 5] = 0  # one continuous variable in the knapsack instance that fails
    with pdhg.Batch(lps, precision=1) as b:
        res = b.solve(tol=1e-4, iter_limit=2000, autotune=0)
        assert [r["status"] for r in res][1:] == [pdhg.NUMERICAL_ERROR] * 2, res
        x_bad = b.solution(1)[0]
        assert not np.all(np.isfinite(x_bad))
        for K in (1, 8):
            xh, feas, _, _ = b.fix_propagate(K, is_int=is_int)
            off = np.cumsum([0] + [lp.n for lp in lps])
            for q, lp in enumerate(lps):
                xq = xh[off[q]:off[q + 1]]
                ii = is_int[off[q]:off[q + 1]].astype(bool)
                assert np.all(np.isfinite(xq[ii])) and np.all(xq[ii] == np.round(xq[ii]))
                assert np.all(xq[ii] >= lp.l[ii]) and np.all(xq[ii] <= lp.u[ii])
                ax = csr(lp) @ xq
                tol = 1e-6 * (1 + np.abs(lp.b))
                held = np.where(lp.senses == ord("G"), ax >= lp.b - tol,
                                np.where(lp.senses == ord("L"), ax <= lp.b + tol, np.abs(ax - lp.b) <= tol))
                assert bool(feas[q]) == bool(np.all(held)), (K, q)
            # the continuous variable with a non-finite reference makes its rows fail
            xq = xh[off[1]:off[2]]
            if not np.isfinite(x_bad[5]):
                assert not np.isfinite(xq[5]) and not feas[1]
