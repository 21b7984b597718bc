"""Restart to the average (PDLP's restart candidates; scylla_params.restart_avg)
on the device against the FP64 oracle, through the C ABI.

The running mean of the iterates since the last restart is folded in by
the pass epilogues, checked by a second KKT check every window, and taken
over the iterate by the decision when its error is lower (termination,
restart, iteration-limit stop).  Bars: the means and the returned point
after 100 iterations with restarts off (no restart decision can flip) to
1e-10 (FP64) / 1e-4 (FP32), in norm and per entry, under every layout; the
FP64 trajectory with restarts on to 1e-8 after 320 iterations (the
restart decisions, taken in FP64 on both sides, agree); solves to 1e-4
checked by the oracle's KKT, constant and adaptive steps."""
import numpy as np
import pytest

import oracle
from paper_2307_03466_amd import instances as I
from lp_util import kkt_numpy, parity_err

pytestmark = pytest.mark.gpu

pdhg = pytest.importorskip("paper_2307_03466_amd.pdhg")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    pdhg.lib()


def _case(name):
    if name == "cover200":
        return I.workload(1)
    if name == "general_small":
        return I.workload(2, scale=0.002)
    if name == "skewed_longrows":
        return I.workload(3, scale=0.01)
    if name == "knapsack":
        return I.cover_knapsack(3000, seed=7)
    if name == "mixed_bounds":
        return I.tiny_lp(np.random.default_rng(3), 40, 70, bounded=False)
    raise KeyError(name)


CASES = ["cover200", "general_small", "skewed_longrows", "knapsack", "mixed_bounds"]


def _returned_matches(x, y, lp, iters, bar):
    """The returned point is the oracle's candidate at the iteration limit
    (restarts off: the trajectory is the one without the average); where the
    two candidates' errors are within 1e-3 of each other the FP32 path may
    take the other one, which then has to match instead."""
    ref = oracle.pdhg(lp, tol=-1.0, iter_limit=iters, restarts=False, restart_avg=True)
    cur = oracle.pdhg(lp, tol=-1.0, iter_limit=iters, restarts=False)
    if parity_err(x, y, ref.x, ref.y) <= bar:
        return True
    e_avg = kkt_numpy(lp, ref.x_avg, ref.y_avg)["rel"]
    e_cur = kkt_numpy(lp, cur.x, cur.y)["rel"]
    other = (cur.x, cur.y) if e_avg < e_cur else (ref.x_avg, ref.y_avg)
    return abs(e_avg - e_cur) <= 1e-3 * max(e_avg, e_cur) and parity_err(x, y, *other) <= bar


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("prec,bar", [(0, 1e-10), (1, 1e-4)])
def test_average_fixed_iteration_parity(name, prec, bar):
    lp = _case(name)
    print(f"restart_avg {name} prec {prec}", flush=True)
    ref = oracle.pdhg(lp, tol=-1.0, iter_limit=100, restarts=False, restart_avg=True)
    with pdhg.Batch([lp], precision=prec) as b:
        r = b.solve(tol=1e-300, iter_limit=100, restarts=0, restart_avg=1, autotune=0)[0]
        x, y = b.solution(0)
        xa, ya = b.average(0)
    assert r["iterations"] == 100
    assert parity_err(xa, ya, ref.x_avg, ref.y_avg) <= bar, name
    assert _returned_matches(x, y, lp, 100, bar), name
    k = oracle.kkt(lp, x, y)
    assert abs(r["rel_kkt"] - k["rel"]) <= 1e-9 * max(1, k["rel"])


LAYOUTS = [(0, 4, 0, 4), (4, 8, 2, 8), (-1, 8, -1, 8), (-2, 8, -2, 8), (-6, 8, -6, 8)]


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("prec,bar", [(0, 1e-10), (1, 1e-4)])
def test_average_under_every_layout(layout, prec, bar):
    """Every epilogue (tiles, long rows, blocked, staged, sliced and direct
    passes) folds its entries into the mean; a batch of instances of
    different sizes (some long rows, some gathered vectors too long for LDS)."""
    lps = [_case("skewed_longrows"), I.cover_knapsack(24_000, seed=5), I.cover_knapsack(900, seed=1)]
    with pdhg.Batch(lps, precision=prec) as b:
        b.set_layout(*layout)
        res = b.solve(tol=1e-300, iter_limit=100, restarts=0, restart_avg=1)
        out = [(b.solution(q), b.average(q)) for q in range(len(lps))]
    for q, lp in enumerate(lps):
        ref = oracle.pdhg(lp, tol=-1.0, iter_limit=100, restarts=False, restart_avg=True)
        (x, y), (xa, ya) = out[q]
        assert res[q]["iterations"] == 100
        assert parity_err(xa, ya, ref.x_avg, ref.y_avg) <= bar, (layout, q)
        assert _returned_matches(x, y, lp, 100, bar), (layout, q)


@pytest.mark.parametrize("name", CASES)
def test_fp64_trajectory_with_restarts(name):
    """FP64, restarts on: after 320 iterations (five checks, restarts to the
    mean or the current iterate, weight updates) the device follows the
    oracle."""
    lp = _case(name)
    ref = oracle.pdhg(lp, tol=-1.0, iter_limit=320, restart_avg=True)
    with pdhg.Batch([lp], precision=0) as b:
        r = b.solve(tol=1e-300, iter_limit=320, restart_avg=1, autotune=0)[0]
        x, y = b.solution(0)
    print(f"{name}: restarts {r['restarts']} oracle {ref.restarts}", flush=True)
    assert r["restarts"] == ref.restarts
    assert abs(r["omega"] - ref.omega) <= 1e-8 * ref.omega
    assert parity_err(x, y, ref.x, ref.y) <= 1e-8, name


@pytest.mark.parametrize("adaptive", [0, 1])
@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("prec", [0, 1])
def test_restart_to_average_reaches_the_tolerance(name, prec, adaptive):
    lp = _case(name)
    ref = oracle.pdhg(lp, tol=1e-4, iter_limit=300_000, restart_avg=True, adaptive=bool(adaptive))
    plain = oracle.pdhg(lp, tol=1e-4, iter_limit=300_000)
    with pdhg.Batch([lp], precision=prec) as b:
        r = b.solve(tol=1e-4, iter_limit=300_000, restart_avg=1, adaptive=adaptive)[0]
        x, y = b.solution(0)
    print(f"{name} prec {prec} adaptive {adaptive}: {r['iterations']} it (oracle {ref.iterations}, "
          f"without the average {plain.iterations})", flush=True)
    assert r["status"] == pdhg.OPTIMAL
    k = oracle.kkt(lp, x, y)
    assert k["rel"] <= 1e-4 * (1 + 1e-6)
    assert abs(r["rel_kkt"] - k["rel"]) <= 1e-9 * max(1, k["rel"])
    assert r["iterations"] <= 1.5 * ref.iterations + 128


def test_batch_to_tolerance_and_repeatable():
    lps = I.uneven_batch(count=6, lo=300, hi=6000, seed=21) + [_case("skewed_longrows")]
    outs = []
    for rep in range(2):
        with pdhg.Batch(lps, precision=1) as b:
            res = b.solve(tol=1e-4, iter_limit=200_000, restart_avg=1)
            outs.append([b.solution(q) for q in range(len(lps))])
        for q, lp in enumerate(lps):
            assert res[q]["status"] == pdhg.OPTIMAL
            assert oracle.kkt(lp, *outs[-1][q])["rel"] <= 1e-4 * (1 + 1e-6)
    for a, b2 in zip(outs[0], outs[1]):
        np.testing.assert_array_equal(a[0], b2[0])
        np.testing.assert_array_equal(a[1], b2[1])


def test_bad_arguments():
    lp = _case("cover200")
    with pdhg.Batch([lp], precision=1) as b:
        with pytest.raises(pdhg.ScyllaError):
            b.average(0)  # no solve with the average yet
        with pytest.raises(pdhg.ScyllaError):
            b.solve(tol=1e-4, iter_limit=10, restart_avg=2)
