"""Cutting finished instances out of the iteration launches of a batched
solve (scylla_params.compact): the cut tile lists keep the running
instances' tiles in their order and renumber the adaptive-step slots, so the
iterates, iteration counts and KKT values are the same bit for bit as
without cutting, under every layout, with constant or adaptive steps and
with restarts to the average; and cuts do happen on a batch whose instances
finish far apart."""
import numpy as np
import pytest

import oracle
from paper_2307_03466_amd import instances as I
from paper_2307_03466_amd import pdhg

pytestmark = pytest.mark.gpu


def _batch():
    # 40 cover/knapsack LPs of 500-8,000 rows: they need from a few hundred
    # to several thousand iterations, so most tiles finish early
    return I.uneven_batch(count=40, lo=500, hi=8_000, seed=5)


LAYOUTS = [None, (0, 8, 0, 8), (-1, 8, -1, 8), (-2, 8, -2, 8), (-6, 8, -6, 8)]
MODES = [dict(), dict(adaptive=1), dict(restart_avg=1), dict(adaptive=1, restart_avg=1)]


@pytest.mark.parametrize("mode", MODES, ids=["const", "adaptive", "avg", "avg_adaptive"])
@pytest.mark.parametrize("layout", LAYOUTS, ids=["tuned", "normal", "staged", "sliced", "direct"])
def test_cutting_is_bitwise_neutral(layout, mode, capfd, monkeypatch, tmp_path):
    lps = _batch()
    # the tuned layout is chosen once and reused by the second handle
    monkeypatch.setenv("SCYLLA_TUNE_CACHE", str(tmp_path / "tune.txt"))
    monkeypatch.setenv("SCYLLA_CUT_TRACE", "1")
    print(f"cut parity layout {layout} mode {mode}", flush=True)
    out = {}
    for compact in (0, 1):
        capfd.readouterr()
        with pdhg.Batch(lps, precision=1) as b:
            if layout:
                b.set_layout(*layout)
            res = b.solve(tol=1e-4, iter_limit=50_000, fused_window=0, compact=compact, **mode)
            sols = [b.solution(i) for i in range(len(lps))]
        cuts = capfd.readouterr().err.count("cut after window")
        out[compact] = (res, sols, cuts)
    assert out[0][2] == 0
    assert out[1][2] >= 1, "no cut on a batch that finishes far apart"
    its = [r["iterations"] for r in out[0][0]]
    assert max(its) >= 2 * min(its), its
    for i in range(len(lps)):
        r0, r1 = out[0][0][i], out[1][0][i]
        for k in ("status", "iterations", "restarts", "rel_kkt", "primal_obj", "dual_obj", "omega"):
            assert r0[k] == r1[k], (i, k, r0[k], r1[k])
        np.testing.assert_array_equal(out[0][1][i][0], out[1][1][i][0])
        np.testing.assert_array_equal(out[0][1][i][1], out[1][1][i][1])
    for i in (0, len(lps) // 2, len(lps) - 1):
        assert out[1][0][i]["status"] == pdhg.OPTIMAL
        k = oracle.kkt(lps[i], *out[1][1][i])
        assert k["rel"] <= 1e-4 * (1 + 1e-6)
        assert abs(out[1][0][i]["rel_kkt"] - k["rel"]) <= 1e-9 * max(1, k["rel"])


def test_cut_then_warm_resolve_uses_the_full_lists(capfd, monkeypatch):
    """A solve that cut leaves the handle with its full tile lists: a warm
    re-solve with a changed objective runs every instance again and equals
    the same re-solve on a handle that never cut."""
    lps = _batch()
    monkeypatch.setenv("SCYLLA_CUT_TRACE", "1")
    out = []
    for compact in (0, 1):
        with pdhg.Batch(lps, precision=1) as b:
            b.set_layout(-2, 8, -2, 8)
            b.solve(tol=1e-4, iter_limit=50_000, fused_window=0, compact=compact)
            for i, lp in enumerate(lps):
                b.set_objective(i, 0.5 * lp.c)
            res = b.solve(warm=True, tol=1e-5, iter_limit=50_000, fused_window=0, compact=compact)
            out.append((res, [b.solution(i) for i in range(len(lps))]))
    assert capfd.readouterr().err.count("cut after window") >= 2
    for i in range(len(lps)):
        assert out[0][0][i]["iterations"] == out[1][0][i]["iterations"] > 0
        np.testing.assert_array_equal(out[0][1][i][0], out[1][1][i][0])
        np.testing.assert_array_equal(out[0][1][i][1], out[1][1][i][1])


@pytest.mark.parametrize("layout", [None, (-2, 8, -2, 8)], ids=["tuned", "sliced"])
def test_cutting_is_bitwise_neutral_fp64(layout, capfd, monkeypatch, tmp_path):
    """The same in the FP64 path (its own tile sizes and slices)."""
    lps = _batch()
    monkeypatch.setenv("SCYLLA_TUNE_CACHE", str(tmp_path / "tune.txt"))
    monkeypatch.setenv("SCYLLA_CUT_TRACE", "1")
    out = {}
    for compact in (0, 1):
        capfd.readouterr()
        with pdhg.Batch(lps, precision=0) as b:
            if layout:
                b.set_layout(*layout)
            res = b.solve(tol=1e-4, iter_limit=50_000, fused_window=0, compact=compact, adaptive=1)
            sols = [b.solution(i) for i in range(len(lps))]
        out[compact] = (res, sols, capfd.readouterr().err.count("cut after window"))
    assert out[0][2] == 0 and out[1][2] >= 1
    for i in range(len(lps)):
        assert out[0][0][i]["iterations"] == out[1][0][i]["iterations"]
        assert out[0][0][i]["rel_kkt"] == out[1][0][i]["rel_kkt"]
        np.testing.assert_array_equal(out[0][1][i][0], out[1][1][i][0])
        np.testing.assert_array_equal(out[0][1][i][1], out[1][1][i][1])


def test_instances_without_iterations_are_cut_before_the_first_window(capfd, monkeypatch):
    """The pump's two-group schedule solves half the batch at a time: the
    other half takes no iterations and is cut before the first window; the
    loop's result equals the lockstep loop's and the uncut run's."""
    lps = I.uneven_batch(count=40, lo=400, hi=3_000, seed=9)
    monkeypatch.setenv("SCYLLA_CUT_TRACE", "1")
    out = []
    for compact in (0, 1):
        capfd.readouterr()
        with pdhg.Batch(lps, precision=1) as b:
            b.set_layout(-2, 8, -2, 8)
            recs, outs, x = b.pump_ex(pump=dict(rounds=4, seed=0, pipeline=1, early_exit=0), iter_limit=20_000,
                                      compact=compact, fused_window=0)
        err = capfd.readouterr().err
        out.append((recs, outs, x, err))
    assert "cut after window -1" not in out[0][3]
    assert "cut after window -1" in out[1][3]
    np.testing.assert_array_equal(out[0][2], out[1][2])
    for a, b2 in zip(out[0][1], out[1][1]):
        assert a == b2


def test_time_limit_with_cut_lists_then_a_full_solve(monkeypatch):
    """A solve stopped by its time limit while the lists are cut leaves the
    handle whole: the next cold solve runs every instance to the tolerance
    and equals a fresh handle's solve bit for bit."""
    lps = _batch()
    res_fresh = None
    with pdhg.Batch(lps, precision=1) as b:
        b.set_layout(-2, 8, -2, 8)
        # to 1e-6 the small instances finish and are cut out while the
        # large ones run into the time limit
        r = b.solve(tol=1e-6, iter_limit=5_000_000, fused_window=0, time_limit_s=0.2)
        assert {x["status"] for x in r} <= {pdhg.OPTIMAL, pdhg.TIME_LIMIT}, r
        res = b.solve(tol=1e-4, iter_limit=50_000, fused_window=0)
        sols = [b.solution(i) for i in range(len(lps))]
    with pdhg.Batch(lps, precision=1) as b:
        b.set_layout(-2, 8, -2, 8)
        res_fresh = b.solve(tol=1e-4, iter_limit=50_000, fused_window=0)
        fresh = [b.solution(i) for i in range(len(lps))]
    for i in range(len(lps)):
        assert res[i]["status"] == pdhg.OPTIMAL
        assert res[i]["iterations"] == res_fresh[i]["iterations"]
        np.testing.assert_array_equal(sols[i][0], fresh[i][0])
        np.testing.assert_array_equal(sols[i][1], fresh[i][1])
