"""GPU tests of the warm-started pump re-solves (Algorithm 1 outer loop with
the objective update; Sections 2.1, 2.3, 2.4) through the C ABI.

The round of first success is not pinned (it depends on rounding choices the
paper leaves open).  What is checked: (1) open-loop replay -- device
re-solves driven by the oracle's roundings reproduce the oracle's pump
round by round (FP64: same iteration counts and iterates; FP32: the
oracle's KKT of the device iterate meets the tolerance); (2) the native
pump's records are consistent (integral, in-bounds roundings; feasibility
flags and objective values recomputed independently; set cover always
rounds feasibly)."""
import numpy as np
import pytest

import oracle
from paper_2307_03466_amd import instances as I
from lp_util import parity_err, rel_err

pytestmark = pytest.mark.gpu
pdhg = pytest.importorskip("paper_2307_03466_amd.pdhg")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    pdhg.lib()


@pytest.mark.parametrize("prec", [0, 1])
def test_open_loop_replay_matches_oracle_pump(prec):
    lp = I.cover_knapsack(1500, seed=5)
    rounds = 4
    ref = oracle.pump(lp, rounds=rounds, tol=1e-4, iter_limit=50_000)
    kappa = np.sqrt(lp.is_int.sum()) / np.linalg.norm(lp.c)
    with pdhg.Batch([lp], precision=prec) as b:
        b.set_layout(0, 8, 0, 8)
        for K in range(1, rounds + 1):
            r = b.solve(warm=K > 1, tol=1e-4, iter_limit=50_000)[0]
            x, y = b.solution(0)
            c_hat = lp.c if K == 1 else oracle.objective_update(lp.c, ref[K - 2]["xhat"], lp.l, lp.u,
                                                                lp.is_int, K - 1)
            k = oracle.kkt(lp, x, y, c=c_hat)
            assert r["status"] == pdhg.OPTIMAL and k["rel"] <= 1e-4 * (1 + 1e-6)
            if prec == 0:
                assert r["iterations"] == ref[K - 1]["iterations"]
                assert parity_err(x, y, ref[K - 1]["x"], ref[K - 1]["y"]) <= 1e-8
            # the next round's objective from the oracle's rounding of this round
            b.set_blend(0, ref[K - 1]["xhat"] == lp.u, oracle.ALPHA ** K, kappa)


def test_native_pump_records_are_consistent():
    lps = I.pump_batch(count=6, m=1500, n=3000, seed=77)
    rounds = 5
    with pdhg.Batch(lps, precision=1) as b:
        recs, xh = b.pump(rounds=rounds, alpha=0.9, tol=1e-4, iter_limit=50_000)
    off = np.cumsum([0] + [lp.n for lp in lps])
    for q, lp in enumerate(lps):
        x_hat = xh[off[q]:off[q + 1]]
        assert np.all(x_hat == np.round(x_hat)) and np.all(x_hat >= 0) and np.all(x_hat <= 1)
        feas_rounds = [recs[k][q]["round"] for k in range(rounds) if recs[k][q]["xhat_feasible"]]
        assert bool(feas_rounds) == oracle.mip_feasible(lp, x_hat)
        for k in range(rounds):
            r = recs[k][q]
            assert r["round"] == k + 1
            assert r["status"] in (pdhg.OPTIMAL, pdhg.ITERATION_LIMIT)
        if feas_rounds:
            first = feas_rounds[0]
            assert abs(recs[first - 1][q]["xhat_obj"] - lp.c @ x_hat) <= 1e-9 * (1 + abs(lp.c @ x_hat))
    # later rounds are warm-started: they need fewer iterations in total
    it1 = sum(recs[0][q]["iterations"] for q in range(len(lps)))
    itl = sum(recs[-1][q]["iterations"] for q in range(len(lps)))
    assert itl < it1


def test_native_pump_set_cover_always_feasible():
    lps = [I.set_cover(200, 500, seed=s) for s in range(4)]
    with pdhg.Batch(lps, precision=1) as b:
        recs, xh = b.pump(rounds=3, tol=1e-4, iter_limit=50_000)
    for k in range(3):
        for q in range(4):
            assert recs[k][q]["xhat_feasible"] == 1 and recs[k][q]["ignored_rows"] == 0


def test_native_rounding_matches_oracle_on_device_iterate():
    """The rounding the native pump applies is the oracle's rounding of the
    same iterate (bit for bit)."""
    lp = I.cover_knapsack(2500, seed=8)
    with pdhg.Batch([lp], precision=1) as b:
        recs, xh = b.pump(rounds=1, tol=1e-4, iter_limit=50_000)
        x, _ = b.solution(0)
    xo, feas, ign = oracle.fix_propagate(lp, x)
    np.testing.assert_array_equal(xh, xo)
    assert recs[0][0]["xhat_feasible"] == int(feas) and recs[0][0]["ignored_rows"] == ign


# ------------------------------------------- complete Algorithm 1 loop
def _loop_batch():
    lps = [I.set_partition(12, 40, seed=s) for s in range(6)]
    lps += [I.set_partition(20, 100, seed=4), I.set_partition(20, 100, seed=5), I.cover_knapsack(300, seed=0)]
    return lps


def _oracle_loop(lps, **kw):
    return [oracle.scylla(lp, instance=q, **kw) for q, lp in enumerate(lps)]


def _compare_loop(lps, recs, outs, xo, ref):
    off = np.cumsum([0] + [lp.n for lp in lps])
    for q, lp in enumerate(lps):
        kind, K, point, rr = ref[q]
        o = outs[q]
        print(q, o, (kind, K, len(rr)), flush=True)
        assert (o["found_kind"], o["found_round"], o["rounds_run"]) == (kind, K, len(rr)), q
        assert o["perturbations"] == sum(r["perturbed"] for r in rr), q
        assert o["iterations"] == sum(r["iterations"] for r in rr), q
        for k, r in enumerate(rr):
            d = recs[k][q]
            assert d["round"] == k + 1 and d["iterations"] == r["iterations"], (q, k)
            assert d["lp_feasible"] == int(r["lp_mip_feasible"]) and d["perturbed"] == int(r["perturbed"])
            if "xhat" in r:
                assert d["xhat_feasible"] == int(r["xhat_feasible"]) and d["xhat_obj"] == pytest.approx(r["obj"], rel=1e-12)
        for k in range(len(rr), len(recs)):
            assert recs[k][q]["round"] == 0
        xq = xo[off[q]:off[q + 1]]
        if point is None:
            assert np.all(xq == 0)
        elif kind == 1:
            assert rel_err(xq, point) <= 1e-9
        else:
            np.testing.assert_array_equal(xq, point)
        assert o["obj"] == pytest.approx(float(lp.c @ xq), rel=1e-12, abs=1e-12)


def test_full_loop_matches_oracle_fp64():
    """Closed loop in FP64: the device iterates match the oracle's to
    rounding, so every round's rounding, cycle check and perturbation and
    the round of the first find are the oracle's."""
    lps = _loop_batch()
    ref = _oracle_loop(lps, rounds=20, seed=5)
    with pdhg.Batch(lps, precision=0) as b:
        recs, outs, xo = b.pump_ex(pump=dict(rounds=20, seed=5))
    _compare_loop(lps, recs, outs, xo, ref)
    assert any(o["perturbations"] for o in outs) and any(o["found_kind"] == 2 for o in outs)


def test_full_loop_with_restart_to_average_matches_oracle_fp64():
    """The closed loop with restarts to the average in every round's solve:
    the same finds, rounds and perturbations as the oracle's loop with the
    same option.  (With adaptive steps as well the rounds' iterates move
    apart by more than rounding -- that rule is not nonexpansive -- so
    only the constant-step loop is compared decision for decision.)"""
    lps = _loop_batch()
    ref = _oracle_loop(lps, rounds=20, seed=5, restart_avg=True)
    with pdhg.Batch(lps, precision=0) as b:
        recs, outs, xo = b.pump_ex(pump=dict(rounds=20, seed=5), restart_avg=1)
    _compare_loop(lps, recs, outs, xo, ref)


@pytest.mark.parametrize("K", [1, 4])
def test_full_loop_with_device_rounding_matches_oracle_fp64(K):
    """The closed loop with the batched rounding on the device: the same
    finds, rounds, perturbations and returned points as the oracle's loop
    with its batched rounding."""
    lps = _loop_batch()
    ref = _oracle_loop(lps, rounds=20, seed=5, fp_batch=K)
    with pdhg.Batch(lps, precision=0) as b:
        recs, outs, xo = b.pump_ex(pump=dict(rounds=20, seed=5, fp_batch=K))
    _compare_loop(lps, recs, outs, xo, ref)
    assert any(o["found_kind"] == 2 for o in outs)


def test_full_loop_budget_and_no_early_exit_fp64():
    lps = _loop_batch()[:4]
    ref = _oracle_loop(lps, rounds=12, seed=9, total_iter_limit=3000, iter_limit=700, early_exit=False,
                       eps_sched=False, tol=1e-5)
    with pdhg.Batch(lps, precision=0) as b:
        recs, outs, xo = b.pump_ex(pump=dict(rounds=12, seed=9, total_iter_limit=3000, early_exit=0,
                                             eps_schedule=0), tol=1e-5, iter_limit=700)
    _compare_loop(lps, recs, outs, xo, ref)
    assert all(o["iterations"] <= 3000 for o in outs)


def test_full_loop_fp32_invariants():
    lps = _loop_batch()
    with pdhg.Batch(lps, precision=1) as b:
        recs, outs, xo = b.pump_ex(pump=dict(rounds=20, seed=5))
    off = np.cumsum([0] + [lp.n for lp in lps])
    for q, lp in enumerate(lps):
        o = outs[q]
        xq = xo[off[q]:off[q + 1]]
        run = [recs[k][q] for k in range(20) if recs[k][q]["round"]]
        assert len(run) == o["rounds_run"] and sum(r["iterations"] for r in run) == o["iterations"]
        for k, r in enumerate(run):
            assert r["round"] == k + 1
            assert r["status"] != pdhg.OPTIMAL or r["rel_kkt"] <= oracle.eps_schedule(k + 1) * (1 + 1e-6)
        if o["found_kind"]:
            assert o["found_round"] == o["rounds_run"]  # early exit
            assert oracle.mip_feasible(lp, xq)
        else:
            assert o["rounds_run"] == 20 and np.all((xq == 0) | (xq == 1))
    assert outs[-1]["found_kind"] in (1, 2) and outs[-1]["found_round"] == 1  # cover + knapsack


def test_full_loop_rejects_bad_options():
    lps = _loop_batch()[:2]
    with pdhg.Batch(lps, precision=1) as b:
        for bad in (dict(rounds=0), dict(alpha=1.0), dict(eps1=0.0), dict(beta=1.5), dict(total_iter_limit=-1)):
            with pytest.raises(pdhg.ScyllaError):
                b.pump_ex(pump=bad)


_TIMING = ("solve_seconds", "round_seconds", "tune_seconds", "rounding_seconds", "group", "pad")


def _strip(recs):
    return [[{k: v for k, v in r.items() if k not in _TIMING} for r in rnd] for rnd in recs]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("opts", [dict(rounds=20, seed=5),
                                  dict(rounds=12, seed=9, total_iter_limit=3000, early_exit=0, eps_schedule=0)])
def test_pipelined_groups_equal_lockstep(prec, opts):
    """Two instance groups alternating on the device (one group's rounding
    during the other's solve) give the lockstep loop's records, outcomes
    and points bit for bit; both groups are used."""
    lps = _loop_batch()
    kw = dict(tol=1e-5, iter_limit=700) if "total_iter_limit" in opts else {}
    with pdhg.Batch(lps, precision=prec) as b:
        r1, o1, x1 = b.pump_ex(pump=dict(opts, pipeline=1), **kw)
    with pdhg.Batch(lps, precision=prec) as b:
        r0, o0, x0 = b.pump_ex(pump=dict(opts, pipeline=0), **kw)
    assert {r["group"] for r in r1[0]} == {0, 1} and {r["group"] for r in r0[0]} == {0}
    assert _strip(r1) == _strip(r0)
    assert o1 == o0
    np.testing.assert_array_equal(x1, x0)


def test_pipelined_l2_loop_equals_lockstep():
    lps = I.int_pump_batch(6, 300, 600, seed=3)
    with pdhg.Batch(lps, precision=1) as b:
        r1, o1, x1 = b.pump_ex(pump=dict(rounds=8, seed=1, distance=2, perturb=0, early_exit=0, pipeline=1))
    with pdhg.Batch(lps, precision=1) as b:
        r0, o0, x0 = b.pump_ex(pump=dict(rounds=8, seed=1, distance=2, perturb=0, early_exit=0, pipeline=0))
    assert _strip(r1) == _strip(r0) and o1 == o0
    np.testing.assert_array_equal(x1, x0)


@pytest.mark.parametrize("native", ["pump", "pump_ex"])
def test_failed_solve_leaves_the_loop_unrounded(native):
    """An instance whose solve ends with NUMERICAL_ERROR is not rounded and
    not solved again; the other instances of the batch carry on."""
    good = [I.set_cover(200, 500, seed=1), I.cover_knapsack(800, seed=2)]
    bad = I.cover_knapsack(800, seed=2)
    bad.c = bad.c * 1e60  # FP32: c -> inf and t -> 0, so the iterations yield NaN
    lps = [good[0], bad, good[1]]
    with pdhg.Batch(lps, precision=1) as b:
        if native == "pump":
            recs, xh = b.pump(rounds=3, tol=1e-4, iter_limit=20_000)
        else:
            recs, outs, xo = b.pump_ex(pump=dict(rounds=3, early_exit=0), tol=1e-4, iter_limit=20_000)
    # the round in which the solve failed (the start point may meet a loose
    # round-1 tolerance of the schedule before any iteration runs)
    fail = next(k for k in range(3) if recs[k][1]["status"] == pdhg.NUMERICAL_ERROR)
    r = recs[fail][1]
    assert r["round"] == fail + 1 and r["xhat_feasible"] == 0 and r["lp_feasible"] == 0
    for k in range(fail + 1, 3):
        assert recs[k][1]["status"] == 0 and recs[k][1]["round"] == 0
    if native == "pump_ex":
        assert outs[1]["rounds_run"] == fail + 1
        assert outs[0]["found_kind"] > 0  # set cover always rounds feasibly
    for k in range(3):
        for q in (0, 2):
            if recs[k][q]["round"]:
                assert recs[k][q]["status"] != pdhg.NUMERICAL_ERROR
    assert recs[0][0]["round"] == 1 and recs[0][2]["round"] == 1
