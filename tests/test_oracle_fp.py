"""Pins of the oracle's fix-and-propagate (Section 2.3), objective update
(Algorithm 1 objective step, Section 2.4) and tolerance schedule
(Section 2.2)."""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
from paper_2307_03466_amd import instances as I
from lp_util import GOLDEN, dense, lp_from_dense

with open(os.path.join(GOLDEN, "paper_constants.json")) as f:
    PAPER = json.load(f)


def _row_ok(lp, x, tol=1e-9):
    A = dense(lp)
    ax = A @ x
    s = lp.senses
    return np.where(s == ord("G"), ax >= lp.b - tol,
                    np.where(s == ord("L"), ax <= lp.b + tol, np.abs(ax - lp.b) <= tol))


# ------------------------------------------- P10 integral and within bounds
@pytest.mark.parametrize("seed", range(6))
def test_fp_output_integral_and_in_bounds(seed):
    rng = np.random.default_rng(seed)
    lp = I.cover_knapsack(300, seed=seed)
    xbar = rng.random(lp.n)
    xhat, feas, ign = oracle.fix_propagate(lp, xbar)
    assert PAPER["fp_output_integer_feasible"]["value"]
    assert np.all(xhat == np.round(xhat))
    assert np.all(xhat >= lp.l) and np.all(xhat <= lp.u)
    assert feas == bool(_row_ok(lp, xhat, 1e-6 * (1 + np.abs(lp.b))).all())


def test_fp_mixed_integer_continuous_projection():
    """Continuous variables keep the reference value projected on their
    (possibly tightened) domain; integers are integral."""
    rng = np.random.default_rng(4)
    lp = I.tiny_lp(rng, 4, 8)
    lp.is_int = (rng.random(lp.n) < 0.5).astype(np.uint8)
    xbar = lp.l + rng.random(lp.n) * (lp.u - lp.l)
    xhat, _, _ = oracle.fix_propagate(lp, xbar)
    ii = lp.is_int.astype(bool)
    assert np.all(xhat[ii] == np.round(xhat[ii]))
    assert np.all(xhat >= lp.l - 1e-12) and np.all(xhat <= lp.u + 1e-12)


# ------------------------------------------ P11 identity on feasible input
def test_fp_identity_on_feasible_integral_point():
    lp = I.workload(1)
    rng = np.random.default_rng(0)
    for _ in range(5):
        # random minimal-ish cover: start from all ones, drop columns greedily
        x = np.ones(lp.n)
        A = dense(lp)
        for j in rng.permutation(lp.n):
            x[j] = 0
            if np.any(A @ x < 1):
                x[j] = 1
        xhat, feas, ign = oracle.fix_propagate(lp, x)
        np.testing.assert_array_equal(xhat, x)
        assert feas and ign == 0


# --------------------------------------------- P12 set cover always feasible
@pytest.mark.parametrize("seed", range(8))
def test_fp_always_succeeds_on_set_cover(seed):
    lp = I.set_cover(200, 500, seed=seed + 10)
    rng = np.random.default_rng(seed)
    xbar = rng.random(lp.n) * rng.random(lp.n)  # mostly small values
    xhat, feas, ign = oracle.fix_propagate(lp, xbar)
    assert feas and ign == 0
    assert np.all(dense(lp) @ xhat >= 1)


# ---------------------------------- P13 propagation soundness by brute force
@pytest.mark.parametrize("seed", range(10))
def test_fp_never_cuts_off_a_feasible_point(seed):
    """For every feasible binary point x' of a small cover/knapsack problem,
    a reference that rounds to x' must come back as x' exactly: a fixing
    sequence consistent with x' can only leave x' if propagation removed a
    feasible point (unsound) or ignored a row that x' satisfies."""
    rng = np.random.default_rng(seed)
    n = 10
    m = 6
    A = np.zeros((m, n))
    senses = []
    b = []
    for i in range(m):
        cols = rng.choice(n, size=int(rng.integers(2, 6)), replace=False)
        if rng.random() < 0.5:
            A[i, cols] = 1
            senses.append("G")
            b.append(1.0)
        else:
            w = rng.integers(1, 20, size=cols.size)
            A[i, cols] = w
            senses.append("L")
            b.append(float(np.floor(0.5 * w.sum())))
    lp = lp_from_dense(A, b, "".join(senses), rng.integers(1, 10, size=n), np.zeros(n), np.ones(n),
                       is_int=np.ones(n))
    feasible = []
    for bits in itertools.product([0.0, 1.0], repeat=n):
        x = np.array(bits)
        if _row_ok(lp, x).all():
            feasible.append(x)
    assert feasible
    for x in feasible[:: max(1, len(feasible) // 40)]:
        noise = rng.uniform(-0.45, 0.45, size=n)
        xbar = np.clip(x + noise, 0, 1)
        xhat, feas, ign = oracle.fix_propagate(lp, xbar)
        np.testing.assert_array_equal(xhat, x)
        assert feas and ign == 0


def test_fp_ignores_conflicting_rows_and_still_returns_integral():
    # x0 + x1 >= 2 forces both to 1; 3 x0 + 3 x1 <= 4 then conflicts
    A = np.array([[1.0, 1.0], [3.0, 3.0]])
    lp = lp_from_dense(A, [2.0, 4.0], "GL", [1.0, 1.0], [0, 0], [1, 1], is_int=[1, 1])
    xhat, feas, ign = oracle.fix_propagate(lp, np.array([0.9, 0.8]))
    assert np.all(xhat == np.round(xhat)) and not feas and ign >= 1


# ------------------------------------------------ P9 objective update / eps
def test_eps_schedule_closed_form():
    e1 = PAPER["eps_initial"]["value"]
    beta = PAPER["eps_beta"]["value"]
    floor = PAPER["eps_floor"]["value"]
    assert oracle.eps_schedule(1) == e1
    for K in (2, 3, 10, 100, 500, 684, 685, 686, 1000):
        closed = max(e1 * beta ** (K - 1), floor)
        assert abs(oracle.eps_schedule(K) - closed) <= 1e-12 * closed
    # first floored round: 0.01 * 0.98^(K-1) < 1e-8  <=>  K - 1 > ln(1e-6) / ln(0.98)
    kstar = int(np.floor(np.log(1e-6) / np.log(0.98))) + 2
    assert oracle.eps_schedule(kstar) == floor and oracle.eps_schedule(kstar - 1) > floor


@pytest.mark.parametrize("K", [1, 2, 5, 20])
def test_objective_update_identities(K):
    alpha = PAPER["alpha"]["value"]
    lp = I.cover_knapsack(500, seed=K)
    rng = np.random.default_rng(K)
    xhat = (rng.random(lp.n) < 0.3).astype(float)
    c_hat = oracle.objective_update(lp.c, xhat, lp.l, lp.u, lp.is_int, K)
    nI = int(lp.is_int.sum())
    g = c_hat - alpha ** K * np.sqrt(nI) / np.linalg.norm(lp.c) * lp.c
    g /= (1 - alpha ** K)
    # the distance part is the +-1 subgradient of the L1 distance
    np.testing.assert_allclose(g, np.where(xhat == 0, 1.0, -1.0), atol=1e-9)
    # the objective part has norm alpha^K sqrt(|I|)
    part = c_hat - (1 - alpha ** K) * np.where(xhat == 0, 1.0, -1.0)
    assert abs(np.linalg.norm(part) - alpha ** K * np.sqrt(nI)) < 1e-9 * np.sqrt(nI)
    assert abs(np.linalg.norm(np.where(xhat == 0, 1.0, -1.0)) - np.sqrt(nI)) < 1e-9
    # Delta(x, x_hat) = g^T x + sum x_hat on [0,1]^n (L1 distance)
    for _ in range(5):
        x = rng.random(lp.n)
        gg = oracle.distance_gradient(xhat, lp.l, lp.u, lp.is_int)
        assert abs(np.abs(x - xhat).sum() - (gg @ x + xhat.sum())) < 1e-9


def test_objective_update_zero_c_drops_term_and_rejects_general_integers():
    n = 4
    z = oracle.objective_update(np.zeros(n), np.array([0.0, 1, 0, 1]), np.zeros(n), np.ones(n),
                                np.ones(n, dtype=np.uint8), 1)
    np.testing.assert_allclose(z, 0.1 * np.array([1.0, -1, 1, -1]))
    with pytest.raises(ValueError):
        oracle.distance_gradient(np.array([1.0]), np.zeros(1), np.array([3.0]), np.ones(1, np.uint8))


# ------------------------------------------------------------ pump (P14)
def test_pump_invariants_small():
    """Parity unpinned (round of first success depends on open rounding
    choices); check invariants only: every rounding is integral and in
    bounds, the set-cover instance is always rounded to a feasible point."""
    lp = I.workload(1)
    recs = oracle.pump(lp, rounds=3, tol=1e-4, iter_limit=20_000)
    assert len(recs) == 3
    for r in recs:
        assert np.all(r["xhat"] == np.round(r["xhat"]))
        assert r["xhat_feasible"]


def test_fp_propagates_through_a_single_infinite_term():
    """A row whose activity bound has exactly one infinite term still bounds
    that term's variable (closed form): with x0 fixed to 1,
    x0 + 2 x1 <= 3 gives x1 <= 1, and x0 - x2 >= -4 gives x2 <= 5."""
    inf = np.inf
    A = np.array([[1.0, 2.0, 0.0], [1.0, 0.0, -1.0]])
    lp = lp_from_dense(A, [3.0, -4.0], "LG", [0.0, 0.0, 0.0], [0.0, -inf, -inf], [1.0, inf, inf],
                       is_int=[1, 0, 0])
    xhat, feas, ign = oracle.fix_propagate(lp, np.array([0.9, 10.0, 20.0]))
    np.testing.assert_array_equal(xhat, [1.0, 1.0, 5.0])
    assert feas and ign == 0


# ---------------------------------------------- Algorithm 1 outer loop
def test_splitmix64_reference_values():
    """Published SplitMix64 outputs for seed 0 (first three draws of the
    reference generator: 0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4,
    0x06c45d188009454f)."""
    assert [oracle.splitmix64(0, k) for k in range(3)] == [
        0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    for K in range(1, 50):
        assert 10 <= oracle.perturb_count(7, 3, K) <= 30


def test_perturbation_flips_the_largest_gaps():
    lp = I.cover_knapsack(200, seed=1)
    rng = np.random.default_rng(0)
    xbar = rng.random(lp.n)
    xhat = np.round(xbar)
    out = oracle.perturb(lp, xbar, xhat, 12)
    flipped = np.flatnonzero(out != xhat)
    assert flipped.size == 12
    gap = np.abs(xbar - xhat)
    assert gap[flipped].min() >= np.delete(gap, flipped).max()
    assert np.all((out == 0) | (out == 1))


def test_scylla_loop_early_exit_and_schedule():
    lp = I.workload(1)  # set cover: the first rounding is always feasible
    kind, K, point, recs = oracle.scylla(lp, rounds=5)
    assert kind in (1, 2) and K == 1 and len(recs) == 1
    assert recs[0]["tol"] == PAPER["eps_initial"]["value"]
    assert oracle.mip_feasible(lp, point)
    # without early exit all rounds run, the schedule tightens, and the
    # first find is still reported
    kind2, K2, point2, recs = oracle.scylla(lp, rounds=4, early_exit=False)
    assert (kind2, K2) == (kind, 1) and np.array_equal(point2, point) and len(recs) == 4
    assert [r["tol"] for r in recs] == [oracle.eps_schedule(k) for k in range(1, 5)]


def test_scylla_cumulative_iteration_limit():
    lp = I.cover_knapsack(400, seed=9)
    kind, K, point, recs = oracle.scylla(lp, rounds=50, early_exit=False, eps_sched=False, tol=1e-9,
                                         total_iter_limit=1000, iter_limit=300)
    assert sum(r["iterations"] for r in recs) <= 1000
    assert all(r["iterations"] <= 300 for r in recs)


def test_set_partition_generator_planted_point():
    for seed in range(4):
        lp = I.set_partition(25, 90, seed=seed)
        assert oracle.mip_feasible(lp, lp.x_star)
        assert np.all(lp.val == 1.0) and np.all(lp.senses == ord("E"))


def test_scylla_cycle_perturbation_rule():
    """Set partitioning cycles: each perturbed round's rounding repeated an
    earlier rounding as used, and exactly T = perturb_count(seed, q, K)
    binaries were flipped, those with the largest |x_bar - x_hat|."""
    seen = 0
    for q, seed in enumerate(range(3)):
        lp = I.set_partition(20, 60, seed=seed)
        kind, K, point, recs = oracle.scylla(lp, rounds=20, seed=11, instance=q)
        used = []
        for r in recs:
            if "xhat" not in r:
                continue
            if r["perturbed"]:
                seen += 1
                assert any(np.array_equal(r["xhat"], u) for u in used)
                flipped = np.flatnonzero(r["xhat_used"] != r["xhat"])
                T = oracle.perturb_count(11, q, r["K"])
                assert flipped.size == min(T, lp.n)
                gap = np.abs(r["x"] - r["xhat"])
                assert gap[flipped].min() >= np.delete(gap, flipped).max(initial=0.0)
            else:
                assert not any(np.array_equal(r["xhat"], u) for u in used)
                assert r["xhat_used"] is r["xhat"]
            used.append(r["xhat_used"])
    assert seen >= 3


# ------------------------------------------------ L2 distance (Section 5)
def test_l2_objective_update_equals_definition():
    """c_hat^T x + x^T diag(q) x / 2 differs from alpha^K kappa c^T x +
    (1 - alpha^K) |x_I - x_hat_I|^2 by a constant: the same at every x."""
    rng = np.random.default_rng(4)
    n = 30
    c = rng.normal(size=n)
    is_int = (rng.random(n) < 0.6).astype(np.uint8)
    xhat = np.where(is_int == 1, rng.integers(-3, 7, size=n), 0).astype(float)
    K = 3
    c_hat, q = oracle.objective_update_l2(c, xhat, is_int, K)
    a = oracle.ALPHA ** K
    kappa = np.sqrt(is_int.sum()) / np.linalg.norm(c)
    ii = is_int.astype(bool)
    diffs = []
    for _ in range(5):
        x = rng.normal(size=n) * 4
        f = c_hat @ x + 0.5 * (q * x) @ x
        d = a * kappa * (c @ x) + (1 - a) * np.sum((x[ii] - xhat[ii]) ** 2)
        diffs.append(f - d)
    assert np.ptp(diffs) <= 1e-9 * (1 + abs(diffs[0]))
    assert np.all(q[~ii] == 0) and np.all(q[ii] == 2 * (1 - a))


def test_l2_loop_handles_general_integers():
    """General integers strictly inside their bounds: the L1 update rejects
    them, the L2 loop runs (its PDHG solves are QPs) and every rounding is
    integral and within bounds."""
    rng = np.random.default_rng(8)
    lp = I.tiny_lp(rng, 8, 12)
    lp.is_int = np.ones(lp.n, dtype=np.uint8)
    lp.l = np.zeros(lp.n)
    lp.u = np.full(lp.n, 6.0)
    xs = np.round(rng.random(lp.n) * 6)
    A = np.zeros((lp.m, lp.n))
    A[np.repeat(np.arange(lp.m), np.diff(lp.row_ptr)), lp.col_idx] = lp.val
    lp.b = A @ xs - np.where(lp.senses == ord("L"), -1.0, np.where(lp.senses == ord("G"), 1.0, 0.0))
    kind, K, point, recs = oracle.scylla(lp, rounds=6, distance="l2", cycle_perturb=False, early_exit=False)
    for r in recs:
        xh = r["xhat"]
        assert np.all(xh == np.round(xh)) and np.all(xh >= lp.l) and np.all(xh <= lp.u)
    assert any(r["K"] > 1 for r in recs)
    if kind:
        assert oracle.mip_feasible(lp, point)


def test_int_cover_knapsack_planted_point():
    for seed in range(3):
        lp = I.int_cover_knapsack(400, seed=seed)
        assert lp.u.min() >= 2 and lp.u.max() <= 5
        rows = lp.row_of_entry()
        ax = np.bincount(rows, weights=lp.val * lp.x_star[lp.col_idx], minlength=lp.m)
        assert np.all(np.where(lp.senses == ord("G"), ax >= lp.b - 1e-9, ax <= lp.b + 1e-9))
    # the binary family is unchanged by the general-integer option
    a, b = I.cover_knapsack(300, seed=5), I.cover_knapsack(300, seed=5, umax=1)
    assert np.array_equal(a.b, b.b) and np.all(a.u == 1)
