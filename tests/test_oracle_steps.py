"""Pins of the oracle's step-size and restart readings (Section 2.1 names
PDLP's restarts and step sizes without giving them; Algorithm 1 updates
the step sizes every iteration).  The readings themselves are stated in the
oracle's header; here each is restated from the iterates, which snapshot
runs expose: a run with the iteration limit at k reproduces the longer run
up to iteration k, so its returned (x, y), restart count, primal weight and
step factor are the longer run's state there.  The norms and products the
rules need are recomputed with scipy from those iterates (the preconditioner
comes from the oracle; it is pinned separately by the Ruiz and
Pock-Chambolle tests), so a mistake in any constant or formula of the
oracle's rules shows up as a disagreement with the restatement.

Planted mistakes these tests catch (each checked on a scratch copy of the
oracle): restart thresholds 0.2 and 0.8 swapped; the artificial restart
factor 0.36 changed to 0.5 or to 0.3; E > E_p flipped to E < E_p; the
primal step taken as eta omega instead of eta / omega; the primal-weight
update with the ratio
inverted (|dx|/|dy|) or without the geometric mean; the cold-start weight
inverted (|D_r b| / |D_c c|) or with D^2 in place of D; the factor 2
dropped from eta_bar; the exponents -0.3 and -0.6 swapped; the iteration
count k used in place of k + 1 in the step rule."""
import numpy as np
import pytest
import scipy.sparse as sps

import oracle
from paper_2307_03466_amd import instances as I
from lp_util import csr, kkt_numpy, lp_from_dense, rel_err


# ------------------------------------------------------- cold-start weight
def test_omega0_closed_form_on_a_diagonal_matrix():
    """A = diag(a): the first Ruiz round gives d_r = d_c = a^-1/2, after which
    A~ = I and neither the remaining Ruiz rounds nor Pock-Chambolle change
    it, so omega0 = |D_c c| / |D_r b| = |c / sqrt(a)| / |b / sqrt(a)|."""
    rng = np.random.default_rng(11)
    n = 12
    a = rng.integers(1, 50, size=n).astype(float)
    c = rng.normal(size=n)
    b = rng.normal(size=n) * 3
    lp = lp_from_dense(np.diag(a), b, "E" * n, c, -10 * np.ones(n), 10 * np.ones(n))
    dr, dc = oracle.precondition(lp)
    np.testing.assert_allclose(dr, 1 / np.sqrt(a), rtol=1e-14)
    np.testing.assert_allclose(dc, 1 / np.sqrt(a), rtol=1e-14)
    r = oracle.pdhg(lp, tol=-1.0, iter_limit=0)
    w = np.linalg.norm(c / np.sqrt(a)) / np.linalg.norm(b / np.sqrt(a))
    assert abs(r.omega - w) <= 1e-14 * w
    assert r.eta == 0.99
    # no objective or no right-hand side: weight 1
    assert oracle.pdhg(lp, tol=-1.0, iter_limit=0, c=np.zeros(n)).omega == 1.0
    lp0 = lp_from_dense(np.diag(a), np.zeros(n), "E" * n, c, -10 * np.ones(n), 10 * np.ones(n))
    assert oracle.pdhg(lp0, tol=-1.0, iter_limit=0).omega == 1.0


@pytest.mark.parametrize("name", ["cover", "general"])
def test_omega0_from_the_preconditioned_norms(name):
    lp = I.set_cover(150, 400, seed=5) if name == "cover" else I.workload(2, scale=0.001)
    dr, dc = oracle.precondition(lp)
    w = np.linalg.norm(dc * lp.c) / np.linalg.norm(dr * lp.b)
    r = oracle.pdhg(lp, tol=-1.0, iter_limit=0)
    assert abs(r.omega - w) <= 1e-13 * w
    # a given weight is used as is
    assert oracle.pdhg(lp, tol=-1.0, iter_limit=0, omega0=3.25).omega == 3.25


# ------------------------------------------------------------ restart rule
def _restart_cases():
    return [
        ("cover", I.set_cover(150, 400, seed=5), 64),
        ("cover_R16", I.set_cover(150, 400, seed=8), 16),
        ("knapsack", I.cover_knapsack(300, seed=6), 64),
        ("knapsack_R7", I.cover_knapsack(300, seed=9), 7),
        ("general", I.workload(2, scale=0.0005), 32),
        ("mixed", I.tiny_lp(np.random.default_rng(3), 40, 70, bounded=False), 5),
    ]


@pytest.mark.parametrize("avg", [False, True])
def test_restart_rule_and_weight_update_restated_from_checks(avg):
    """At each check after the start, with E the relative KKT error of the
    current point, E_r its value at the last restart (the start counts) and
    E_p at the previous check, the solve restarts iff E <= 0.2 E_r, or
    E <= 0.8 E_r and E > E_p, or k - k_r >= 0.36 k.  At a restart the primal
    weight becomes the geometric mean of the old weight and |dy~| / |dx~|,
    with dx~ = (x - x_r) / d_c and dy~ = (y - y_r) / d_r the moves since the
    last restart point (unchanged if either is <= 1e-10).  With the average
    on, "the current point" is the candidate: what a run stopped at that
    check returns (the mean when its error is lower)."""
    decisive = {"0.2": 0, "0.8": 0, "0.36": 0, "none": 0, "weight": 0}
    for name, lp, R in _restart_cases():
        dr, dc = oracle.precondition(lp)
        full = oracle.pdhg(lp, tol=1e-7, iter_limit=60 * R, check_period=R, restart_avg=avg)
        nchk = full.iterations // R
        snaps = [oracle.pdhg(lp, tol=-1.0, iter_limit=c * R, check_period=R, restart_avg=avg)
                 for c in range(nchk + 1)]
        # checks 0..nchk-1 take a decision (the last one ends the run)
        E = [kkt_numpy(lp, s.x, s.y)["rel"] for s in snaps]
        w = snaps[0].omega
        Er, Ep, kr = E[0], E[0], 0
        xr, yr = snaps[0].x, snaps[0].y
        nrest = 0
        for c in range(1, nchk):
            k = c * R
            c1, c2, c3 = E[c] <= 0.2 * Er, E[c] <= 0.8 * Er and E[c] > Ep, (k - kr) >= 0.36 * k
            fire = c1 or c2 or c3
            if fire and [c1, c2, c3].count(True) == 1:
                decisive["0.2" if c1 else ("0.8" if c2 else "0.36")] += 1
            if not fire:
                decisive["none"] += 1
            if fire:
                nrest += 1
                dx = np.linalg.norm((snaps[c].x - xr) / dc)
                dy = np.linalg.norm((snaps[c].y - yr) / dr)
                if dx > 1e-10 and dy > 1e-10:
                    w = np.sqrt(w * dy / dx)
                    decisive["weight"] += 1
                xr, yr, Er, kr = snaps[c].x, snaps[c].y, E[c], k
            Ep = E[c]
            nxt = snaps[c + 1]
            assert nxt.restarts == nrest, (name, c, E[c], Er, Ep, kr)
            assert abs(nxt.omega - w) <= 1e-11 * w, (name, c, nxt.omega, w)
    # every condition decided some restart on its own, and some checks did not restart
    if not avg:
        assert min(decisive.values()) >= 1, decisive
    else:
        assert decisive["0.36"] >= 1 and decisive["none"] >= 1 and decisive["weight"] >= 1, decisive
        assert decisive["0.2"] + decisive["0.8"] >= 1, decisive


def test_restarts_off_keep_the_cold_start_weight():
    lp = I.cover_knapsack(300, seed=6)
    w0 = oracle.pdhg(lp, tol=-1.0, iter_limit=0).omega
    r = oracle.pdhg(lp, tol=-1.0, iter_limit=1000, restarts=False)
    assert r.restarts == 0 and r.omega == w0


# ------------------------------------------------------ adaptive step rule
def _adaptive_cases():
    return [
        ("cover", I.set_cover(150, 400, seed=5)),
        ("knapsack", I.cover_knapsack(300, seed=6)),
        ("general", I.workload(2, scale=0.0005)),
        ("mixed", I.tiny_lp(np.random.default_rng(3), 40, 70, bounded=False)),
    ]


@pytest.mark.parametrize("case", range(4))
def test_adaptive_step_rule_restated_from_iterates(case):
    """After the k-th iteration (k from 1), with dx = x_k - x_(k-1),
    dy = y_k - y_(k-1) and omega the primal weight:
    eta_bar = (omega |dx / d_c|^2 + |dy / d_r|^2 / omega) / (2 |dy^T A dx|) and
    eta_k = min((1 - (k+1)^-0.3) eta_bar, (1 + (k+1)^-0.6) eta_(k-1)),
    eta_bar infinite when dy^T A dx = 0; eta unchanged when nothing moved.
    The step of iteration k is t = eta_(k-1) / omega (read back from the
    coordinates that the bounds did not clip)."""
    name, lp = _adaptive_cases()[case]
    A = csr(lp)
    dr, dc = oracle.precondition(lp)
    K = 60
    snaps = [oracle.pdhg(lp, tol=-1.0, iter_limit=k, restarts=False, adaptive=True) for k in range(K + 1)]
    w = snaps[0].omega
    assert all(s.omega == w for s in snaps)
    branches = {"shrink": 0, "grow": 0}
    for k in range(1, K + 1):
        x0, y0, x1, y1 = snaps[k - 1].x, snaps[k - 1].y, snaps[k].x, snaps[k].y
        dx, dy = x1 - x0, y1 - y0
        nx, ny = np.sum((dx / dc) ** 2), np.sum((dy / dr) ** 2)
        inter = dy @ (A @ dx)
        eta_prev = snaps[k - 1].eta
        grow = (1 + (k + 1) ** -0.6) * eta_prev
        if nx + ny == 0:
            want = eta_prev
        elif inter == 0:
            want = grow
        else:
            ebar = (w * nx + ny / w) / (2 * abs(inter))
            shrink = (1 - (k + 1) ** -0.3) * ebar
            want = min(shrink, grow)
            branches["shrink" if shrink < grow else "grow"] += 1
        assert abs(snaps[k].eta - want) <= 1e-9 * want, (name, k, snaps[k].eta, want)
        # the primal step of iteration k used t = eta_(k-1) / omega
        g = A.T @ y0 - lp.c
        free = (x1 > lp.l + 1e-9) & (x1 < lp.u - 1e-9) & (np.abs(g) > 1e-6)
        if np.any(free):
            t = dx[free] / (dc[free] ** 2 * g[free])
            np.testing.assert_allclose(t, eta_prev / w, rtol=1e-6)
    assert branches["shrink"] >= 1 and branches["grow"] >= 1, branches


def test_adaptive_trajectory_amplifies_rounding_constant_steps_do_not():
    """Why the adaptive option's fixed-iteration parity bar is set at a
    short horizon: the rule lets eta exceed the global step bound
    (t s |A~|^2 < 1) whenever the last move allowed it, so the map is no
    longer nonexpansive.  A perturbation of c of FP32 storage size (2^-24
    relative) moves the oracle's own iterate by more than 1e-3 after 100
    adaptive iterations on the general LP, while with constant steps it
    stays below 1e-6 (nonexpansive map)."""
    lp = I.workload(2, scale=0.002)
    rng = np.random.default_rng(0)
    c2 = lp.c * (1 + 2.0 ** -24 * rng.standard_normal(lp.n))
    for adaptive, lo, hi in ((True, 1e-3, np.inf), (False, 0.0, 1e-6)):
        a = oracle.pdhg(lp, tol=-1.0, iter_limit=100, restarts=False, adaptive=adaptive)
        b = oracle.pdhg(lp, tol=-1.0, iter_limit=100, restarts=False, adaptive=adaptive, c=c2)
        e = max(rel_err(a.x, b.x), rel_err(a.y, b.y))
        assert lo <= e <= hi, (adaptive, e)
    # after 10 adaptive iterations the same perturbation is still small
    a = oracle.pdhg(lp, tol=-1.0, iter_limit=10, restarts=False, adaptive=True)
    b = oracle.pdhg(lp, tol=-1.0, iter_limit=10, restarts=False, adaptive=True, c=c2)
    assert max(rel_err(a.x, b.x), rel_err(a.y, b.y)) <= 1e-5


# ------------------------------------------------------ restart to average
def _avg_cases():
    return [
        ("cover", I.set_cover(150, 400, seed=5)),
        ("knapsack", I.cover_knapsack(300, seed=6)),
        ("general", I.workload(2, scale=0.0005)),
        ("mixed", I.tiny_lp(np.random.default_rng(3), 40, 70, bounded=False)),
    ]


@pytest.mark.parametrize("case", range(4))
def test_running_average_is_the_mean_of_the_iterates(case):
    """With restarts off the running average only changes what a check
    returns, not the trajectory; it is the plain mean of the iterates
    x_1 .. x_K (snapshot runs without the average), through a check."""
    name, lp = _avg_cases()[case]
    K = 70
    snaps = [oracle.pdhg(lp, tol=-1.0, iter_limit=k, restarts=False) for k in range(1, K + 1)]
    r = oracle.pdhg(lp, tol=-1.0, iter_limit=K, restarts=False, restart_avg=True)
    xm = np.mean([s.x for s in snaps], axis=0)
    ym = np.mean([s.y for s in snaps], axis=0)
    assert rel_err(r.x_avg, xm) <= 1e-12 and rel_err(r.y_avg, ym) <= 1e-12, name
    # the same trajectory: at the iteration limit the current iterate is
    # the snapshot's (returned unless the mean wins)
    cur = snaps[-1]
    e_cur, e_avg = kkt_numpy(lp, cur.x, cur.y)["rel"], kkt_numpy(lp, r.x_avg, r.y_avg)["rel"]
    want_x, want_y = (r.x_avg, r.y_avg) if e_avg < e_cur else (cur.x, cur.y)
    np.testing.assert_allclose(r.x, want_x, rtol=0, atol=1e-12 * (1 + np.abs(want_x).max()))
    np.testing.assert_allclose(r.y, want_y, rtol=0, atol=1e-12 * (1 + np.abs(want_y).max()))
    assert abs(r.rel_kkt - min(e_cur, e_avg)) <= 1e-12 * max(1.0, r.rel_kkt)


def test_candidate_choice_goes_both_ways():
    """Across the cases and check counts the mean wins some checks and the
    current iterate others, so both branches of the rule are exercised."""
    wins = {"avg": 0, "cur": 0}
    for name, lp in _avg_cases():
        for K in (64, 128, 192, 320):
            r = oracle.pdhg(lp, tol=-1.0, iter_limit=K, restarts=False, restart_avg=True)
            cur = oracle.pdhg(lp, tol=-1.0, iter_limit=K, restarts=False)
            e_avg = kkt_numpy(lp, r.x_avg, r.y_avg)["rel"]
            e_cur = kkt_numpy(lp, cur.x, cur.y)["rel"]
            wins["avg" if e_avg < e_cur else "cur"] += 1
    assert min(wins.values()) >= 1, wins


@pytest.mark.parametrize("case", range(4))
def test_restart_to_the_candidate_restated(case):
    """The first check after the start always restarts (k - k_r = k >= 0.36
    k).  With the average on, the solve restarts at k = R to the candidate
    (the mean when its KKT error is lower), with the primal weight updated
    from the candidate's distance to the start point, and starts a new
    mean.  One iteration later the iterate equals one plain iteration from
    the candidate with that weight, and the new mean is that iterate."""
    name, lp = _avg_cases()[case]
    R = 64
    dr, dc = oracle.precondition(lp)
    start = oracle.pdhg(lp, tol=-1.0, iter_limit=0)
    # the candidate at k = R: returned by a run that stops there
    cand = oracle.pdhg(lp, tol=-1.0, iter_limit=R, restarts=False, restart_avg=True)
    dx = np.linalg.norm((cand.x - start.x) / dc)
    dy = np.linalg.norm((cand.y - start.y) / dr)
    w = start.omega
    if dx > 1e-10 and dy > 1e-10:
        w = np.exp(0.5 * np.log(dy / dx) + 0.5 * np.log(w))
    one = oracle.pdhg(lp, tol=-1.0, iter_limit=1, restarts=False, x0=cand.x, y0=cand.y, omega0=w)
    r = oracle.pdhg(lp, tol=-1.0, iter_limit=R + 1, restarts=True, restart_avg=True)
    assert r.restarts == 1 and abs(r.omega - w) <= 1e-12 * w, (name, r.omega, w)
    assert rel_err(r.x, one.x) <= 1e-12 and rel_err(r.y, one.y) <= 1e-12, name
    assert rel_err(r.x_avg, one.x) <= 1e-15 and rel_err(r.y_avg, one.y) <= 1e-15, name


def test_restart_to_average_takes_the_mean_on_some_case():
    """On at least one case the candidate at the first restart is the mean
    (so the restatement above covers restarting to it)."""
    took = 0
    for name, lp in _avg_cases():
        cand = oracle.pdhg(lp, tol=-1.0, iter_limit=64, restarts=False, restart_avg=True)
        cur = oracle.pdhg(lp, tol=-1.0, iter_limit=64, restarts=False)
        took += int(not np.array_equal(cand.x, cur.x))
    assert took >= 1


@pytest.mark.parametrize("adaptive", [False, True])
@pytest.mark.parametrize("case", range(4))
def test_restart_to_average_reaches_the_tolerance(case, adaptive):
    name, lp = _avg_cases()[case]
    r = oracle.pdhg(lp, tol=1e-6, iter_limit=200_000, restart_avg=True, adaptive=adaptive)
    assert r.status == oracle.OPTIMAL, name
    assert kkt_numpy(lp, r.x, r.y)["rel"] <= 1e-6 * (1 + 1e-9)


@pytest.mark.parametrize("case", range(4))
def test_termination_uses_the_candidate(case):
    """A tolerance between the mean's error and the current iterate's at a
    check where the mean wins stops the solve there, OPTIMAL, returning the
    mean; without the average the same tolerance does not stop it there."""
    name, lp = _avg_cases()[case]
    for K in (64, 128, 192, 256, 320):
        r = oracle.pdhg(lp, tol=-1.0, iter_limit=K, restarts=False, restart_avg=True)
        cur = oracle.pdhg(lp, tol=-1.0, iter_limit=K, restarts=False)
        e_avg = kkt_numpy(lp, r.x_avg, r.y_avg)["rel"]
        e_cur = kkt_numpy(lp, cur.x, cur.y)["rel"]
        earlier = [kkt_numpy(lp, s.x, s.y)["rel"] for s in
                   (oracle.pdhg(lp, tol=-1.0, iter_limit=k, restarts=False, restart_avg=True)
                    for k in range(0, K, 64))]
        if e_avg < e_cur and e_avg < min(earlier):
            tol = 0.5 * (e_avg + min(e_cur, min(earlier)))
            t = oracle.pdhg(lp, tol=tol, iter_limit=10 * K, restarts=False, restart_avg=True)
            assert t.status == oracle.OPTIMAL and t.iterations == K, (name, K, t.iterations)
            assert rel_err(t.x, r.x_avg) <= 1e-14
            p = oracle.pdhg(lp, tol=tol, iter_limit=K, restarts=False)
            assert p.status != oracle.OPTIMAL
            return
    pytest.skip(f"{name}: no check where the mean wins first")
