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


def test_restart_rule_and_weight_update_restated_from_checks():
    """At each check after the start, with E the relative KKT error of the
    current point, E_r its value at the last restart (the start counts) and
    E_p at the previous check, the solve restarts iff E <= 0.2 E_r, or
    E <= 0.8 E_r and E > E_p, or k - k_r >= 0.36 k.  At a restart the primal
    weight becomes the geometric mean of the old weight and |dy~| / |dx~|,
    with dx~ = (x - x_r) / d_c and dy~ = (y - y_r) / d_r the moves since the
    last restart point (unchanged if either is <= 1e-10)."""
    decisive = {"0.2": 0, "0.8": 0, "0.36": 0, "none": 0, "weight": 0}
    for name, lp, R in _restart_cases():
        dr, dc = oracle.precondition(lp)
        full = oracle.pdhg(lp, tol=1e-7, iter_limit=60 * R, check_period=R)
        nchk = full.iterations // R
        snaps = [oracle.pdhg(lp, tol=-1.0, iter_limit=c * R, check_period=R) for c in range(nchk + 1)]
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
    assert min(decisive.values()) >= 1, decisive


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
