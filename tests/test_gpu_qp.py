"""Diagonal-Hessian QP objectives on the device (Section 5: PDHG for QPs
with a diagonal Hessian, and the L2 distance of the objective update)
against the oracle, through the C ABI: fixed-iteration parity under every
layout and in the fused window, termination at the oracle's iteration
count, and the complete loop with the L2 distance in a closed FP64 loop."""
import numpy as np
import pytest

import oracle
from paper_2307_03466_amd import instances as I
from lp_util import kkt_numpy, parity_err, rel_err

pytestmark = pytest.mark.gpu
pdhg = pytest.importorskip("paper_2307_03466_amd.pdhg")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    pdhg.lib()


def _cases():
    rng = np.random.default_rng(17)
    out = {}
    for name, lp in (("general", I.workload(2, scale=0.002)), ("skewed_longrows", I.workload(3, scale=0.01)),
                     ("knapsack", I.cover_knapsack(3000, seed=7)), ("cover200", I.workload(1)),
                     ("mixed", I.tiny_lp(np.random.default_rng(3), 40, 70, bounded=False))):
        q = np.where(rng.random(lp.n) < 0.5, rng.random(lp.n) * 3, 0.0)
        out[name] = (lp, q)
    return out


CASES = ["general", "skewed_longrows", "knapsack", "cover200", "mixed"]


@pytest.mark.parametrize("fused", [0, 1])
@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("prec,bar", [(0, 1e-10), (1, 1e-4)])
def test_qp_fixed_iteration_parity(name, prec, bar, fused):
    lp, q = _cases()[name]
    ref = oracle.pdhg(lp, tol=-1.0, iter_limit=100, restarts=False, q=q)
    with pdhg.Batch([lp], precision=prec) as b:
        b.set_quadratic(0, q)
        r = b.solve(tol=1e-300, iter_limit=100, restarts=0, fused_window=fused, autotune=0)[0]
        x, y = b.solution(0)
    e = parity_err(x, y, ref.x, ref.y)
    print(f"qp {name} prec {prec} fused {fused}: e={e:.2e}", flush=True)
    assert r["iterations"] == 100 and e <= bar
    k = oracle.kkt(lp, x, y, q=q)
    assert abs(r["rel_kkt"] - k["rel"]) <= 1e-9 * max(1, k["rel"])


@pytest.mark.parametrize("layout", [(0, 4, 0, 16), (4, 8, 2, 8), (-1, 8, -1, 8), (-2, 8, -2, 8), (-3, 8, -3, 8)])
def test_qp_parity_under_every_layout(layout):
    lps = [I.general_lp(m=20_000, n=50_000, seed=31), I.cover_knapsack(500, seed=1),
           I.cover_knapsack(24_000, seed=2)]
    rng = np.random.default_rng(5)
    qs = [rng.random(lp.n) * 2 for lp in lps]
    with pdhg.Batch(lps, precision=0) as b:
        b.set_layout(*layout)
        for i, q in enumerate(qs):
            b.set_quadratic(i, q)
        res = b.solve(tol=1e-300, iter_limit=100, restarts=0, fused_window=0)
        sols = [b.solution(i) for i in range(len(lps))]
    for i, lp in enumerate(lps):
        ref = oracle.pdhg(lp, tol=-1.0, iter_limit=100, restarts=False, q=qs[i])
        assert res[i]["iterations"] == 100
        assert parity_err(sols[i][0], sols[i][1], ref.x, ref.y) <= 1e-10, (layout, i)


@pytest.mark.parametrize("name", ["general", "knapsack", "mixed"])
def test_qp_termination_matches_oracle(name):
    lp, q = _cases()[name]
    ref = oracle.pdhg(lp, tol=1e-6, iter_limit=500_000, q=q)
    s_b = pdhg.Batch([lp], precision=0)
    s_b.set_quadratic(0, q)
    r = s_b.solve(tol=1e-6, iter_limit=500_000)[0]
    x, y = s_b.solution(0)
    s_b.close()
    assert r["status"] == pdhg.OPTIMAL and ref.status == oracle.OPTIMAL
    assert r["iterations"] == ref.iterations
    assert kkt_numpy(lp, x, y, q=q)["rel"] <= 1e-6 * (1 + 1e-6)
    assert abs(r["primal_obj"] - ref.pobj) <= 1e-6 * (1 + abs(ref.pobj))


def test_qp_reset_and_validation():
    lp, q = _cases()["knapsack"]
    with pdhg.Batch([lp], precision=0) as b:
        with pytest.raises(pdhg.ScyllaError):
            b.set_quadratic(0, -np.ones(lp.n))
        with pytest.raises(pdhg.ScyllaError):
            b.set_quadratic(0, np.full(lp.n, np.nan))
        b.set_quadratic(0, q)
        b.set_quadratic(0, None)  # back to the LP
        r = b.solve(tol=1e-300, iter_limit=100, restarts=0, autotune=0)[0]
        x, y = b.solution(0)
    ref = oracle.pdhg(lp, tol=-1.0, iter_limit=100, restarts=False)
    assert parity_err(x, y, ref.x, ref.y) <= 1e-10


def _general_int(seed, m=10, n=16):
    rng = np.random.default_rng(seed)
    lp = I.tiny_lp(rng, m, n)
    lp.is_int = np.ones(lp.n, dtype=np.uint8)
    lp.l, lp.u = np.zeros(lp.n), np.full(lp.n, 6.0)
    xs = np.round(rng.random(lp.n) * 6)
    A = np.zeros((lp.m, lp.n))
    A[np.repeat(np.arange(lp.m), np.diff(lp.row_ptr)), lp.col_idx] = lp.val
    lp.b = A @ xs - np.where(lp.senses == ord("L"), -1.0, np.where(lp.senses == ord("G"), 1.0, 0.0))
    return lp


def test_l2_loop_matches_oracle_fp64():
    """General integers (no L1 form without auxiliary variables): the
    device's complete loop with the L2 distance follows the oracle's closed
    loop round by round."""
    lps = [_general_int(s) for s in range(5)]
    opts = dict(rounds=8, distance=2, perturb=0, early_exit=0, eps_schedule=0)
    with pdhg.Batch(lps, precision=0) as b:
        recs, outs, xo = b.pump_ex(pump=opts, tol=1e-6, iter_limit=100_000)
    off = np.cumsum([0] + [lp.n for lp in lps])
    for q, lp in enumerate(lps):
        kind, K, point, rr = oracle.scylla(lp, rounds=8, distance="l2", cycle_perturb=False, early_exit=False,
                                           eps_sched=False, tol=1e-6, iter_limit=100_000, instance=q)
        o = outs[q]
        print(q, o, (kind, K), [r["iterations"] for r in rr], flush=True)
        assert (o["found_kind"], o["found_round"], o["rounds_run"]) == (kind, K, len(rr))
        for k, r in enumerate(rr):
            assert recs[k][q]["iterations"] == r["iterations"], (q, k)
            assert recs[k][q]["xhat_feasible"] == int(r["xhat_feasible"])
        xq = xo[off[q]:off[q + 1]]
        if kind == 1:
            assert rel_err(xq, point) <= 1e-9
        elif point is not None:
            np.testing.assert_array_equal(xq, point)


def test_l2_loop_on_binaries_with_perturbation():
    lps = [I.set_partition(12, 40, seed=s) for s in range(4)] + [I.cover_knapsack(300, seed=0)]
    with pdhg.Batch(lps, precision=1) as b:
        recs, outs, xo = b.pump_ex(pump=dict(rounds=20, distance=2, seed=3))
    off = np.cumsum([0] + [lp.n for lp in lps])
    for q, lp in enumerate(lps):
        xq = xo[off[q]:off[q + 1]]
        if outs[q]["found_kind"]:
            assert oracle.mip_feasible(lp, xq)
        else:
            assert outs[q]["rounds_run"] == 20
    assert outs[-1]["found_kind"] and outs[-1]["found_round"] == 1
    with pdhg.Batch(lps[:1], precision=1) as b:
        with pytest.raises(pdhg.ScyllaError):
            b.pump_ex(pump=dict(distance=3))
