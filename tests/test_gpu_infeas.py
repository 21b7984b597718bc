"""Infeasibility certificates on the device (PDLP's reading: rays from the
moves between two checks) against the oracle and HiGHS: primal-infeasible
and unbounded families, per-pass kernels and fused windows, and no false
alarm on the feasible workloads."""
import numpy as np
import pytest

import oracle
from paper_2307_03466_amd import instances as I
from test_oracle_pdhg import _highs_status, _infeasible, _unbounded

pytestmark = pytest.mark.gpu
pdhg = pytest.importorskip("paper_2307_03466_amd.pdhg")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    pdhg.lib()


@pytest.mark.parametrize("fused", [1, 0])
@pytest.mark.parametrize("prec,itol", [(0, 1e-8), (1, 1e-8), (1, 1e-6)])
@pytest.mark.parametrize("kind,seed", [("primal", s) for s in range(4)] + [("dual", s) for s in range(4)])
def test_certificates_match_oracle(kind, seed, prec, itol, fused):
    lp = _infeasible(seed) if kind == "primal" else _unbounded(seed)
    want = 2 if kind == "primal" else 3
    if _highs_status(lp) != want:
        pytest.skip("construction did not give the intended status")
    ref = oracle.pdhg(lp, tol=1e-6, iter_limit=200_000, infeas_tol=itol)
    s = pdhg.solve(lp, tol=1e-6, iter_limit=200_000, precision=prec, infeas_tol=itol, fused_window=fused)
    status = s.result["status"]
    print(f"{kind} {seed} prec {prec} tol {itol} fused {fused}: device {status} at {s.result['iterations']}, "
          f"oracle {ref.status} at {ref.iterations}", flush=True)
    expect = pdhg.PRIMAL_INFEASIBLE if kind == "primal" else pdhg.DUAL_INFEASIBLE
    assert ref.status == expect
    assert status == expect
    if prec == 0:
        assert s.result["iterations"] == ref.iterations


@pytest.mark.parametrize("prec", [0, 1])
def test_mixed_batch_statuses(prec):
    """One handle: feasible instances finish OPTIMAL while the infeasible
    and unbounded ones stop with their certificates."""
    lps = [I.cover_knapsack(2000, seed=1), _infeasible(1), I.set_cover(200, 500, seed=4), _unbounded(2),
           I.cover_knapsack(800, seed=2)]
    with pdhg.Batch(lps, precision=prec) as b:
        res = b.solve(tol=1e-4, iter_limit=200_000, fused_window=0)
    got = [r["status"] for r in res]
    assert got == [pdhg.OPTIMAL, pdhg.PRIMAL_INFEASIBLE, pdhg.OPTIMAL, pdhg.DUAL_INFEASIBLE, pdhg.OPTIMAL], got


def test_certificates_off():
    lp = _infeasible(0)
    s = pdhg.solve(lp, tol=1e-6, iter_limit=3000, precision=0, infeas_tol=0.0)
    assert s.result["status"] == pdhg.ITERATION_LIMIT
