"""Parity at the workloads' full sizes, in the launch configuration the
benchmark times (autotuned layout), through the C ABI.

100 iterations with restarts off against the FP64 oracle (full vectors:
the oracle finishes them in seconds), FP32 bar 1e-4 and FP64 bar 1e-10;
device KKT against the oracle's KKT of the returned iterate; batches are
checked on sampled instances plus invariants on all of them."""
import numpy as np
import pytest

import oracle
from paper_2307_03466_amd import instances as I
from lp_util import rel_err

pytestmark = pytest.mark.gpu
pdhg = pytest.importorskip("paper_2307_03466_amd.pdhg")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    pdhg.lib()


def _solve100(lps, prec):
    with pdhg.Batch(lps, precision=prec) as b:
        b.solve(tol=1e-300, iter_limit=0)  # autotunes the layout, as the benchmark does
        info = b.info()
        res = b.solve(tol=1e-300, iter_limit=100, restarts=0)
        sols = [b.solution(i) for i in range(len(lps))]
    return info, res, sols


@pytest.mark.parametrize("k", [2, 3])
def test_single_lp_full_size(k):
    lp = I.workload(k)
    print(f"workload {k}: m={lp.m} n={lp.n} nnz={lp.nnz}", flush=True)
    ref = oracle.pdhg(lp, tol=-1.0, iter_limit=100, restarts=False)
    for prec, bar in ((1, 1e-4), (0, 1e-10)):
        info, res, sols = _solve100([lp], prec)
        print("layout", info, flush=True)
        x, y = sols[0]
        assert res[0]["iterations"] == 100
        ex, ey = rel_err(x, ref.x), rel_err(y, ref.y)
        print(f"prec {prec}: e_x={ex:.3e} e_y={ey:.3e}", flush=True)
        assert max(ex, ey) <= bar
        assert np.all(x >= lp.l) and np.all(x <= lp.u)
        assert np.all(y[lp.senses == ord("G")] >= 0) and np.all(y[lp.senses == ord("L")] <= 0)
        kk = oracle.kkt(lp, x, y)
        assert abs(res[0]["rel_kkt"] - kk["rel"]) <= 1e-9 * max(1, kk["rel"])


@pytest.mark.parametrize("k", [4, 5])
def test_batch_full_size(k):
    lps = I.workload(k)
    print(f"workload {k}: {len(lps)} instances, nnz={sum(l.nnz for l in lps)}", flush=True)
    info, res, sols = _solve100(lps, 1)
    print("layout", info, flush=True)
    for i, lp in enumerate(lps):
        x, y = sols[i]
        assert res[i]["iterations"] == 100
        assert np.all(x >= lp.l) and np.all(x <= lp.u)
        assert np.all(y[lp.senses == ord("G")] >= 0) and np.all(y[lp.senses == ord("L")] <= 0)
    sample = sorted(set(np.linspace(0, len(lps) - 1, 6).astype(int).tolist()
                        + [int(np.argmax([l.m for l in lps]))]))
    for i in sample:
        lp = lps[i]
        ref = oracle.pdhg(lp, tol=-1.0, iter_limit=100, restarts=False)
        x, y = sols[i]
        assert max(rel_err(x, ref.x), rel_err(y, ref.y)) <= 1e-4, i
        kk = oracle.kkt(lp, x, y)
        assert abs(res[i]["rel_kkt"] - kk["rel"]) <= 1e-9 * max(1, kk["rel"])


def test_pump_full_size_two_rounds():
    lps = I.workload(5)
    with pdhg.Batch(lps, precision=1) as b:
        recs, xh = b.pump(rounds=2, alpha=0.9, tol=1e-4, iter_limit=200_000)
        x, y = b.solution(len(lps) - 1)
    assert len(recs) == 2 and len(recs[0]) == len(lps)
    assert np.all(xh == np.round(xh)) and np.all((xh == 0) | (xh == 1))
    for rnd in recs:
        for r in rnd:
            assert r["status"] == pdhg.OPTIMAL and r["rel_kkt"] <= 1e-4
    off = np.cumsum([0] + [lp.n for lp in lps])
    for q in (0, len(lps) // 2, len(lps) - 1):
        xo, feas, ign = oracle.fix_propagate(lps[q], xh[off[q]:off[q + 1]])
        # the returned rounding is a fixed point of the rounding (integral, sound)
        if feas:
            np.testing.assert_array_equal(xo, xh[off[q]:off[q + 1]])
