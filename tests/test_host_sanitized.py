"""The CPU-side C and C++ code under AddressSanitizer and UBSan: the oracle
(tests/host/oracle_driver.c), the library's host preparation
(tests/host/prep_driver.cpp + host_prep.cpp) and the library's host
fix-and-propagate (tests/host/fixprop_driver.cpp + fixprop.cpp), each built
with -fsanitize=address,undefined and -fno-sanitize-recover=all (any
finding aborts the run), on the shapes the pins and host tests use.  Every
sanitized run's output must equal the regular build's bit for bit, so the
checks in the other test files carry over to the sanitized code."""
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from paper_2307_03466_amd import instances as I
from lp_util import csr
from test_abi_host import SANITIZE, _run_prep

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
_EXE = {}


def _build(name):
    if name not in _EXE:
        d = tempfile.mkdtemp()
        exe = os.path.join(d, name)
        if name == "oracle_driver":
            cmd = ["gcc", "-O1", "-std=c11"] + SANITIZE + ["-o", exe,
                                                           os.path.join(ROOT, "tests", "host", "oracle_driver.c"),
                                                           "-lm"]
        else:
            cmd = ["g++", "-O1", "-std=c++17"] + SANITIZE + [
                "-o", exe, os.path.join(ROOT, "tests", "host", "fixprop_driver.cpp"),
                os.path.join(ROOT, "paper_2307_03466_amd", "csrc", "fixprop.cpp")]
        subprocess.check_call(cmd)
        _EXE[name] = exe
    return _EXE[name]


def _run(exe, payload):
    d = tempfile.mkdtemp()
    fin, fout = os.path.join(d, "in.bin"), os.path.join(d, "out.bin")
    with open(fin, "wb") as f:
        f.write(payload)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, fin, fout], capture_output=True, text=True, env=env)
    assert r.returncode == 0, r.stderr[-3000:]
    return open(fout, "rb").read()


def _lp_bytes(lp, with_c=True):
    parts = [np.array([lp.m, lp.n], np.int32), np.array([lp.nnz], np.int64),
             np.ascontiguousarray(lp.row_ptr, np.int64), np.ascontiguousarray(lp.col_idx, np.int32),
             np.ascontiguousarray(lp.val, np.float64)]
    if with_c:
        parts.append(np.ascontiguousarray(lp.c, np.float64))
    parts += [np.ascontiguousarray(lp.b, np.float64), np.ascontiguousarray(lp.senses, np.uint8),
              np.ascontiguousarray(lp.l, np.float64), np.ascontiguousarray(lp.u, np.float64),
              np.ascontiguousarray(lp.is_int, np.uint8)]
    return b"".join(p.tobytes() for p in parts)


def _oracle_cases():
    rng = np.random.default_rng(4)
    mixed = I.tiny_lp(rng, 30, 50, bounded=False)
    mixed.is_int = (rng.random(mixed.n) < 0.5).astype(np.uint8)
    return [("cover", I.set_cover(200, 500, seed=1), 0, 3),
            ("knapsack", I.cover_knapsack(400, seed=2), 1, 1),
            ("general", I.workload(2, scale=0.0005), 0, 7),
            ("skewed", I.workload(3, scale=0.0005), 1, 5),
            ("mixed", mixed, 0, 2),
            ("partition", I.set_partition(30, 90, seed=3), 1, 4)]


@pytest.mark.parametrize("k", range(6))
def test_oracle_under_sanitizers(k):
    name, lp, adaptive, K = _oracle_cases()[k]
    rng = np.random.default_rng(k)
    lo = np.where(np.isfinite(lp.l), lp.l, -3.0)
    hi = np.where(np.isfinite(lp.u), lp.u, lo + 3.0)
    xref = lo + rng.random(lp.n) * (hi - lo)
    tol, iters, R, restarts = 1e-6, 700, 64, 1
    payload = _lp_bytes(lp) + np.ascontiguousarray(xref, np.float64).tobytes() + \
        np.array([tol], np.float64).tobytes() + np.array([iters], np.int64).tobytes() + \
        np.array([R, restarts, adaptive, K], np.int32).tobytes()
    raw = _run(_build("oracle_driver"), payload)
    pos = 0

    def take(dt, cnt):
        nonlocal pos
        a = np.frombuffer(raw, dt, cnt, pos)
        pos += cnt * np.dtype(dt).itemsize
        return a
    x, y = take(np.float64, lp.n), take(np.float64, lp.m)
    st, nres = take(np.int32, 2)
    it = take(np.int64, 1)[0]
    rv, kk = take(np.float64, 8), take(np.float64, 8)
    xh, info = take(np.float64, lp.n), take(np.int32, 2)
    xb, info_b = take(np.float64, lp.n), take(np.int32, 2)
    mask = take(np.uint8, max(lp.m, 1))[: lp.m].astype(bool)
    ref = oracle.pdhg(lp, tol=tol, iter_limit=iters, check_period=R, restarts=bool(restarts),
                      adaptive=bool(adaptive))
    np.testing.assert_array_equal(x, ref.x)
    np.testing.assert_array_equal(y, ref.y)
    assert (st, nres, it) == (ref.status, ref.restarts, ref.iterations)
    np.testing.assert_array_equal(rv, [ref.rel_kkt, ref.rho_p, ref.rho_d, ref.rho_g, ref.pobj, ref.dobj,
                                       ref.omega, ref.eta])
    k2 = oracle.kkt(lp, x, y)
    np.testing.assert_array_equal(kk, [k2[f] for f in ("rel", "rho_p", "rho_d", "rho_g", "pobj", "dobj",
                                                        "bnorm", "cnorm")])
    a = oracle.fix_propagate(lp, xref)
    np.testing.assert_array_equal(xh, a[0])
    assert (bool(info[0]), int(info[1])) == a[1:]
    bb = oracle.fix_propagate_batched(lp, xref, K)
    np.testing.assert_array_equal(xb, bb[0])
    assert (bool(info_b[0]), int(info_b[1])) == bb[1:3]
    np.testing.assert_array_equal(mask, bb[3])


def _round_lib(lp, xref):
    raw = _run(_build("fixprop_driver"), _lp_bytes(lp, with_c=False) + np.ascontiguousarray(xref, np.float64).tobytes())
    xh = np.frombuffer(raw, np.float64, lp.n, 0)
    feas, ign = np.frombuffer(raw, np.int32, 2, 8 * lp.n)
    return xh, bool(feas), int(ign)


@pytest.mark.parametrize("k", range(6))
def test_library_rounding_under_sanitizers(k):
    """The library's sequential rounding (exact integer mode and the
    floating-point mode) equals the oracle's bit for bit."""
    name, lp, _, _ = _oracle_cases()[k]
    rng = np.random.default_rng(10 + k)
    for trial in range(3):
        lo = np.where(np.isfinite(lp.l), lp.l, -5.0)
        hi = np.where(np.isfinite(lp.u), lp.u, lo + 5.0)
        xref = lo + rng.random(lp.n) * (hi - lo)
        if trial == 1:
            xref = np.round(xref * 2) / 2
        a = oracle.fix_propagate(lp, xref)
        b = _round_lib(lp, xref)
        np.testing.assert_array_equal(a[0], b[0])
        assert a[1:] == b[1:], (name, trial)


@pytest.mark.parametrize("name", ["cover", "knapsack"])
def test_library_rounding_of_a_non_finite_iterate(name):
    """A failed solve's iterate (NaN or infinite entries) is never reported
    as a rounding that satisfies the rows: non-finite integer entries are
    fixed last to the lower end of their domain, and a row whose activity is
    not finite counts as violated.  The rounding stays integral and in
    bounds on the integer variables."""
    lp = I.set_cover(200, 500, seed=1) if name == "cover" else I.cover_knapsack(400, seed=2)
    rng = np.random.default_rng(3)
    x = rng.random(lp.n)
    x[rng.random(lp.n) < 0.3] = np.nan
    x[:3] = [np.inf, -np.inf, np.nan]
    xh, feas, _ = _round_lib(lp, x)
    ii = lp.is_int.astype(bool)
    assert np.all(np.isfinite(xh[ii])) and np.all(xh[ii] == np.round(xh[ii]))
    assert np.all(xh >= lp.l) and np.all(xh <= lp.u)
    # every entry NaN: the integers are fixed in index order to their lower
    # bound, propagation still repairs the covering rows, and a reported
    # feasible rounding really satisfies every row
    xh, feas, _ = _round_lib(lp, np.full(lp.n, np.nan))
    assert np.all(xh == np.round(xh))
    ax = csr(lp) @ xh
    held = np.where(lp.senses == ord("G"), ax >= lp.b - 1e-6 * (1 + abs(lp.b)),
                    np.where(lp.senses == ord("L"), ax <= lp.b + 1e-6 * (1 + abs(lp.b)),
                             abs(ax - lp.b) <= 1e-6 * (1 + abs(lp.b))))
    assert feas == bool(np.all(held))
    if name == "cover":
        assert feas
    # a continuous variable with a NaN reference keeps a NaN value, and the
    # rows it enters count as violated
    lp2 = I.set_cover(200, 500, seed=1)
    lp2.is_int = np.ones(lp2.n, np.uint8)
    lp2.is_int[7] = 0
    xr = np.ones(lp2.n)
    xr[7] = np.nan
    xh, feas, _ = _round_lib(lp2, xr)
    assert np.isnan(xh[7]) and not feas
    # with the NaN removed the same point is feasible (all ones covers every row)
    xr[7] = 1.0
    assert _round_lib(lp2, xr)[1]


@pytest.mark.parametrize("mode", ["plain", "blocked", "staged", "sliced"])
def test_host_preparation_under_sanitizers(mode):
    """CSC copy, exact packing and every tile plan built by the sanitized
    host preparation equal the regular build's output."""
    if mode in ("plain", "blocked"):
        lps = [I.workload(3, scale=0.002), I.workload(2, scale=0.0003)]
        extra = () if mode == "plain" else (4,)
        args = (lps, 1, 256, 64, extra)
    elif mode == "staged":
        lps = I.uneven_batch(count=8, lo=200, hi=6000, seed=3) + [I.workload(3, scale=0.0005)]
        args = (lps, 1, 1024, 1024, (0, 9000, 4096, 16384))
    else:
        lps = I.uneven_batch(count=10, lo=200, hi=9000, seed=5)
        args = (lps, 1, 1024, 1024, (0, 6000, 4096, 16384, 4))
    a = _run_prep(*args, sanitize=True)
    b = _run_prep(*args, sanitize=False)

    def flat(v):
        if isinstance(v, dict):
            return [w for k in sorted(v) for w in flat(v[k])]
        if isinstance(v, (list, tuple)):
            return [w for e in v for w in flat(e)]
        return [v]
    fa, fb = flat(a), flat(b)
    assert len(fa) == len(fb)
    for u, v in zip(fa, fb):
        if isinstance(u, np.ndarray):
            np.testing.assert_array_equal(u, v)
        else:
            assert u == v
