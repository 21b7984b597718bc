"""CPU-side checks of the C-ABI library: it loads, exports every symbol the
public header declares, rejects invalid input with -EINVAL before touching
any GPU, and its host preparation (block-diagonal concatenation, the
transposed copy, exact compact formats, tile plans) is correct."""
import ctypes
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

from paper_2307_03466_amd import instances as I
from paper_2307_03466_amd import pdhg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
           if f.endswith(".h")]
EINVAL = -22


def _declared_functions():
    names = set()
    for h in HEADERS:
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"\b(scylla_[a-z0-9_]+)\s*\(", txt):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(pdhg.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return pdhg.lib()


def test_library_exports_every_declared_symbol(L):
    declared = _declared_functions()
    assert declared, "no declarations parsed"
    assert declared == set(pdhg.EXPORTS), declared ^ set(pdhg.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", pdhg.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\b(scylla_[a-z0-9_]+)\b", out))
    missing = declared - exported
    assert not missing, missing


def test_params_default(L):
    p = pdhg.params()
    assert p.tol == 1e-4 and p.check_period == 64 and p.eta == 0.99 and p.restarts == 1
    assert p.adaptive == 0 and p.fused_window == 1 and p.infeas_tol == 1e-8
    assert p.stall_tol == 0.0 and p.stall_checks == 3
    assert p.restart_avg == 0 and p.compact == 1
    assert L.scylla_params_default(None) == EINVAL


def test_pump_params_default(L):
    """The paper's loop configuration, host rounding, one group."""
    o = pdhg.pump_params()
    assert o.rounds == 20 and o.eps_schedule == 1 and o.alpha == 0.9 and o.perturb == 1
    assert o.distance == 1 and o.pipeline == 0 and o.fp_batch == 0 and o.fp_max_rounds == 1000
    assert L.scylla_pump_params_default(None) == EINVAL


def test_device_rounding_rejects_a_null_handle(L):
    xh = np.zeros(4)
    info = np.zeros(2, dtype=np.int32)
    assert L.scylla_batch_fix_propagate(None, None, None, 4, 10, pdhg._ptr(xh), pdhg._ptr(info), None) == EINVAL


def _bad(lp, **changes):
    a = pdhg._LPArrays(lp)
    for k, v in changes.items():
        setattr(a, k, v)
    a.csr = pdhg.CSR(lp.m, lp.n, int(a.row_ptr[-1]), pdhg._ptr(a.row_ptr), pdhg._ptr(a.col_idx), pdhg._ptr(a.val))
    a.desc = pdhg.LPDesc(a.csr, pdhg._ptr(a.c), pdhg._ptr(a.b), pdhg._ptr(a.senses), pdhg._ptr(a.l), pdhg._ptr(a.u))
    return a


@pytest.mark.parametrize("case", ["ok", "col_range", "col_order", "nan_val", "sense", "l_gt_u",
                                  "inf_lower", "nan_c", "inf_b", "rowptr"])
def test_validation(L, case):
    lp = I.workload(1)
    if case == "ok":
        a = _bad(lp)
    elif case == "col_range":
        ci = lp.col_idx.copy(); ci[5] = lp.n
        a = _bad(lp, col_idx=ci)
    elif case == "col_order":
        ci = lp.col_idx.copy(); s = lp.row_ptr[3]; ci[s], ci[s + 1] = ci[s + 1], ci[s]
        a = _bad(lp, col_idx=ci)
    elif case == "nan_val":
        v = lp.val.copy(); v[7] = np.nan
        a = _bad(lp, val=v)
    elif case == "sense":
        s = lp.senses.copy(); s[2] = ord("X")
        a = _bad(lp, senses=s)
    elif case == "l_gt_u":
        l = lp.l.copy(); l[4] = 2.0
        a = _bad(lp, l=l)
    elif case == "inf_lower":
        l = lp.l.copy(); l[4] = np.inf
        a = _bad(lp, l=l)
    elif case == "nan_c":
        c = lp.c.copy(); c[0] = np.nan
        a = _bad(lp, c=c)
    elif case == "inf_b":
        b = lp.b.copy(); b[0] = np.inf
        a = _bad(lp, b=b)
    elif case == "rowptr":
        rp = lp.row_ptr.copy(); rp[5] = rp[6] + 1
        a = _bad(lp, row_ptr=rp)
    rc = L.scylla_validate_lp(ctypes.byref(a.desc))
    if case == "ok":
        assert rc == 0
    else:
        assert rc == EINVAL and L.scylla_last_error()
        # the one-shot solve rejects it before any device work and writes nothing
        x = np.full(lp.n, 7.0)
        y = np.full(lp.m, 7.0)
        res = pdhg.Result()
        rc2 = L.scylla_pdhg_solve(ctypes.byref(a.csr), pdhg._ptr(a.c), pdhg._ptr(a.b), pdhg._ptr(a.senses),
                                  pdhg._ptr(a.l), pdhg._ptr(a.u), ctypes.byref(pdhg.params()), None, None,
                                  pdhg._ptr(x), pdhg._ptr(y), ctypes.byref(res))
        assert rc2 == EINVAL
        assert np.all(x == 7.0) and np.all(y == 7.0)


def test_bad_params_rejected(L):
    lp = I.workload(1)
    for kw in (dict(check_period=0), dict(eta=1.5), dict(iter_limit=-1), dict(precision=7), dict(adaptive=2),
               dict(infeas_tol=-1.0), dict(infeas_tol=float("nan")), dict(stall_tol=-1.0),
               dict(stall_tol=float("inf")), dict(stall_tol=1e-6, stall_checks=0), dict(restart_avg=2),
               dict(compact=2), dict(compact=-1)):
        with pytest.raises(pdhg.ScyllaError) as e:
            pdhg.solve(lp, **kw)
        assert e.value.code == EINVAL


# ------------------------------------------------------------- host prep
_DRIVER = {}
SANITIZE = ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _driver(sanitize=False):
    """The host-preparation driver, optionally built with AddressSanitizer
    and UBSan (every finding aborts the run)."""
    if sanitize not in _DRIVER:
        exe = os.path.join(tempfile.mkdtemp(), "prep_driver")
        subprocess.check_call(["g++", "-O1", "-std=c++17"] + (SANITIZE if sanitize else []) + ["-o", exe,
                               os.path.join(ROOT, "tests", "host", "prep_driver.cpp"),
                               os.path.join(ROOT, "paper_2307_03466_amd", "csrc", "host_prep.cpp")])
        _DRIVER[sanitize] = exe
    return _DRIVER[sanitize]


def _run_prep(lps, precision, chunk, max_rows, extra=(), sanitize=False):
    d = tempfile.mkdtemp()
    fin, fout = os.path.join(d, "in.bin"), os.path.join(d, "out.bin")
    with open(fin, "wb") as f:
        f.write(np.array([len(lps), precision], dtype=np.int32).tobytes())
        for lp in lps:
            f.write(np.array([lp.m, lp.n], dtype=np.int32).tobytes())
            f.write(np.array([lp.nnz], dtype=np.int64).tobytes())
            for arr, dt in ((lp.row_ptr, np.int64), (lp.col_idx, np.int32), (lp.val, np.float64),
                            (lp.c, np.float64), (lp.b, np.float64), (lp.senses, np.uint8),
                            (lp.l, np.float64), (lp.u, np.float64)):
                f.write(np.ascontiguousarray(arr, dtype=dt).tobytes())
    subprocess.check_call([_driver(sanitize), fin, fout, str(chunk), str(max_rows)] + [str(a) for a in extra])
    raw = open(fout, "rb").read()
    pos = 0
    out = []

    def take(dt):
        nonlocal pos
        n = int(np.frombuffer(raw, np.int64, 1, pos)[0])
        pos += 8
        a = np.frombuffer(raw, dt, n, pos).copy()
        pos += n * np.dtype(dt).itemsize
        return a
    hdr = take(np.int32)
    ro, co = take(np.int32), take(np.int32)
    orient = [dict(ptr=take(np.int32), ent=take(np.uint32), v16=take(np.uint16), v32=take(np.float32),
                   v64=take(np.float64)) for _ in range(2)]
    plans = [dict(tiles=take(np.int32).reshape(-1, 4), longs=take(np.int32).reshape(-1, 4),
                  tb=take(np.int32), te=take(np.int32), lb=take(np.int32), le=take(np.int32)) for _ in range(2)]
    more = []
    if len(extra) >= 1 and int(extra[0]) < 0:
        more.append([dict(direct=take(np.int32), tiles=take(np.int32).reshape(-1, 4)) for _ in range(2)])
        return (hdr, ro, co, orient, plans) + tuple(more)
    if len(extra) >= 1 and int(extra[0]) > 0:
        more.append([dict(bounds=take(np.int32), bptr=take(np.int32), ent=take(np.uint32), v16=take(np.uint16),
                          v32=take(np.float32), v64=take(np.float64), tiles=take(np.int32).reshape(-1, 4),
                          longs=take(np.int32).reshape(-1, 4), ctiles=take(np.int32).reshape(-1, 4))
                     for _ in range(2)])
    if len(extra) >= 4:
        st = []
        for _ in range(2):
            d = dict(tiles=take(np.int32).reshape(-1, 4), sub=take(np.int32).reshape(-1, 4),
                     sublongs=take(np.int32).reshape(-1, 4), staged=take(np.int32),
                     rest=take(np.int32).reshape(-1, 4), restlongs=take(np.int32).reshape(-1, 4))
            if len(extra) >= 5:
                hd = take(np.int32)
                d["sliced"] = dict(S=int(hd[0]), max_slice=int(hd[1]), inst=take(np.int32), Sq=take(np.int32),
                                   bptr=take(np.int32),
                                   ent=take(np.uint32), tiles=take(np.int32).reshape(-1, 4),
                                   sub=take(np.int32).reshape(-1, 4), ctiles=take(np.int32).reshape(-1, 4))
            st.append(d)
        more.append(st)
    if more:
        return (hdr, ro, co, orient, plans) + tuple(more)
    return hdr, ro, co, orient, plans


def _decode(o, hdr, which, fmt):
    shift, mask = (hdr[1], hdr[2]) if which == 0 else (hdr[3], hdr[4])
    mask = np.uint32(int(mask) & 0xFFFFFFFF)
    if fmt == 0:
        idx = (o["ent"] & mask).astype(np.int64)
        val = (o["ent"].view(np.int32) >> shift).astype(np.float64)
    else:
        idx = o["ent"].astype(np.int64)
        if fmt == 1:
            val = (o["v16"].astype(np.uint32) << 16).view(np.float32).astype(np.float64)
        elif fmt == 2:
            val = o["v32"].astype(np.float64)
        else:
            val = o["v64"]
    return idx, val


def _block_diag(lps):
    import scipy.sparse as sps
    return sps.block_diag([sps.csr_matrix((lp.val, lp.col_idx, lp.row_ptr), shape=(lp.m, lp.n))
                           for lp in lps], format="csr")


@pytest.mark.parametrize("kind,precision,expect_fmt", [
    ("cover_knapsack", 1, 0), ("skewed", 1, 0), ("general", 0, 3), ("bf16", 1, 1), ("real", 1, 2)])
def test_orientations_and_formats(kind, precision, expect_fmt):
    rng = np.random.default_rng(0)
    if kind == "cover_knapsack":
        lps = I.uneven_batch(count=5, lo=50, hi=400, seed=1)
    elif kind == "skewed":
        lps = [I.workload(3, scale=0.001)]
    elif kind == "general":
        lps = [I.workload(2, scale=0.0005), I.workload(2, scale=0.0003)]
    else:
        lp = I.workload(2, scale=0.0005)
        lp.val = lp.val * (1000.5 if kind == "bf16" else np.pi)
        if kind == "bf16":
            # BF16-exact values too large for the packed integer range
            lp.val = np.sign(lp.val) * 2.0 ** rng.integers(24, 30, size=lp.val.size)
        lps = [lp]
    hdr, ro, co, orient, plans = _run_prep(lps, precision, 256, 64)
    assert hdr[0] == expect_fmt
    ref = _block_diag(lps)
    # CSR
    idx, val = _decode(orient[0], hdr, 0, hdr[0])
    np.testing.assert_array_equal(orient[0]["ptr"], ref.indptr)
    np.testing.assert_array_equal(idx, ref.indices)
    rnd = (lambda v: v.astype(np.float32).astype(np.float64)) if hdr[0] == 2 else (lambda v: v)
    np.testing.assert_array_equal(val, rnd(ref.data))
    # CSC = CSR of the transpose with increasing rows per column
    refT = ref.T.tocsr()
    refT.sort_indices()
    idx, val = _decode(orient[1], hdr, 1, hdr[0])
    np.testing.assert_array_equal(orient[1]["ptr"], refT.indptr)
    np.testing.assert_array_equal(idx, refT.indices)
    np.testing.assert_array_equal(val, rnd(refT.data))
    np.testing.assert_array_equal(ro, np.cumsum([0] + [lp.m for lp in lps]))
    np.testing.assert_array_equal(co, np.cumsum([0] + [lp.n for lp in lps]))


@pytest.mark.parametrize("chunk,max_rows", [(256, 64), (1024, 1024), (64, 8)])
def test_tile_plan_covers_every_row_once(chunk, max_rows):
    lps = [I.workload(3, scale=0.002), I.workload(2, scale=0.0003)]
    hdr, ro, co, orient, plans = _run_prep(lps, 1, chunk, max_rows)
    for o, plan, off in ((orient[0], plans[0], ro), (orient[1], plans[1], co)):
        ptr = o["ptr"]
        rows = ptr.size - 1
        covered = np.zeros(rows, dtype=np.int64)
        seg_cover = {}
        for t, (a, b, inst, slot) in enumerate(plan["tiles"]):
            assert plan["tb"][inst] <= t < plan["te"][inst]
            if slot < 0:
                assert off[inst] <= a < b <= off[inst + 1]
                assert b - a <= max_rows
                assert ptr[b] - ptr[a] <= chunk
                covered[a:b] += 1
            else:
                assert 0 < b - a <= chunk
                seg_cover[slot] = (a, b)
        for q, (row, slot0, nseg, inst) in enumerate(plan["longs"]):
            assert plan["lb"][inst] <= q < plan["le"][inst]
            length = ptr[row + 1] - ptr[row]
            assert length > chunk and nseg == -(-length // chunk)
            spans = [seg_cover[slot0 + s] for s in range(nseg)]
            assert spans[0][0] == ptr[row] and spans[-1][1] == ptr[row + 1]
            assert all(spans[s][1] == spans[s + 1][0] for s in range(nseg - 1))
            covered[row] += 1
        assert np.all(covered == 1)


def test_nnz_limit_rejected_before_reading_arrays(L):
    rp = np.array([0, 2 ** 31], dtype=np.int64)
    ci = np.zeros(1, dtype=np.int32)
    v = np.zeros(1)
    one = np.ones(1)
    sense = np.array([ord("G")], dtype=np.uint8)
    csr = pdhg.CSR(1, 1, 2 ** 31, pdhg._ptr(rp), pdhg._ptr(ci), pdhg._ptr(v))
    desc = pdhg.LPDesc(csr, pdhg._ptr(one), pdhg._ptr(one), pdhg._ptr(sense), pdhg._ptr(one), pdhg._ptr(one))
    assert L.scylla_validate_lp(ctypes.byref(desc)) == EINVAL
    assert "nnz" in L.scylla_last_error().decode()


def _decode_idx(ent, hdr, which, fmt):
    if fmt != 0:
        return ent.astype(np.int64)
    mask = np.uint32(int(hdr[2] if which == 0 else hdr[4]) & 0xFFFFFFFF)
    return (ent & mask).astype(np.int64)


def _check_cover(ptr_rows, plan_tiles, plan_longs, rows_wanted, chunk=None, max_rows=None):
    """Normal tiles + long rows cover every wanted row once."""
    covered = np.zeros(ptr_rows.size - 1, dtype=np.int64)
    segs = {}
    for a, b, inst, slot in plan_tiles:
        if slot < 0:
            covered[a:b] += 1
            if max_rows:
                assert b - a <= max_rows
            if chunk:
                assert ptr_rows[b] - ptr_rows[a] <= chunk
        else:
            segs[slot] = (a, b)
    for row, slot0, nseg, inst in plan_longs:
        spans = [segs[slot0 + s] for s in range(nseg)]
        assert spans[0][0] == ptr_rows[row] and spans[-1][1] == ptr_rows[row + 1]
        covered[row] += 1
    assert np.all(covered[rows_wanted] == 1) and np.all(np.delete(covered, rows_wanted) == 0)


@pytest.mark.parametrize("B", [2, 4, 8])
def test_gather_blocked_layout(B):
    """Every row's nonzeros are split by gathered-index slice without loss or
    reordering, tiles of block b sit where workgroups run on XCDs x with
    x mod B = b, and the block tiles plus long sub-rows cover every
    (block, row) once; combine tiles cover every row once."""
    lps = [I.workload(3, scale=0.002), I.workload(2, scale=0.0003)]
    chunk, max_rows = 256, 64
    hdr, ro, co, orient, plans, blk = _run_prep(lps, 1, chunk, max_rows, extra=(B,))
    for which in (0, 1):
        o, bl = orient[which], blk[which]
        rows = o["ptr"].size - 1
        g = (co if which == 0 else ro)[-1]
        np.testing.assert_array_equal(bl["bounds"], [(g * b) // B for b in range(B + 1)])
        idx = _decode_idx(o["ent"], hdr, which, hdr[0])
        bidx = _decode_idx(bl["ent"], hdr, which, hdr[0])
        bptr = bl["bptr"].reshape(B, rows + 1)
        for i in np.random.default_rng(which).choice(rows, size=min(rows, 400), replace=False):
            parts = []
            for b in range(B):
                seg = bidx[bptr[b, i]:bptr[b, i + 1]]
                assert np.all((seg >= bl["bounds"][b]) & (seg < bl["bounds"][b + 1]))
                parts.append(bl["ent"][bptr[b, i]:bptr[b, i + 1]])
            np.testing.assert_array_equal(np.concatenate(parts), o["ent"][o["ptr"][i]:o["ptr"][i + 1]])
        # tiles: XCD placement and coverage per block
        for p, (a, bnd, z, slot) in enumerate(bl["tiles"]):
            if slot >= 0 or bnd > a:
                assert (p % 8) % B == (z >> 24)
        for b in range(B):
            tb = [t for t in bl["tiles"] if (t[2] >> 24) == b and (t[3] >= 0 or t[1] > t[0])]
            lb = [l for l in bl["longs"] if (l[3] >> 24) == b]
            # long sub-rows reference segment slots of all blocks; keep only this block's
            slots = {l[1] + s for l in lb for s in range(l[2])}
            tb = [t for t in tb if t[3] < 0 or t[3] in slots]
            nonempty = np.flatnonzero(np.diff(bptr[b]) > 0)
            covered = np.zeros(rows, dtype=np.int64)
            for a, bnd, z, slot in tb:
                if slot < 0:
                    covered[a:bnd] += 1
                    assert bptr[b, bnd] - bptr[b, a] <= chunk
            for row, *_ in lb:
                covered[row] += 1
            assert np.all(covered[nonempty] == 1)
        off = ro if which == 0 else co
        cov = np.zeros(rows, dtype=np.int64)
        for a, bnd, q, _ in bl["ctiles"]:
            assert off[q] <= a < bnd <= off[q + 1] and bnd - a <= 256
            cov[a:bnd] += 1
        assert np.all(cov == 1)


def test_lds_staged_plan():
    """Instances qualify when their gathered vector has at most max_vec
    elements and no row exceeds a sub-tile; their sub-tiles cover every row
    once and are grouped in order into tiles of about group_nnz nonzeros;
    the other instances are covered by normal tiles."""
    lps = I.uneven_batch(count=8, lo=200, hi=6000, seed=3) + [I.workload(3, scale=0.0005)]
    chunk, max_rows, max_vec, sub_chunk, group = 1024, 1024, 9000, 4096, 16384
    out = _run_prep(lps, 1, chunk, max_rows, extra=(0, max_vec, sub_chunk, group))
    hdr, ro, co, orient, plans, st = out
    for which in (0, 1):
        o, sp = orient[which], st[which]
        ptr = o["ptr"]
        off, gof = (ro, co) if which == 0 else (co, ro)
        for q in range(len(lps)):
            rl = np.diff(ptr[off[q]:off[q + 1] + 1])
            want = gof[q + 1] - gof[q] <= max_vec and off[q + 1] > off[q] and rl.max(initial=0) <= sub_chunk
            assert bool(sp["staged"][q]) == want, (which, q)
        staged_rows = np.concatenate([np.arange(off[q], off[q + 1]) for q in range(len(lps)) if sp["staged"][q]]
                                     + [np.zeros(0, dtype=np.int64)])
        rest_rows = np.setdiff1d(np.arange(ptr.size - 1), staged_rows)
        _check_cover(ptr, sp["sub"], sp["sublongs"], staged_rows, chunk=sub_chunk, max_rows=4096)
        assert sp["sublongs"].size == 0
        _check_cover(ptr, sp["rest"], sp["restlongs"], rest_rows, chunk=chunk)
        # staged tiles: consecutive sub-tile ranges of one instance, in order,
        # ceil(nnz / group) of them per instance with about equal counts
        nxt, per = {}, {}
        for s0, s1, q, _ in sp["tiles"]:
            assert sp["staged"][q] and s1 > s0
            assert nxt.get(q, s0) == s0
            nxt[q] = s1
            subs = sp["sub"][s0:s1]
            assert np.all(subs[:, 2] == q)
            per.setdefault(q, []).append(sum(ptr[b] - ptr[a] for a, b, _, _ in subs))
        for q, nzs in per.items():
            total = ptr[off[q + 1]] - ptr[off[q]]
            k = max(1, -(-total // group))
            assert len(nzs) == k and sum(nzs) == total, (q, nzs)
            assert max(nzs) <= total / k + sub_chunk and min(nzs) >= total / k - sub_chunk, (q, nzs)


def test_lds_sliced_plan():
    """Instances too long for LDS but at most max_slices LDS capacities long
    get their gathered range cut into S_q = ceil(length / capacity) equal
    slices: each row's nonzeros are regrouped by slice without loss or
    reordering, every one of the instance's slices has sub-tiles covering
    each of its rows once (and slices beyond S_q none), and combine tiles
    cover those rows once."""
    lps = I.uneven_batch(count=10, lo=200, hi=9000, seed=5)
    chunk, max_rows, max_vec, sub_chunk, group, max_slices = 1024, 1024, 6000, 4096, 16384, 4
    hdr, ro, co, orient, plans, st = _run_prep(lps, 1, chunk, max_rows,
                                               extra=(0, max_vec, sub_chunk, group, max_slices))
    seen, counts = 0, set()
    for which in (0, 1):
        o, sp = orient[which], st[which]
        x = sp["sliced"]
        ptr = o["ptr"]
        rows = ptr.size - 1
        off, gof = (ro, co) if which == 0 else (co, ro)
        glen = np.diff(gof)
        want = np.array([not sp["staged"][q] and max_vec < glen[q] <= max_slices * max_vec
                         and np.diff(ptr[off[q]:off[q + 1] + 1]).max(initial=0) <= sub_chunk
                         and off[q + 1] > off[q] for q in range(len(lps))])
        np.testing.assert_array_equal(x["inst"].astype(bool), want)
        if not want.any():
            assert x["S"] == 0
            continue
        seen += 1
        S = x["S"]
        Sq = x["Sq"]
        assert S == -(-glen[want].max() // max_vec)
        np.testing.assert_array_equal(Sq, np.where(want, -(-glen // max_vec), 0))
        counts.update(Sq[want].tolist())
        assert x["max_slice"] <= max_vec
        idx = _decode_idx(o["ent"], hdr, which, hdr[0])
        xidx = _decode_idx(x["ent"], hdr, which, hdr[0])
        bptr = x["bptr"].reshape(S, rows + 1)
        cover = [np.zeros(rows, dtype=np.int64) for _ in range(S)]
        per = {}
        for s0, s1, z, kind in x["tiles"]:
            q, s = z & 0xFFFFFF, z >> 24
            assert kind == -2 and want[q] and s < Sq[q]
            nz = 0
            for a, b, qq, _ in x["sub"][s0:s1]:
                assert qq == q and off[q] <= a <= b <= off[q + 1]
                assert bptr[s, b] - bptr[s, a] <= sub_chunk and b - a <= 4096
                cover[s][a:b] += 1
                nz += bptr[s, b] - bptr[s, a]
            per.setdefault((q, s), []).append(nz)
        # ceil(nnz / group) tiles of about equal counts per (instance, slice)
        for (q, s), nzs in per.items():
            total = bptr[s, off[q + 1]] - bptr[s, off[q]]
            k = max(1, -(-total // group))
            assert len(nzs) == k and sum(nzs) == total
            assert max(nzs) <= total / k + sub_chunk and min(nzs) >= total / k - sub_chunk
        for q in np.flatnonzero(want):
            r = np.arange(off[q], off[q + 1])
            n_s = Sq[q]
            lo = [gof[q] + (glen[q] * s) // n_s for s in range(n_s + 1)]
            for s in range(S):
                assert np.all(cover[s][r] == (1 if s < n_s else 0))
                if s >= n_s:
                    assert np.all(bptr[s, off[q]:off[q + 1] + 1] == bptr[s, off[q]])
            for i in r[:: max(1, r.size // 50)]:
                parts = []
                for s in range(n_s):
                    seg = xidx[bptr[s, i]:bptr[s, i + 1]]
                    assert np.all((seg >= lo[s]) & (seg < lo[s + 1]))
                    parts.append(x["ent"][bptr[s, i]:bptr[s, i + 1]])
                np.testing.assert_array_equal(np.concatenate(parts), o["ent"][ptr[i]:ptr[i + 1]])
        other = np.flatnonzero(~want)
        for q in other:
            assert np.all(bptr[:, off[q]:off[q + 1] + 1] == bptr[:, off[q]:off[q] + 1])
        cov = np.zeros(rows, dtype=np.int64)
        for a, b, q, _ in x["ctiles"]:
            assert want[q] and off[q] <= a < b <= off[q + 1] and b - a <= 256
            cov[a:b] += 1
        rows_w = np.concatenate([np.arange(off[q], off[q + 1]) for q in np.flatnonzero(want)])
        assert np.all(cov[rows_w] == 1) and cov.sum() == rows_w.size
    assert seen >= 1 and len(counts) > 1  # the cases mix slice counts


@pytest.mark.parametrize("lanes_min,group", [(1, 16384), (4, 3000)])
def test_direct_staged_tiles(lanes_min, group):
    """Direct staged tiles: instances with rows whose gathered vector has at
    most max_vec elements qualify; their rows are covered once, in order, by
    ceil(nnz / group_nnz) runs of whole rows per instance with about equal
    nonzero counts; the lanes per row are the smallest power of two >= lanes_min (at most 64)
    with which the longest row of the tile takes at most four rounds of K
    nonzeros per lane (K = 8, 4, 2 for at least 1-2, 4, 8 lanes)."""
    lps = I.uneven_batch(count=10, lo=200, hi=9000, seed=5) + [I.workload(3, scale=0.002)]
    max_vec = 4000
    hdr, ro, co, orient, plans, dr = _run_prep(lps, 1, 1024, 1024, extra=(-6, max_vec, group, lanes_min))
    for which in (0, 1):
        ptr = orient[which]["ptr"]
        off, gof = (ro, co) if which == 0 else (co, ro)
        want = np.array([np.diff(gof)[q] <= max_vec and off[q + 1] > off[q] for q in range(len(lps))])
        np.testing.assert_array_equal(dr[which]["direct"].astype(bool), want)
        assert want.any() and not want.all()
        cover = np.zeros(ptr.size - 1, dtype=np.int64)
        last, per = {}, {}
        for r0, r1, q, L in dr[which]["tiles"]:
            assert want[q] and off[q] <= r0 < r1 <= off[q + 1]
            assert last.get(q, off[q]) == r0
            last[q] = r1
            lens = np.diff(ptr[r0:r1 + 1])
            per.setdefault(q, []).append(int(lens.sum()))
            Lw = max(1, lanes_min)
            k = 8 if lanes_min <= 2 else (4 if lanes_min <= 4 else 2)  # nonzeros per lane and round
            while Lw < 64 and lens.max() > 4 * k * Lw:
                Lw *= 2
            assert L == Lw
            cover[r0:r1] += 1
        for q in np.flatnonzero(want):
            assert last[q] == off[q + 1]
            assert np.all(cover[off[q]:off[q + 1]] == 1)
            total = ptr[off[q + 1]] - ptr[off[q]]
            k = max(1, -(-total // group))
            longest = np.diff(ptr[off[q]:off[q + 1] + 1]).max()
            nzs = per[q]
            assert sum(nzs) == total
            # k runs unless a zero-length tail run was merged away
            assert len(nzs) <= k and max(nzs) <= total / k + longest, (q, nzs, k)
        assert cover.sum() == sum(off[q + 1] - off[q] for q in np.flatnonzero(want))
