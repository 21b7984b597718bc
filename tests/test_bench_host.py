"""Host checks of bench.py: the one-GPU contract and the byte models the
bandwidth figures are computed from."""
import os
import subprocess
import sys

import bench
from paper_2307_03466_amd import instances as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def _lp(rows, n):
    """LP from a list of rows [(column, value), ...] (other fields unused)."""
    import numpy as np
    ptr = np.cumsum([0] + [len(r) for r in rows]).astype(np.int64)
    cols = np.array([c for r in rows for c, _ in r], np.int32)
    vals = np.array([v for r in rows for _, v in r], np.float64)
    m = len(rows)
    return I.LP(m=m, n=n, row_ptr=ptr, col_idx=cols, val=vals, c=np.zeros(n), b=np.zeros(m),
                senses=np.full(m, ord("G"), np.uint8), l=np.zeros(n), u=np.ones(n),
                is_int=np.zeros(n, np.uint8))


def test_canonical_bytes_by_hand():
    """Per nonzero 4 B of index plus 0 (pattern: every value of the row is
    +-1), 2 (BF16-exact integers up to 256) or 4 (anything else) value
    bytes; pointers; 28 B per column (x, c, l, u, D_c^2 read, x and x_bar
    written) and one gather of y in the column pass; 17 B per row (y, b,
    D_r^2, sense read, y written) and one gather of x_bar in the row pass;
    a 4-byte split offset per column when mixed row formats are cheaper
    than one format for all rows; FP64: 12 B per nonzero, 56 / 33 B."""
    m, n = 6, 4
    # one BF16 row (2 nonzeros), four pattern rows (4 each), one FP32 row (2)
    pat = [(0, 1.0), (1, -1.0), (2, 1.0), (3, 1.0)]
    lp = _lp([[(0, 3.0), (2, -200.0)], pat, pat, pat, pat, [(0, 0.5), (3, 1.0)]], n)
    per_row = 2 * 6 + 16 * 4 + 2 * 8
    uniform = 20 * 8
    assert per_row + 4 * n < uniform
    row, col = bench.canonical_pass_bytes([lp])
    assert row == per_row + 4 * (m + 1) + 17 * m + 4 * n
    assert col == per_row + 4 * n + 4 * (n + 1) + 28 * n + 4 * m
    # all BF16 but one short pattern row: one format for all rows is cheaper
    lp2 = _lp([[(0, 3.0), (2, -20.0), (3, 7.0)], [(1, 1.0)], [(0, 5.0), (4, 2.0), (1, 9.0)]], 5)
    m2, n2 = 3, 5
    row, col = bench.canonical_pass_bytes([lp2])
    assert row == 7 * 6 + 4 * (m2 + 1) + 17 * m2 + 4 * n2
    assert col == 7 * 6 + 4 * (n2 + 1) + 28 * n2 + 4 * m2
    # batches add up instance by instance; FP64 ignores the formats
    r2, c2 = bench.canonical_pass_bytes([lp, lp2])
    assert (r2, c2) == tuple(a + b for a, b in zip(bench.canonical_pass_bytes([lp]),
                                                   bench.canonical_pass_bytes([lp2])))
    row, col = bench.canonical_pass_bytes([lp], fp64=True)
    assert row == 20 * 12 + 4 * (m + 1) + 33 * m + 8 * n
    assert col == 20 * 12 + 4 * (n + 1) + 56 * n + 8 * m
    assert bench.canonical_bytes([lp]) == sum(bench.canonical_pass_bytes([lp]))


def test_canonical_bytes_of_the_workloads():
    """The byte model's figures for the workloads: the 1M x 2M LP moves
    128.05 MB in the column pass, 217 MB per FP32 iteration and 421 MB per
    FP64 iteration; the skewed LP (70 % pattern rows) about 237 MB; the pump
    batch about 275 MB."""
    lp = I.workload(2)
    row, col = bench.canonical_pass_bytes([lp])
    assert abs(col / 1e6 - 128.05) < 0.01
    assert abs((row + col) / 1e6 - 217) < 1
    assert abs(bench.canonical_bytes([lp], True) / 1e6 - 421) < 1
    assert abs(bench.canonical_bytes([I.workload(3)]) / 1e6 - 237) < 3
    assert abs(bench.canonical_bytes(I.workload(5)) / 1e6 - 275) < 2


def test_pass_bytes_follow_the_storage_format():
    info = dict(m_total=10, n_total=20, nnz_total=100, format=0)  # packed integers: no value bytes
    row, col = bench.pass_bytes(info, 4)
    assert row == 100 * 4 + 4 * 11 + 4 * 20 + 17 * 10
    assert col == 100 * 4 + 4 * 21 + 4 * 10 + 28 * 20
    info["format"] = 3  # FP64 values
    row, col = bench.pass_bytes(info, 8)
    assert row == 100 * 12 + 4 * 11 + 8 * 20 + 33 * 10
    assert col == 100 * 12 + 4 * 21 + 8 * 10 + 56 * 20


def test_pump_workload_shape():
    lps = I.pump_batch(2, 2000, 4000)
    assert [(lp.m, lp.n) for lp in lps] == [(2000, 4000)] * 2


def test_pass_kernel_names_match_the_traffic_table():
    """The kernels bench.py looks up for the headline LP's tuned layouts
    (normal column pass and 4-block row pass on 256-thread tiles of 1024
    nonzeros, both with cacheable matrix loads) are named as in the counter
    table, which was taken on that workload; a layout the table does not hold
    gives no traffic figure rather than another kernel's."""
    import json
    table = json.load(open(os.path.join(ROOT, "profiles", "pmc_traffic.json")))["kernels"]
    info = dict(format=0, col_blocks=0, row_blocks=4, col_chunk=1024, row_chunk=1024,
                col_tile_threads=256, row_tile_threads=256, col_cached=1, row_cached=1)
    for is_col in (True, False):
        names = bench.pass_kernels(info, is_col)
        assert names and all(n in table for n in names), names
    assert bench.pass_kernels(info, True) == ["void k_pass<float, 8, 1, 256, 4>(PassArgs<float>, int)"]
    assert bench.pass_kernels(info, False) == ["void k_bpart<float, float, 8, 256, 4>(PassArgs<float>, int, int)",
                                               "void k_bcombine<float, 0>(PassArgs<float>, int)"]
    if json.load(open(os.path.join(ROOT, "profiles", "pmc_traffic.json")))["kernels_hip_sha256"] == \
            bench.kernels_sha256():
        assert bench.measured_traffic(bench.pass_kernels(info, True)) > 0
        assert bench.measured_traffic(bench.pass_kernels(info, False)) > 0
    # the non-temporal variant of the same layout is another kernel
    info["col_cached"] = 0
    assert bench.pass_kernels(info, True) == ["void k_pass<float, 0, 1, 256, 4>(PassArgs<float>, int)"]
    assert bench.measured_traffic(bench.pass_kernels(info, True)) is None
    info.update(col_tile_threads=1024, col_chunk=8192)
    assert bench.pass_kernels(info, True) == ["void k_pass<float, 0, 1, 1024, 8>(PassArgs<float>, int)"]
    assert bench.measured_traffic(["void k_pass<float, 0, 1, 1024, 8>(PassArgs<float>, int)"]) is None
    info["col_blocks"] = -1
    assert bench.pass_kernels(info, True) is None
