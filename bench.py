#!/usr/bin/env python
"""Benchmark of the PDHG hot path on one MI355X.

Headline workload: the single large general LP (m = 1,000,000 rows,
n = 2,000,000 columns, ~10M nonzeros, geometric row lengths, integer
coefficients in [-20, 20]), synthetic and seeded.  A step is one check
window of the solver: the FP64 KKT check and decision plus R = 64 PDHG
iterations (column pass + row pass), replayed from one hipGraph.
value = PDHG iterations/s of the FP32 path with the problem resident in HBM.

Also reported: the plain FP64 path on the same LP, both paths' time to
relative KKT <= 1e-4, the dominant kernel's HBM roofline (algorithmic bytes
per launch over its HIP-event launch time) and its random-gather ceiling
(measured live), the other four workloads (tiny set cover, skewed LP,
256-instance batch, 64-instance pump loop), and the FP64 CPU oracle on a
bounded sample as a baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "PDHG iter/s + HBM GB/s vs peak; FP32-batched vs FP64 plain at 1e-4 rel KKT"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pass_bytes(info: dict, vb: int):
    """Algorithmic bytes of one launch of each pass: every matrix word/value
    and pointer read once, the gathered vector read once, the pass's own
    vectors read / written once (row pass: y, b, D_r^2, sense, y out; column
    pass: x, c, l, u, D_c^2, x out, x_bar out)."""
    m, n, nnz = info["m_total"], info["n_total"], info["nnz_total"]
    vbytes = {0: 0, 1: 2, 2: 4, 3: 8}[info["format"]]
    row = nnz * (4 + vbytes) + 4 * (m + 1) + vb * n + (4 * vb + 1) * m
    col = nnz * (4 + vbytes) + 4 * (n + 1) + vb * m + 7 * vb * n
    return row, col


def row_value_bytes(lp):
    """Value bytes v per nonzero of each row in the canonical byte model:
    0 for a pattern row (every value +1 or -1: the sign fits in the index
    word), 2 when every value is an integer with |a| <= 256 (exact in BF16),
    4 otherwise."""
    import numpy as np
    a = np.abs(np.asarray(lp.val, dtype=np.float64))
    rows = np.repeat(np.arange(lp.m), np.diff(lp.row_ptr))
    not_pat = np.bincount(rows, weights=(a != 1.0), minlength=lp.m) > 0
    not_bf = np.bincount(rows, weights=((a != np.round(a)) | (a > 256)), minlength=lp.m) > 0
    return np.where(not_bf, 4, np.where(not_pat, 2, 0)), np.diff(lp.row_ptr)


def canonical_pass_bytes(lps, fp64=False):
    """Canonical bytes of one launch of the row pass (dual step) and of the
    column pass (primal step), summed over the instances: every matrix
    entry (4-byte index + v value bytes, v by row format; 8 on the FP64
    path) and pointer read once, one full gather of the other vector, and
    the pass's own vectors -- row pass 17 B per row (y, b, D_r^2, sense
    read, y written; 33 B in FP64), column pass 28 B per column (x, c, l, u,
    D_c^2 read, x and x_bar written; 56 B in FP64).  An instance's matrix
    takes the cheaper of its two exact encodings: one format for every row
    (the widest any row needs), or each row in its own format with a 4-byte
    split offset per column in the column pass.  This is the per-iteration
    model of the hot-path scope (pattern 4 B, BF16 6 B per nonzero),
    independent of the layout the library picks."""
    import numpy as np
    row = col = 0
    for lp in lps:
        m, n, nnz = lp.m, lp.n, lp.nnz
        if fp64:
            mat = 12 * nnz
            row += mat + 4 * (m + 1) + 33 * m + 8 * n
            col += mat + 4 * (n + 1) + 56 * n + 8 * m
            continue
        v, lens = row_value_bytes(lp)
        uniform = (4 + int(v[lens > 0].max(initial=0))) * nnz
        per_row = int(np.sum((4 + v) * lens))
        split = 4 * n if per_row + 4 * n < uniform else 0
        mat = per_row if split else uniform
        row += mat + 4 * (m + 1) + 17 * m + 4 * n
        col += mat + split + 4 * (n + 1) + 28 * n + 4 * m
    return int(row), int(col)


def canonical_bytes(lps, fp64=False):
    """Canonical bytes of one PDHG iteration (both passes)."""
    return sum(canonical_pass_bytes(lps, fp64))


def pass_kernels(info, is_col):
    """Names (as rocprofv3 prints them) of the FP32 kernels one pass
    launches in the layout `info` describes, or None for the LDS-staged
    layouts."""
    blocks = info["col_blocks"] if is_col else info["row_blocks"]
    # the kernels' format parameter carries the cached-load flag (8)
    fmt = info["format"] | (8 if info.get("col_cached" if is_col else "row_cached") else 0)
    nt = info["col_tile_threads" if is_col else "row_tile_threads"] or 256
    ept = (info["col_chunk"] if is_col else info["row_chunk"]) // nt
    if blocks > 0:  # gather-blocked pass: partial sums, then the combine with the epilogue
        return [f"void k_bpart<float, float, {fmt}, {nt}, {ept}>(PassArgs<float>, int, int)",
                f"void k_bcombine<float, {1 if is_col else 0}>(PassArgs<float>, int)"]
    if blocks == 0:
        return [f"void k_pass<float, {fmt}, {1 if is_col else 0}, {nt}, {ept}>(PassArgs<float>, int)"]
    return None


def kernels_sha256() -> str:
    """Hash of the kernel source the traffic counters were taken on."""
    import hashlib
    with open(os.path.join(ROOT, "paper_2307_03466_amd", "csrc", "kernels.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(kernels):
    """HBM bytes per launch of a pass made of `kernels` (sum over them of
    FETCH_SIZE x calibration + WRITE_SIZE per dispatch) from
    profiles/pmc_traffic.json, or None when the counters were taken on
    another version of the kernel source."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernels_hip_sha256") != kernels_sha256():
        return None
    total = 0
    for kernel in kernels:
        k = d["kernels"].get(kernel)
        if not k or "fetch_bytes" not in k or "write_bytes" not in k:
            return None
        total += k["fetch_bytes"] + k["write_bytes"]
    return int(total)


def probe_gather_ms(vec_bytes, gathers):
    """Average ms of one launch of `gathers` random 4-byte gathers from a
    vector of `vec_bytes` bytes (the passes' ceiling), measured by the
    probe library built beside the solver (csrc/gather_probe.hip)."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2307_03466_amd", "libgather_probe.so"))
    lib.gather_probe_ms.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]
    lib.gather_probe_ms.restype = ctypes.c_int
    ms = ctypes.c_double()
    rc = lib.gather_probe_ms(int(vec_bytes), int(gathers), ctypes.byref(ms))
    if rc != 0:
        raise RuntimeError(f"gather probe failed ({rc})")
    return ms.value


def timed_steps(batch, steps, R, **kw):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = batch.solve(tol=1e-300, iter_limit=steps * R, check_period=R, **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert all(r["iterations"] == steps * R for r in res), res[0]
    return dt, res


def measure(pdhg, lps, prec, steps, warmup, R, to_tol, tol_time_limit, passes=True):
    """Iteration rate (timed windows), pass timings and time to 1e-4 of one
    handle holding `lps`."""
    b = pdhg.Batch(lps, precision=prec)
    setup = b.solve(tol=1e-300, iter_limit=0)[0]["setup_seconds"]  # includes the tuning run
    b.solve(tol=1e-300, iter_limit=max(1, warmup) * R, check_period=R)
    info = b.info()
    dt, _ = timed_steps(b, steps, R)
    its = steps * R
    rec = dict(info=info, setup_s=setup, seconds=dt, iters=its, iter_per_s=its / dt,
               ms_per_step=1000 * dt / steps)
    canon = canonical_pass_bytes(lps, fp64=prec != pdhg.FP32)
    rec.update(canon_row=canon[0], canon_col=canon[1], canon_iter=sum(canon))
    if passes:
        ms_row, ms_col = b.time_passes(20)
        rb, cb = pass_bytes(info, 4 if prec == pdhg.FP32 else 8)
        rec.update(ms_row=ms_row, ms_col=ms_col, bytes_row=rb, bytes_col=cb)
    if to_tol:
        # the iteration rate with restarts to the average (the means folded in
        # by every pass, a second check per window)
        b.solve(tol=1e-300, iter_limit=R, check_period=R, restart_avg=1)
        dt_avg, _ = timed_steps(b, steps, R, restart_avg=1)
        rec["iter_per_s_avg"] = its / dt_avg
        # constant and adaptive steps, each without and with restarts to the
        # average
        for key, adaptive, avg in (("to_tol", 0, 0), ("to_tol_adaptive", 1, 0), ("to_tol_avg", 0, 1),
                                   ("to_tol_avg_adaptive", 1, 1)):
            res = b.solve(tol=1e-4, iter_limit=2_000_000, time_limit_s=tol_time_limit, adaptive=adaptive,
                          restart_avg=avg)
            rec[key] = dict(status=max(r["status"] for r in res), optimal=sum(r["status"] == 1 for r in res),
                            count=len(res), iterations_max=max(r["iterations"] for r in res),
                            iterations_sum=sum(r["iterations"] for r in res),
                            seconds=res[0]["solve_seconds"], rel_kkt_max=max(r["rel_kkt"] for r in res))
            # the handle's setup (upload, CSC copy, packing, preconditioning,
            # tuning) happened in its first solve, timed in setup_s
    b.close()
    return rec


def host_cpu():
    """CPU model and the number of cores this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def cpu_baseline(lp, iters):
    """The FP64 oracle on the headline LP, one core: iter/s over a bounded
    number of iterations (its preconditioning and start check subtracted)."""
    import oracle
    t0 = time.perf_counter()
    oracle.pdhg(lp, tol=-1.0, iter_limit=0)
    t1 = time.perf_counter()
    oracle.pdhg(lp, tol=-1.0, iter_limit=iters)
    t2 = time.perf_counter()
    per_iter = ((t2 - t1) - (t1 - t0)) / iters
    model, ncpu = host_cpu()
    return dict(value=round(1.0 / per_iter, 3), unit="iter/s", cores=1, kind="oracle", cpu_model=model,
                nproc=ncpu,
                sample=f"{iters} FP64 PDHG iterations of the same 1M x 2M LP by the single-threaded C "
                       f"oracle (preconditioning and the start check subtracted; {t2 - t0:.1f} s of CPU)")


def cpu_baselines_other(instances, sel, iters_batched=300, iters_skewed=100):
    """The FP64 oracle on the other workloads: single LPs on one core, the
    batched ones with one instance per core on all cores (the C oracle
    releases the interpreter lock).  Each on a bounded sample."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    model, ncpu = host_cpu()
    out = dict(cpu_model=model, nproc=ncpu)
    if "1" in sel:
        lp = instances.workload(1)
        t = time.perf_counter()
        r = oracle.pdhg(lp, tol=1e-4, iter_limit=200_000)
        el = time.perf_counter() - t
        t = time.perf_counter()
        xh, feas, _ = oracle.fix_propagate(lp, r.x)
        fp = time.perf_counter() - t
        out["set_cover_200x500"] = dict(value=round(r.iterations / el, 1), unit="iter/s", cores=1,
                                        iterations_to_tol=r.iterations, seconds_to_tol=round(el, 4),
                                        rounding_seconds=round(fp, 5), rounding_feasible=feas,
                                        sample="whole solve to 1e-4 relative KKT, then fix-and-propagate")
    if "3" in sel:
        lp = instances.workload(3)
        t0 = time.perf_counter()
        oracle.pdhg(lp, tol=-1.0, iter_limit=0)
        t1 = time.perf_counter()
        oracle.pdhg(lp, tol=-1.0, iter_limit=iters_skewed)
        t2 = time.perf_counter()
        out["skewed_lp_500kx1M"] = dict(value=round(iters_skewed / max((t2 - t1) - (t1 - t0), 0.5 * (t2 - t1)), 3),
                                        unit="iter/s",
                                        cores=1, sample=f"{iters_skewed} iterations (setup subtracted)")
        del lp
    for k, key in ((4, "batch_256_uneven"), (5, "pump_64x20k")):
        if str(k) not in sel:
            continue
        lps = instances.workload(k)
        workers = min(ncpu, len(lps))

        def run(lp, it):
            oracle.pdhg(lp, tol=-1.0, iter_limit=it, restarts=False)
        with ThreadPoolExecutor(workers) as ex:
            t0 = time.perf_counter()
            list(ex.map(lambda lp: run(lp, 0), lps))
            t1 = time.perf_counter()
            list(ex.map(lambda lp: run(lp, iters_batched), lps))
            t2 = time.perf_counter()
        # the setup run's time subtracted (never more than half the run)
        per_iter = max((t2 - t1) - (t1 - t0), 0.5 * (t2 - t1)) / iters_batched
        out[key] = dict(value=round(1.0 / per_iter, 2), unit="batch-iter/s", cores=workers,
                        instance_iter_per_s=round(len(lps) / per_iter, 1),
                        sample=f"{iters_batched} iterations of all {len(lps)} instances, one instance per core "
                               f"on {workers} cores (setup subtracted)")
        del lps
    return out


def rounding_comparison(pdhg, b, lps):
    """Fix-and-propagate of the first pump round's iterate (the LP
    relaxations solved to 1e-4): the sequential procedure on the host (one
    call per instance, 16 threads) against the batched procedure on the
    device (one workgroup per instance) at K = 1 and K = 64, with the number
    of roundings that satisfy every row."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    b.solve(tol=1e-4, iter_limit=200_000)
    x = b.x_all()
    offs = np.cumsum([0] + [lp.n for lp in lps])

    def host(q):
        return pdhg.fix_propagate(lps[q], x[offs[q]:offs[q + 1]])
    with ThreadPoolExecutor(16) as ex:
        t = time.perf_counter()
        res = list(ex.map(host, range(len(lps))))
        host_s = time.perf_counter() - t
    rec = dict(host_sequential=dict(seconds=round(host_s, 4), threads=16,
                                    feasible=int(sum(r[1] for r in res))))
    for K in (1, 64):
        ts = []
        for _ in range(2):
            t = time.perf_counter()
            xh, feas, nign, _ = b.fix_propagate(K)
            ts.append(time.perf_counter() - t)
        rec[f"device_batched_K{K}"] = dict(seconds=round(min(ts), 4), feasible=int(feas.sum()),
                                           ignored_rows=int(nign.sum()))
    return rec


def other_workloads(pdhg, instances, args, R):
    out = {}
    sel = set(args.workloads.split(","))
    if "1" in sel:  # tiny set cover, FP64, latency-bound; then rounding on the host
        lp = instances.workload(1)
        r = measure(pdhg, [lp], pdhg.FP64, 50, 3, R, args.to_tol, 30, passes=False)
        s = pdhg.solve(lp, tol=1e-4, iter_limit=200_000, precision=pdhg.FP64)
        t = time.perf_counter()
        xh, feas, ign = pdhg.fix_propagate(lp, s.x)
        out["set_cover_200x500_fp64"] = dict(iter_per_s=round(r["iter_per_s"], 1),
                                             canonical_GBps=round(r["canon_iter"] * r["iter_per_s"] / 1e9, 2),
                                             to_tol=r.get("to_tol"),
                                             to_tol_adaptive_steps=r.get("to_tol_adaptive"),
                                             to_tol_restart_avg=r.get("to_tol_avg"),
                                             to_tol_restart_avg_adaptive_steps=r.get("to_tol_avg_adaptive"),
                                             rounding_s=round(time.perf_counter() - t, 6),
                                             rounding_feasible=feas, rounded_obj=float(lp.c @ xh))
        log(f"w1: {r['iter_per_s']:,.0f} iter/s to_tol={r.get('to_tol')} adaptive={r.get('to_tol_adaptive')} "
            f"rounding feasible={feas}")
    if "3" in sel:  # skewed LP, FP32 and FP64
        lp = instances.workload(3)
        rec = {}
        for prec, tag in ((pdhg.FP32, "fp32"), (pdhg.FP64, "fp64")):
            r = measure(pdhg, [lp], prec, 20, 2, R, args.to_tol, args.tol_time_limit)
            rb, cb = r["bytes_row"], r["bytes_col"]
            rec[tag] = dict(iter_per_s=round(r["iter_per_s"], 1), ms_row=round(r["ms_row"], 4),
                            ms_col=round(r["ms_col"], 4), row_GBps=round(rb / r["ms_row"] / 1e6, 1),
                            col_GBps=round(cb / r["ms_col"] / 1e6, 1),
                            row_canonical_GBps=round(r["canon_row"] / r["ms_row"] / 1e6, 1),
                            col_canonical_GBps=round(r["canon_col"] / r["ms_col"] / 1e6, 1),
                            canonical_GBps=round(r["canon_iter"] * r["iter_per_s"] / 1e9, 1),
                            to_tol=r.get("to_tol"),
                            to_tol_adaptive_steps=r.get("to_tol_adaptive"),
                            to_tol_restart_avg=r.get("to_tol_avg"),
                            to_tol_restart_avg_adaptive_steps=r.get("to_tol_avg_adaptive"),
                            iter_per_s_restart_avg=round(r["iter_per_s_avg"], 1) if "iter_per_s_avg" in r else None,
                            layout=[r["info"]["row_blocks"], r["info"]["row_chunk"], r["info"]["col_blocks"],
                                    r["info"]["col_chunk"]], long_rows=r["info"]["long_rows"])
            log(f"w3 {tag}: {r['iter_per_s']:,.0f} iter/s to_tol={r.get('to_tol')} adaptive={r.get('to_tol_adaptive')}")
        out["skewed_lp_500kx1M"] = rec
        del lp
    if "4" in sel:  # 256 uneven LPs in one handle; FP64 plain = one instance at a time
        lps = instances.workload(4)
        r = measure(pdhg, lps, pdhg.FP32, 20, 2, R, args.to_tol, args.tol_time_limit)
        rec = dict(count=len(lps), batch_iter_per_s=round(r["iter_per_s"], 1),
                   instance_iter_per_s=round(r["iter_per_s"] * len(lps), 1), ms_row=round(r["ms_row"], 4),
                   ms_col=round(r["ms_col"], 4), to_tol_fp32_batched=r.get("to_tol"),
                   to_tol_fp32_batched_adaptive_steps=r.get("to_tol_adaptive"),
                   to_tol_fp32_batched_restart_avg=r.get("to_tol_avg"),
                   to_tol_fp32_batched_restart_avg_adaptive_steps=r.get("to_tol_avg_adaptive"),
                   batch_iter_per_s_restart_avg=round(r["iter_per_s_avg"], 1) if "iter_per_s_avg" in r else None,
                   setup_seconds=round(r["setup_s"], 3),
                   canonical_bytes_per_iter=r["canon_iter"],
                   canonical_GBps=round(r["canon_iter"] * r["iter_per_s"] / 1e9, 1),
                   row_canonical_GBps=round(r["canon_row"] / r["ms_row"] / 1e6, 1),
                   col_canonical_GBps=round(r["canon_col"] / r["ms_col"] / 1e6, 1),
                   row_frac_of_peak=round(r["canon_row"] / r["ms_row"] / 1e6 / HBM_PEAK_GBPS, 3),
                   col_frac_of_peak=round(r["canon_col"] / r["ms_col"] / 1e6 / HBM_PEAK_GBPS, 3),
                   iteration_frac_of_peak=round(r["canon_iter"] * r["iter_per_s"] / 1e9 / HBM_PEAK_GBPS, 3))
        log(f"w4 fp32 batched: {r['iter_per_s']:,.0f} batch-iter/s to_tol={r.get('to_tol')} "
            f"adaptive={r.get('to_tol_adaptive')}")
        if args.fp64_plain_batch and args.to_tol:
            # the plain FP64 path, one instance at a time through the one-shot
            # call: its solve_seconds (iterations only) summed, and its
            # setup_seconds (upload, CSC copy, preconditioning, graph) apart
            t = time.perf_counter()
            done, solve_s, setup_s = 0, 0.0, 0.0
            for lp in lps:
                s = pdhg.solve(lp, tol=1e-4, iter_limit=2_000_000, precision=pdhg.FP64, autotune=0)
                done += s.result["status"] == 1
                solve_s += s.result["solve_seconds"]
                setup_s += s.result["setup_seconds"]
                if time.perf_counter() - t > args.tol_time_limit * 3:
                    break
            n_done = lps.index(lp) + 1
            el = time.perf_counter() - t
            rec["to_tol_fp64_plain_sequential"] = dict(solve_seconds=round(solve_s, 3),
                                                       setup_seconds=round(setup_s, 3),
                                                       wall_seconds=round(el, 3), instances=n_done, optimal=done)
            if n_done == len(lps) and r["to_tol"]["optimal"] == len(lps):
                # like for like: iteration time against iteration time, and
                # with each side's setup added
                rec["speedup_fp32_batched_vs_fp64_plain_to_tol"] = round(solve_s / r["to_tol"]["seconds"], 2)
                rec["speedup_fp32_batched_vs_fp64_plain_to_tol_with_setup"] = round(
                    (solve_s + setup_s) / (r["to_tol"]["seconds"] + r["setup_s"]), 2)
                for key, name in (("to_tol_adaptive", "adaptive"), ("to_tol_avg", "restart_avg"),
                                  ("to_tol_avg_adaptive", "restart_avg_adaptive")):
                    if r[key]["optimal"] == len(lps):
                        rec[f"speedup_fp32_batched_{name}_vs_fp64_plain_to_tol"] = round(
                            solve_s / r[key]["seconds"], 2)
            log(f"w4 fp64 plain sequential: {n_done} instances, {solve_s:.2f} s solving + {setup_s:.2f} s setup")
        out["batch_256_uneven"] = rec
        del lps
    if "5" in sel:  # pump loop: 64 x (20k x 40k), 20 rounds
        lps = instances.workload(5)
        b = pdhg.Batch(lps, precision=pdhg.FP32)
        out["rounding_64x20k"] = rounding_comparison(pdhg, b, lps)
        log(f"w5 rounding: {out['rounding_64x20k']}")
        t = time.perf_counter()
        recs, xh = b.pump(rounds=args.pump_rounds, alpha=0.9, tol=1e-4, iter_limit=200_000)
        el = time.perf_counter() - t
        its = [max(r["iterations"] for r in rnd) for rnd in recs]
        inst_its = sum(r["iterations"] for rnd in recs for r in rnd)
        def per_group(key):  # one value per device solve group and round
            return sum(next(r[key] for r in rnd if r["group"] == g)
                       for rnd in recs for g in {r["group"] for r in rnd})
        solve_s, rounding_s, tune_s = (per_group(k) for k in ("solve_seconds", "rounding_seconds",
                                                                "tune_seconds"))
        first = [next((k + 1 for k in range(len(recs)) if recs[k][q]["xhat_feasible"]), None)
                 for q in range(len(lps))]
        out["pump_64x20k"] = dict(rounds=len(recs), seconds=round(el, 3), solve_seconds=round(solve_s, 3),
                                  rounding_seconds=round(rounding_s, 3), tune_seconds=round(tune_s, 3),
                                  groups=len({r["group"] for r in recs[0]}),
                                  batch_iterations=sum(its), batch_iter_per_s=round(sum(its) / solve_s, 1),
                                  canonical_GBps=round(canonical_bytes(lps) * sum(its) / solve_s / 1e9, 1),
                                  instance_iterations=inst_its,
                                  instance_iter_per_s=round(inst_its / solve_s, 1),
                                  iterations_round1=its[0], iterations_last=its[-1],
                                  instances_feasible=sum(f is not None for f in first),
                                  mean_first_feasible_round=(round(sum(f for f in first if f) /
                                                                   max(1, sum(f is not None for f in first)), 2)))
        # the passes of the pump batch alone, with the tuned layout (HIP
        # events), in the byte model
        ms_row, ms_col = b.time_passes(20)
        crow, ccol = canonical_pass_bytes(lps)
        rec5 = out["pump_64x20k"]
        rec5.update(ms_row=round(ms_row, 4), ms_col=round(ms_col, 4),
                    row_canonical_GBps=round(crow / ms_row / 1e6, 1), col_canonical_GBps=round(ccol / ms_col / 1e6, 1),
                    row_frac_of_peak=round(crow / ms_row / 1e6 / HBM_PEAK_GBPS, 3),
                    col_frac_of_peak=round(ccol / ms_col / 1e6 / HBM_PEAK_GBPS, 3),
                    iteration_frac_of_peak=round(rec5["canonical_GBps"] / HBM_PEAK_GBPS, 3))
        log(f"w5 pump: {out['pump_64x20k']}")
        # the complete Algorithm 1 loop: eps schedule, early exit per
        # instance, cycle perturbation (finished instances leave the batch)
        t = time.perf_counter()
        recs, outs, xo = b.pump_ex(pump=dict(rounds=args.pump_rounds, seed=0), iter_limit=200_000)
        el = time.perf_counter() - t
        t = time.perf_counter()
        recs1, outs1, xo1 = b.pump_ex(pump=dict(rounds=args.pump_rounds, seed=0, pipeline=1), iter_limit=200_000)
        el1 = time.perf_counter() - t
        same = bool((xo == xo1).all()) and [o["found_round"] for o in outs] == [o["found_round"] for o in outs1]
        found = [o for o in outs if o["found_kind"]]
        out["scylla_loop_64x20k"] = dict(
            seconds=round(el, 3), rounds_max=max(o["rounds_run"] for o in outs), found=len(found),
            found_lp_iterate=sum(o["found_kind"] == 1 for o in outs),
            found_rounding=sum(o["found_kind"] == 2 for o in outs),
            mean_found_round=round(sum(o["found_round"] for o in found) / max(1, len(found)), 2),
            perturbations=sum(o["perturbations"] for o in outs),
            pdhg_iterations_total=sum(o["iterations"] for o in outs),
            seconds_two_groups=round(el1, 3), same_result_two_groups=same)
        # the same loop with restarts to the average and adaptive steps in
        # every round's solve
        for key, kw in (("restart_avg", dict(restart_avg=1)),
                        ("restart_avg_adaptive_steps", dict(restart_avg=1, adaptive=1))):
            t = time.perf_counter()
            recs2, outs2, _ = b.pump_ex(pump=dict(rounds=args.pump_rounds, seed=0), iter_limit=200_000, **kw)
            el2 = time.perf_counter() - t
            found2 = [o for o in outs2 if o["found_kind"]]
            out["scylla_loop_64x20k"][key] = dict(
                seconds=round(el2, 3), found=len(found2),
                mean_found_round=round(sum(o["found_round"] for o in found2) / max(1, len(found2)), 2),
                pdhg_iterations_total=sum(o["iterations"] for o in outs2))
        log(f"w5 complete loop: {out['scylla_loop_64x20k']}")
        b.close()
    if "6" in sel:  # complete loop with the L2 distance on general integers
        lps = instances.int_pump_batch(64, 5_000, 10_000)
        b = pdhg.Batch(lps, precision=pdhg.FP32)
        t = time.perf_counter()
        recs, outs, xo = b.pump_ex(pump=dict(rounds=args.pump_rounds, seed=0, distance=2, perturb=0),
                                   iter_limit=200_000)
        el = time.perf_counter() - t
        found = [o for o in outs if o["found_kind"]]
        out["scylla_loop_l2_general_int_64x5k"] = dict(
            seconds=round(el, 3), rounds_max=max(o["rounds_run"] for o in outs), found=len(found),
            mean_found_round=round(sum(o["found_round"] for o in found) / max(1, len(found)), 2),
            pdhg_iterations_total=sum(o["iterations"] for o in outs))
        log(f"w6 L2 loop, general integers: {out['scylla_loop_l2_general_int_64x5k']}")
        b.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--check-period", type=int, default=64)
    ap.add_argument("--scale", type=float, default=1.0, help="headline workload scale (1 = full size)")
    ap.add_argument("--to-tol", type=int, default=1, help="also time both paths to 1e-4 rel KKT")
    ap.add_argument("--tol-time-limit", type=float, default=60.0)
    ap.add_argument("--cpu-iters", type=int, default=320)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--legs", default="fp32,fp64", help="paths to run (profiling runs may pick one)")
    ap.add_argument("--workloads", default="1,3,4,5,6", help="other workloads to measure ('' for none)")
    ap.add_argument("--pump-rounds", type=int, default=20)
    ap.add_argument("--fp64-plain-batch", type=int, default=1)
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="first run one plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the batched instances of this solver are independent "
              "and a multi-GPU run would only shard them; pass --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2307_03466_amd import instances, pdhg

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    torch.cuda.set_device(0)
    R = args.check_period

    if args.calib_copy_mb > 0:
        src = torch.empty(args.calib_copy_mb << 18, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calib_copy_mb} MiB read + {args.calib_copy_mb} MiB written")
        del src, dst

    t = time.perf_counter()
    lp = instances.workload(2, scale=args.scale)
    log(f"generated {lp.name}: m={lp.m} n={lp.n} nnz={lp.nnz} in {time.perf_counter() - t:.1f}s")

    out = {}
    legs = [(p, tg) for p, tg in ((pdhg.FP32, "fp32"), (pdhg.FP64, "fp64")) if tg in args.legs.split(",")]
    for prec, tag in legs:
        rec = measure(pdhg, [lp], prec, args.steps, args.warmup, R, args.to_tol, args.tol_time_limit)
        info = rec["info"]
        log(f"{tag}: {rec['iter_per_s']:,.0f} iter/s  row pass {rec['ms_row'] * 1e3:.1f} us "
            f"({rec['bytes_row'] / rec['ms_row'] / 1e6:,.0f} GB/s)  col pass {rec['ms_col'] * 1e3:.1f} us "
            f"({rec['bytes_col'] / rec['ms_col'] / 1e6:,.0f} GB/s)  format={info['format_name']} "
            f"layout row B={info['row_blocks']}/{info['row_chunk']} col B={info['col_blocks']}/{info['col_chunk']}")
        if args.to_tol:
            log(f"{tag}: to 1e-4: {rec['to_tol']}")
            log(f"{tag}: to 1e-4 with adaptive steps: {rec['to_tol_adaptive']}")
            log(f"{tag}: {rec['iter_per_s_avg']:,.0f} iter/s with restarts to the average; to 1e-4: "
                f"{rec['to_tol_avg']}; with adaptive steps too: {rec['to_tol_avg_adaptive']}")
        out[tag] = rec

    if "fp32" not in out or "fp64" not in out:
        if args.workloads:
            log(json.dumps(other_workloads(pdhg, instances, args, R)))
        log("partial run (--legs): no JSON line")
        return
    f32 = out["fp32"]
    info = f32["info"]
    def pass_roofline(is_col):
        """HBM roofline of one FP32 pass: canonical bytes of one launch (the
        hot path's byte model: BF16 values 6 B and pattern 4 B per nonzero,
        pointers, split offsets, the pass's vectors, one full gather) over
        the pass's HIP-event time; the packed-word bytes the library's
        format must move beside them; counter traffic; the random-gather
        ceiling."""
        ms = f32["ms_col"] if is_col else f32["ms_row"]
        nbytes = f32["bytes_col"] if is_col else f32["bytes_row"]
        canon = f32["canon_col"] if is_col else f32["canon_row"]
        achieved = canon / (ms * 1e-3) / 1e9
        blocks = info["col_blocks"] if is_col else info["row_blocks"]
        gathered = (info["m_total"] if is_col else info["n_total"]) * 4 // max(1, blocks)
        probe_ms = probe_gather_ms(gathered, info["nnz_total"])
        # every L2 request of the pass at the probe's rate: the gathers plus
        # the coalesced algorithmic bytes (the gathered vector, read once in
        # the byte model, left out) in 64-byte requests
        coalesced = nbytes - (info["m_total"] if is_col else info["n_total"]) * 4
        requests = info["nnz_total"] + coalesced / 64
        request_ms = probe_ms * requests / info["nnz_total"]
        kernels = pass_kernels(info, is_col)
        return dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBPS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBPS, 4),
                    traffic=measured_traffic(kernels) if kernels else None,
                    kernel=("column" if is_col else "row") + " pass (" +
                    ("k_bpart + k_bcombine, %d gather blocks" % blocks if blocks > 0 else
                     "k_pass" if blocks == 0 else "k_spass, LDS-staged") + ")",
                    bytes_per_launch=canon, bytes_per_launch_packed=nbytes,
                    frac_packed=round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4), launch_ms=round(ms, 5),
                    gather_ceiling={"gathers": info["nnz_total"], "vector_bytes_per_xcd": gathered,
                                    "probe_ms": round(probe_ms, 5), "frac": round(probe_ms / ms, 3),
                                    "requests": int(requests), "request_ms": round(request_ms, 5),
                                    "frac_requests": round(request_ms / ms, 3)})

    # the dominant kernel is the slower pass; the two take about as long, so
    # both are reported
    dom_is_col = f32["ms_col"] >= f32["ms_row"]
    both = {"col": pass_roofline(True), "row": pass_roofline(False)}
    roofline = both["col" if dom_is_col else "row"]
    path_bytes = f32["bytes_row"] + f32["bytes_col"]
    line = {
        "metric": METRIC,
        "value": round(f32["iter_per_s"], 1),
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(f32["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"general LP {lp.m} x {lp.n}, {lp.nnz} nonzeros (geometric row lengths, "
                               f"integers in [-20,20]), one instance",
                   "m": lp.m, "n": lp.n, "nnz": lp.nnz, "check_period": R,
                   "matrix_format": info["format_name"],
                   "layout": {"row_blocks": info["row_blocks"], "row_chunk": info["row_chunk"],
                              "col_blocks": info["col_blocks"], "col_chunk": info["col_chunk"]},
                   "step": f"KKT check + decision + {R} PDHG iterations (one hipGraph)"},
        "roofline": roofline,
        "roofline_passes": both,
        "path_GBps": round(path_bytes * f32["iter_per_s"] / 1e9, 1),
        "canonical_GBps": round(f32["canon_iter"] * f32["iter_per_s"] / 1e9, 1),
        "fp64_plain": {"iter_per_s": round(out["fp64"]["iter_per_s"], 1),
                       "ms_row": round(out["fp64"]["ms_row"], 5), "ms_col": round(out["fp64"]["ms_col"], 5),
                       "canonical_GBps": round(out["fp64"]["canon_iter"] * out["fp64"]["iter_per_s"] / 1e9, 1)},
        "speedup_fp32_vs_fp64_iter": round(f32["iter_per_s"] / out["fp64"]["iter_per_s"], 3),
        "iter_per_s_restart_avg": ({"fp32": round(f32["iter_per_s_avg"], 1),
                                    "fp64": round(out["fp64"]["iter_per_s_avg"], 1)}
                                   if "iter_per_s_avg" in f32 else None),
        "setup_seconds": {"fp32": round(f32["setup_s"], 3), "fp64": round(out["fp64"]["setup_s"], 3)},
    }
    if args.to_tol:
        line["to_tol_1e-4"] = {"fp32": out["fp32"]["to_tol"], "fp64": out["fp64"]["to_tol"],
                               "fp32_adaptive_steps": out["fp32"]["to_tol_adaptive"],
                               "fp64_adaptive_steps": out["fp64"]["to_tol_adaptive"],
                               "fp32_restart_avg": out["fp32"]["to_tol_avg"],
                               "fp64_restart_avg": out["fp64"]["to_tol_avg"],
                               "fp32_restart_avg_adaptive_steps": out["fp32"]["to_tol_avg_adaptive"],
                               "fp64_restart_avg_adaptive_steps": out["fp64"]["to_tol_avg_adaptive"]}
        if out["fp32"]["to_tol"]["status"] == 1 and out["fp64"]["to_tol"]["status"] == 1:
            line["speedup_fp32_vs_fp64_to_tol"] = round(out["fp64"]["to_tol"]["seconds"]
                                                        / out["fp32"]["to_tol"]["seconds"], 3)
    if args.workloads:
        line["workloads"] = other_workloads(pdhg, instances, args, R)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle baseline ...")
        line["cpu_baseline"] = cpu_baseline(lp, args.cpu_iters)
        if args.workloads:
            line["cpu_baseline"]["other_workloads"] = cpu_baselines_other(instances, set(args.workloads.split(",")))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
