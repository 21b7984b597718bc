#!/usr/bin/env python
"""Benchmark of the PDHG hot path on one MI355X.

Workload: the single large general LP (m = 1,000,000 rows, n = 2,000,000
columns, ~10M nonzeros, geometric row lengths, integer coefficients in
[-20, 20]), synthetic and seeded.  A step is one check window of the
solver: the FP64 KKT check and decision plus R = 64 PDHG iterations (column
pass + row pass), all replayed from one hipGraph.  value = PDHG iterations/s
of the FP32 path with the problem resident in HBM.

Also reported: the plain FP64 path's iteration rate on the same LP, the time
of both paths to reach relative KKT <= 1e-4, the dominant kernel's roofline
(algorithmic bytes per launch over its HIP-event launch time, against the
8 TB/s HBM peak) and, as a baseline, the FP64 CPU oracle on a bounded sample.
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


def canonical_bytes(m, n, nnz, fp64=False):
    """Per-iteration byte model of the survey's FP32 / FP64 path (BF16 / FP64
    values, int32 indices): both passes' matrix streams and pointers, the
    per-column and per-row vector traffic and one full gather of each vector."""
    if fp64:
        return 2 * nnz * 12 + 4 * (m + 1) + 4 * (n + 1) + 56 * n + 33 * m + 8 * (m + n)
    return 2 * nnz * 6 + 4 * (m + 1) + 4 * (n + 1) + 28 * n + 17 * m + 4 * (m + n)


def timed_steps(batch, steps, R):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = batch.solve(tol=1e-300, iter_limit=steps * R, check_period=R)[0]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert res["iterations"] == steps * R, res
    return dt, res


def cpu_baseline(lp, iters):
    import oracle
    t0 = time.perf_counter()
    oracle.pdhg(lp, tol=-1.0, iter_limit=0)
    t1 = time.perf_counter()
    oracle.pdhg(lp, tol=-1.0, iter_limit=iters)
    t2 = time.perf_counter()
    per_iter = ((t2 - t1) - (t1 - t0)) / iters
    return dict(value=1.0 / per_iter, unit="iter/s", cores=1, kind="oracle",
                sample=f"{iters} FP64 PDHG iterations of the same 1M x 2M LP by the single-threaded C "
                       f"oracle (preconditioning and the start check subtracted; {t2 - t0:.1f} s of CPU)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--check-period", type=int, default=64)
    ap.add_argument("--scale", type=float, default=1.0, help="workload scale (1 = full size)")
    ap.add_argument("--to-tol", type=int, default=1, help="also time both paths to 1e-4 rel KKT")
    ap.add_argument("--tol-time-limit", type=float, default=60.0)
    ap.add_argument("--cpu-iters", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--legs", default="fp32,fp64", help="paths to run (profiling runs may pick one)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="first run one plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the batched instances of this solver are independent "
              "and a multi-GPU run would only shard them; pass --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
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
    legs = [(p, t) for p, t in ((pdhg.FP32, "fp32"), (pdhg.FP64, "fp64")) if t in args.legs.split(",")]
    for prec, tag in legs:
        b = pdhg.Batch([lp], precision=prec)
        info = b.info()
        setup = b.solve(tol=1e-300, iter_limit=0)[0]["setup_seconds"]
        b.solve(tol=1e-300, iter_limit=max(1, args.warmup) * R, check_period=R)  # autotune + warm-up
        dt, res = timed_steps(b, args.steps, R)
        its = args.steps * R
        ms_row, ms_col = b.time_passes(20)
        vb = 4 if prec == pdhg.FP32 else 8
        rb, cb = pass_bytes(info, vb)
        rec = dict(info=info, setup_s=setup, seconds=dt, iters=its, iter_per_s=its / dt,
                   ms_per_step=1000 * dt / args.steps, ms_row=ms_row, ms_col=ms_col,
                   bytes_row=rb, bytes_col=cb, rel_kkt_end=res["rel_kkt"])
        log(f"{tag}: {its / dt:,.0f} iter/s  row pass {ms_row * 1e3:.1f} us ({rb / ms_row / 1e6:,.0f} GB/s)  "
            f"col pass {ms_col * 1e3:.1f} us ({cb / ms_col / 1e6:,.0f} GB/s)  format={info['format_name']} "
            f"chunks={info['row_chunk']}/{info['col_chunk']}")
        if args.to_tol:
            r = b.solve(tol=1e-4, iter_limit=2_000_000, time_limit_s=args.tol_time_limit)[0]
            rec["to_tol"] = dict(status=r["status"], iterations=r["iterations"], seconds=r["solve_seconds"],
                                 rel_kkt=r["rel_kkt"], restarts=r["restarts"], primal_obj=r["primal_obj"])
            log(f"{tag}: to 1e-4: status={r['status']} iters={r['iterations']} "
                f"{r['solve_seconds']:.2f}s rel={r['rel_kkt']:.3e} obj={r['primal_obj']:.6f}")
        b.close()
        out[tag] = rec

    if "fp32" not in out or "fp64" not in out:
        log("partial run (--legs): no JSON line")
        return
    f32 = out["fp32"]
    dom_is_col = f32["ms_col"] >= f32["ms_row"]
    dom_ms = f32["ms_col"] if dom_is_col else f32["ms_row"]
    dom_bytes = f32["bytes_col"] if dom_is_col else f32["bytes_row"]
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBPS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBPS, 4), traffic=None,
                    kernel="k_pass<float,packed,%s>" % ("column" if dom_is_col else "row"),
                    bytes_per_launch=dom_bytes, launch_ms=round(dom_ms, 5))
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
                   "matrix_format": f32["info"]["format_name"],
                   "step": f"KKT check + decision + {R} PDHG iterations (one hipGraph)"},
        "roofline": roofline,
        "path_GBps": round(path_bytes * f32["iter_per_s"] / 1e9, 1),
        "canonical_GBps": round(canonical_bytes(lp.m, lp.n, lp.nnz) * f32["iter_per_s"] / 1e9, 1),
        "fp64_plain": {"iter_per_s": round(out["fp64"]["iter_per_s"], 1),
                       "ms_row": round(out["fp64"]["ms_row"], 5), "ms_col": round(out["fp64"]["ms_col"], 5),
                       "canonical_GBps": round(canonical_bytes(lp.m, lp.n, lp.nnz, True)
                                               * out["fp64"]["iter_per_s"] / 1e9, 1)},
        "speedup_fp32_vs_fp64_iter": round(f32["iter_per_s"] / out["fp64"]["iter_per_s"], 3),
        "setup_seconds": {"fp32": round(f32["setup_s"], 3), "fp64": round(out["fp64"]["setup_s"], 3)},
    }
    if args.to_tol:
        line["to_tol_1e-4"] = {"fp32": out["fp32"]["to_tol"], "fp64": out["fp64"]["to_tol"]}
        if out["fp32"]["to_tol"]["status"] == 1 and out["fp64"]["to_tol"]["status"] == 1:
            line["speedup_fp32_vs_fp64_to_tol"] = round(out["fp64"]["to_tol"]["seconds"]
                                                        / out["fp32"]["to_tol"]["seconds"], 3)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle baseline ...")
        line["cpu_baseline"] = cpu_baseline(lp, args.cpu_iters)
        line["cpu_baseline"]["value"] = round(line["cpu_baseline"]["value"], 3)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
