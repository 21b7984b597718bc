"""Markdown summaries of rocprofv3 CSV output (kernel trace / statistics and
counter collection), used for the files under profiles/.

  python -m paper_2307_03466_amd.profsum trace  <run_kernel_trace.csv> [top]
  python -m paper_2307_03466_amd.profsum counter <run_counter_collection.csv> <scale> [name-filter]
  python -m paper_2307_03466_amd.profsum traffic <fetch.csv> <write.csv> <fetch-scale> <out.json>
  python -m paper_2307_03466_amd.profsum gather [gathers]   (needs the GPU)

`trace` lists per kernel the launches, total time, rocprofv3's mean, and the
mean over launches longer than 10 us (the solver launches whole check
windows; iterations after an instance finished exit at once and are
short).  `counter` lists per kernel the median counter value per dispatch
longer than 10 us in KiB and that value times `scale` in MB (FETCH_SIZE reads half of a plain
copy's bytes on this device: scale 2.0; WRITE_SIZE: scale 1.0).  `gather`
runs the library's random-gather probe (scylla_probe_gather) for vectors of
1 to 8 MB and prints the rates."""
from __future__ import annotations

import csv
import statistics
import sys
from collections import defaultdict


def _short(name: str, width: int = 88) -> str:
    name = name.replace("scy::", "").replace("(scy::PassArgs<float>, int)", "").replace(
        "(scy::PassArgs<double>, int)", "")
    return name if len(name) <= width else name[: width - 3] + "..."


def trace(path: str, top: int = 14) -> str:
    durs = defaultdict(list)
    for r in csv.DictReader(open(path)):
        durs[r["Kernel_Name"]].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    rows = sorted(durs.items(), key=lambda kv: -sum(kv[1]))[:top]
    out = ["| kernel | launches | total ms | mean us | launches > 10 us | mean of those us |",
           "|---|---|---|---|---|---|"]
    for k, v in rows:
        act = [x for x in v if x > 10_000]
        out.append(f"| `{_short(k)}` | {len(v)} | {sum(v) / 1e6:.2f} | {statistics.mean(v) / 1e3:.1f} | "
                   f"{len(act)} | {statistics.mean(act) / 1e3 if act else 0:.1f} |")
    return "\n".join(out)


def _active(r) -> bool:
    """Dispatches longer than 10 us (launches of windows in which the
    instance already finished exit at once)."""
    try:
        return int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) > 10_000
    except (KeyError, ValueError):
        return True


def counter(path: str, scale: float, filt: str = "") -> str:
    vals = defaultdict(list)
    name = None
    for r in csv.DictReader(open(path)):
        name = r["Counter_Name"]
        if filt in r["Kernel_Name"] and _active(r):
            vals[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    out = [f"| kernel | dispatches | median {name} KiB | x{scale:g} = MB per dispatch |", "|---|---|---|---|"]
    for k, v in sorted(vals.items(), key=lambda kv: -statistics.median(kv[1])):
        med = statistics.median(v)
        out.append(f"| `{_short(k)}` | {len(v)} | {med:,.0f} | {med * scale * 1024 / 1e6:,.1f} |")
    return "\n".join(out)


def kernels_sha256() -> str:
    import hashlib
    import os
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "kernels.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()


def traffic(fetch_csv: str, write_csv: str, fetch_scale: float, out: str) -> None:
    """Median FETCH_SIZE x fetch_scale and WRITE_SIZE bytes per dispatch of
    every kernel, stamped with the hash of the kernel source they measure."""
    import json
    rec = {}
    for path, key, scale in ((fetch_csv, "fetch_bytes", fetch_scale), (write_csv, "write_bytes", 1.0)):
        vals = defaultdict(list)
        for r in csv.DictReader(open(path)):
            if _active(r):
                vals[_short(r["Kernel_Name"], 200)].append(float(r["Counter_Value"]))
        for k, v in vals.items():
            rec.setdefault(k, {})[key] = round(statistics.median(v) * 1024 * scale)
    json.dump({"kernels_hip_sha256": kernels_sha256(), "fetch_scale": fetch_scale, "kernels": rec},
              open(out, "w"), indent=1, sort_keys=True)


def gather(gathers: int = 10_000_000) -> str:
    """Markdown table of the device's random 4-byte gather rate by vector size."""
    from . import pdhg
    out = ["| vector | ms per launch | G gathers/s |", "|---|---|---|"]
    for mb in (1, 2, 4, 8):
        ms = pdhg.probe_gather(mb * 1_000_000, gathers)
        out.append(f"| {mb} MB | {ms:.4f} | {gathers / (ms * 1e-3) / 1e9:.1f} |")
    return "\n".join(out)


if __name__ == "__main__":
    if sys.argv[1] == "gather":
        print(gather(int(sys.argv[2]) if len(sys.argv) > 2 else 10_000_000))
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], float(sys.argv[4]), sys.argv[5])
    elif sys.argv[1] == "trace":
        print(trace(sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 14))
    else:
        print(counter(sys.argv[2], float(sys.argv[3]), sys.argv[4] if len(sys.argv) > 4 else ""))
