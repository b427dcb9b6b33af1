"""Summarize rocprofv3 CSV output into the short text / JSON files kept under
profiles/ (kernel-trace statistics and HBM byte counters).

Usage:
  python -m paper_2602_23525_amd.rocprof_summary trace <kernel_stats.csv> <out.txt> <command>
  python -m paper_2602_23525_amd.rocprof_summary pmc <workload> <fetch.csv> <write.csv> \
        <copy_fetch.csv> <copy_write.csv> <copy_bytes> <kernel_substring> <bench.json> \
        <out.json> <commands>

FETCH_SIZE and WRITE_SIZE are KiB per dispatch.  Each is scaled by the ratio of
a plain copy kernel's known byte count to what the same counter reports for it.
The summary records a hash of the kernel sources and the plan the benchmark ran
(from its JSON line); the benchmark uses the byte count only while both match.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# sources of the specialized leaf kernel (the dominant kernel of the batched
# power-of-two workloads)
KERNEL_SOURCES = ["paper_2602_23525_amd/csrc/leaf.h", "paper_2602_23525_amd/csrc/k_leaf.hip",
                  "paper_2602_23525_amd/csrc/butterfly.h", "paper_2602_23525_amd/csrc/internal.h",
                  "paper_2602_23525_amd/csrc/twiddle4.h"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_mean(path: str, counter: str, kernel_sub: str) -> float:
    vals = defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter and kernel_sub in r["Kernel_Name"]:
            vals[r["Dispatch_Id"]].append(float(r["Counter_Value"]))
    per = [sum(v) for v in vals.values()]
    if not per:
        raise ValueError(f"no {counter} rows for {kernel_sub} in {path}")
    return sum(per) / len(per)


def bench_plan(bench_json: str) -> str:
    """The plan description from the last JSON line of a bench.py run."""
    lines = [ln for ln in open(bench_json).read().splitlines() if ln.startswith("{")]
    return json.loads(lines[-1])["config"]["plan"]


def trace(stats_csv: str, out_txt: str, command: str):
    rows = list(csv.DictReader(open(stats_csv)))
    with open(out_txt, "w") as f:
        f.write(f"# rocprofv3 kernel-trace statistics\n# command: {command}\n")
        f.write("# kernel | calls | average ns | min ns | max ns | share %\n")
        for r in rows:
            f.write(f"{r['Name']} | {r['Calls']} | {float(r['AverageNs']):.1f} | {r['MinNs']} | "
                    f"{r['MaxNs']} | {float(r['Percentage']):.2f}\n")


def pmc(workload, fetch_csv, write_csv, cfetch_csv, cwrite_csv, copy_bytes, kernel_sub,
        bench_json, out_json, commands):
    copy_bytes = float(copy_bytes)
    cf = counter_mean(cfetch_csv, "FETCH_SIZE", "copy") * 1024.0
    cw = counter_mean(cwrite_csv, "WRITE_SIZE", "copy") * 1024.0
    kf = counter_mean(fetch_csv, "FETCH_SIZE", kernel_sub) * 1024.0
    kw = counter_mean(write_csv, "WRITE_SIZE", kernel_sub) * 1024.0
    sf, sw = copy_bytes / cf, copy_bytes / cw
    d = {"workload": workload, "kernel": kernel_sub,
         "fetch_kib_raw": kf / 1024.0, "write_kib_raw": kw / 1024.0,
         "copy_bytes": copy_bytes, "copy_fetch_kib_raw": cf / 1024.0,
         "copy_write_kib_raw": cw / 1024.0, "fetch_scale": sf, "write_scale": sw,
         "traffic_bytes_per_launch": kf * sf + kw * sw,
         "source_hash": kernel_source_hash(), "plan": bench_plan(bench_json),
         "commands": commands}
    with open(out_json, "w") as f:
        json.dump(d, f, indent=1)
    print(json.dumps(d))


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace(*sys.argv[2:5])
    elif sys.argv[1] == "pmc":
        pmc(*sys.argv[2:12])
    else:
        raise SystemExit(__doc__)
