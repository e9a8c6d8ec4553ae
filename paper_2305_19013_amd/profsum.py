"""Summarise rocprofv3 output of a benchmark run into the tables kept under profiles/.

Reads the CSV files rocprofv3 writes (kernel traces, and per-dispatch counter values of
FETCH_SIZE / WRITE_SIZE runs), groups kernels into the solver's classes, and prints a
markdown summary: kernel time per kernel and per class, and calibrated HBM bytes per
dispatch per class.  Calibration: the benchmark's --copy-calibration copies 1 GiB before the
solve; the counter value of that copy dispatch against the 1 GiB it moved gives the factor by
which each counter is scaled.

Usage:
    python -m paper_2305_19013_amd.profsum --trace DIR [--fetch DIR] [--write DIR]
           [--bench JSON] [--title TEXT] [--source FILE]
DIR is a rocprofv3 -d directory (searched recursively); JSON is the benchmark's output line
(for the algorithmic bytes per launch and the HIP-event times of the same workload).
"""

from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 1 << 30  # the benchmark's calibration copy

CLASSES = [
    ("cgs2_update", re.compile(r"k_update(_mfma)?<")),
    ("cgs2_gram_reduce", re.compile(r"k_reduce_chunks")),
    ("cgs2_gram", re.compile(r"k_gram(_mfma)?<")),
    ("spmm", re.compile(r"k_spmm")),
    ("final_update", re.compile(r"k_small_mfma<[^>]*true>|k_final_update")),
    ("times_small", re.compile(r"k_small_mfma<[^>]*false>|k_times_small")),
    ("small_gram", re.compile(r"k_small_gram")),
]


def kernel_class(name: str) -> str:
    for cls, rx in CLASSES:
        if rx.search(name):
            return cls
    return "other"


def short(name: str) -> str:
    name = name.replace("ecg::(anonymous namespace)::", "")
    name = re.sub(r"\(.*\)$", "", name).strip()
    return name[:70]


def _rows(d: str, suffix: str):
    for path in sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)):
        with open(path, newline="") as f:
            yield from csv.DictReader(f)


def trace(d: str):
    """[(kernel name, duration ns)] in dispatch order."""
    out = []
    for r in _rows(d, "kernel_trace.csv"):
        out.append((r["Kernel_Name"], int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    return out


def counters(d: str, counter: str):
    """[(kernel name, counter value)] per dispatch."""
    acc = defaultdict(float)
    names = {}
    for r in _rows(d, "counter_collection.csv"):
        if r.get("Counter_Name") != counter:
            continue
        key = int(r.get("Dispatch_Id") or r.get("Correlation_Id"))
        acc[key] += float(r["Counter_Value"])
        names[key] = r["Kernel_Name"]
    return [(names[k], acc[k]) for k in sorted(acc)]


def calibrate(rows, moved_kib: float):
    """Factor that maps the counter (KiB) of the 1 GiB copy dispatch onto the bytes moved."""
    copies = [v for n, v in rows if "copyBuffer" in n or "copy" in n.lower()]
    if not copies:
        return None, None
    big = max(copies)
    return moved_kib / big, big


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--bench")
    ap.add_argument("--title", default="")
    ap.add_argument("--source", default=os.path.join(HERE, "csrc", "ecg_kernels.hip"))
    args = ap.parse_args()
    out = []
    if args.title:
        out.append(f"# {args.title}\n")
    tr = trace(args.trace)
    per_kernel = defaultdict(lambda: [0, 0])
    per_class = defaultdict(lambda: [0, 0])
    for name, ns in tr:
        if "copyBuffer" in name:
            continue
        per_kernel[name][0] += 1
        per_kernel[name][1] += ns
        c = kernel_class(name)
        per_class[c][0] += 1
        per_class[c][1] += ns
    total = sum(v[1] for v in per_kernel.values())
    out.append("## Kernel time (rocprofv3 --kernel-trace --stats)\n")
    out.append("| kernel | calls | average µs | total s | % of GPU time |")
    out.append("|---|---|---|---|---|")
    for name, (cnt, ns) in sorted(per_kernel.items(), key=lambda kv: -kv[1][1])[:16]:
        out.append(f"| `{short(name)}` | {cnt} | {ns / cnt / 1e3:.1f} | {ns / 1e9:.3f} | {100 * ns / total:.2f} |")
    out.append(f"\nTotal GPU kernel time {total / 1e9:.2f} s.\n")
    bench = None
    if args.bench:
        with open(args.bench) as f:
            bench = json.loads([ln for ln in f.read().splitlines() if ln.strip().startswith("{")][-1])
    for cls in ("cgs2_update", "cgs2_gram", "spmm", "final_update", "times_small"):
        if cls not in per_class:
            continue
        cnt, ns = per_class[cls]
        line = f"- {cls}: rocprofv3 {ns / 1e6:.0f} ms over {cnt} launches (mean {ns / cnt / 1e3:.1f} µs)"
        k = (bench or {}).get("kernels", {}).get(cls)
        if k:
            line += f"; bench HIP events {k['ms']} ms over {k['launches']} launches (mean {k['ms'] / k['launches'] * 1e3:.1f} µs)"
        out.append(line)
    lines = []
    if args.fetch and args.write:
        fr, wr = counters(args.fetch, "FETCH_SIZE"), counters(args.write, "WRITE_SIZE")
        ff, fcopy = calibrate(fr, COPY_BYTES / 1024)
        wf, wcopy = calibrate(wr, COPY_BYTES / 1024)
        out.append("\n## HBM traffic (rocprofv3 --pmc, one counter per run)\n")
        if ff is None or wf is None:
            out.append("No calibration copy found in the counter runs.")
        else:
            out.append(f"Calibration: the 1 GiB copy reads FETCH_SIZE = {fcopy:.0f} KiB and WRITE_SIZE = {wcopy:.0f} "
                       f"KiB, so fetch counts are scaled by {ff:.5f} and write counts by {wf:.5f} (counters in KiB).\n")
            agg = defaultdict(lambda: [0, 0.0, 0.0])
            for name, v in fr:
                if "copy" in name.lower():
                    continue
                a = agg[kernel_class(name)]
                a[0] += 1
                a[1] += v * ff * 1024
            for name, v in wr:
                if "copy" in name.lower():
                    continue
                agg[kernel_class(name)][2] += v * wf * 1024
            out.append("| kernel class | dispatches | calibrated HBM bytes per dispatch | read | written |")
            out.append("|---|---|---|---|---|")
            for cls in ("cgs2_update", "cgs2_gram", "spmm", "final_update", "times_small"):
                if cls not in agg:
                    continue
                n_, rd, wt = agg[cls]
                out.append(f"| {cls} | {n_} | {(rd + wt) / n_ / 1e9:.3f} GB | {rd / n_ / 1e9:.3f} GB | "
                           f"{wt / n_ / 1e9:.3f} GB |")
                lines.append(f"traffic_bytes_per_launch {cls} {(rd + wt) / n_:.6e}")
            roof = (bench or {}).get("roofline") or {}
            if roof.get("algorithmic_bytes_per_launch") and roof.get("kernel") in agg:
                n_, rd, wt = agg[roof["kernel"]]
                ratio = (rd + wt) / n_ / roof["algorithmic_bytes_per_launch"]
                out.append(f"\nMeasured traffic / algorithmic bytes for {roof['kernel']}: {ratio:.3f} "
                           f"({roof['algorithmic_bytes_per_launch'] / 1e9:.3f} GB algorithmic per launch).")
    src = os.path.basename(args.source)
    sha = hashlib.sha256(open(args.source, "rb").read()).hexdigest()[:16]
    out.append("\nMachine-readable lines read by bench.py (traffic is reported only while the kernel source "
               "hash matches):\n")
    out.append("```")
    out.append(f"kernel_source {src}")
    out.append(f"kernels_sha256_16 {sha}")
    out.extend(lines)
    out.append("```")
    print("\n".join(out))


if __name__ == "__main__":
    sys.exit(main())
