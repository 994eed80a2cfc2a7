"""Summaries of rocprofv3 CSV output for one kernel class over the timed window.

The benchmark's event-timed replay is the last part of its run, so the window
of a class is the last D dispatches of its kernel in the trace, D being the
dispatch count the benchmark line reports (``kernel_dispatches``).  Counter
runs (``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE``) are scaled by the same
counter read on a device copy of known size.

    python prof_window.py trace DIR CLASS BENCH_JSON
    python prof_window.py pmc DIR CLASS D [COPY_BYTES]
"""
from __future__ import annotations

import collections
import csv
import glob
import hashlib
import json
import os
import re
import sys


def _one(pattern: str) -> str:
    files = sorted(glob.glob(pattern, recursive=True))
    if not files:
        raise SystemExit(f"no file matches {pattern}")
    return files[0]


def _short(name: str) -> str:
    m = re.search(r"(\w+)_kernel", name)
    return m.group(1) if m else name.split("(")[0][-40:]


def trace(dirname: str, cls: str, bench_json: str) -> None:
    bench = json.loads(open(bench_json).read().strip().splitlines()[-1])
    D = int(bench["kernel_dispatches"][cls])
    stats = _one(os.path.join(dirname, "**", "*kernel_stats.csv"))
    print(f"kernel stats ({os.path.basename(stats)}), top 12 by total time:")
    print("| kernel | calls | total ms | avg us | % |")
    print("|---|---:|---:|---:|---:|")
    for r in list(csv.DictReader(open(stats)))[:12]:
        print(f"| {_short(r['Name'])} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
              f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    rows = sorted(csv.DictReader(open(_one(os.path.join(dirname, "**", "*kernel_trace.csv")))),
                  key=lambda r: int(r["Start_Timestamp"]))
    idx = [i for i, r in enumerate(rows) if _short(r["Kernel_Name"]) == cls]
    win = idx[-D:]
    dur = [int(rows[i]["End_Timestamp"]) - int(rows[i]["Start_Timestamp"]) for i in win]
    print(f"\nwindow: last {len(win)} dispatches of {cls}: average {sum(dur) / max(1, len(dur)) / 1e3:.3f} us, "
          f"total {sum(dur) / 1e6:.2f} ms")
    runs, cur = [], []
    for i in win:
        if cur and i != cur[-1] + 1:
            runs.append(cur)
            cur = []
        cur.append(i)
    if cur:
        runs.append(cur)
    bursts = [r for r in runs if len(r) > 1]
    if bursts:
        bd = [int(rows[i]["End_Timestamp"]) - int(rows[i]["Start_Timestamp"]) for r in bursts for i in r]
        gaps = sorted(int(rows[i + 1]["Start_Timestamp"]) - int(rows[i]["End_Timestamp"]) for r in bursts
                      for i in r[:-1])
        print(f"bursts (back-to-back runs of the class): {len(bursts)} of length "
              f"{collections.Counter(len(r) for r in bursts).most_common(1)[0][0]}; average dispatch "
              f"{sum(bd) / len(bd) / 1e3:.3f} us; gap between dispatches under the tracer: mean "
              f"{sum(gaps) / len(gaps) / 1e3:.2f} us, median {gaps[len(gaps) // 2] / 1e3:.2f} us")
    r = bench["roofline"]
    print(f"benchmark line of this traced run: avg_launch_ms {r['avg_launch_ms']:.6f}, "
          f"launches_timed {r.get('launches_timed')}, dispatches {r.get('dispatches')}")


def pmc(dirname: str, cls: str, D: int, copy_bytes: int = 0) -> None:
    f = _one(os.path.join(dirname, "**", "*counter_collection.csv"))
    by = collections.defaultdict(list)
    for r in csv.DictReader(open(f)):
        by[(_short(r["Kernel_Name"]), r["Counter_Name"])].append(float(r["Counter_Value"]))
    for (k, c), v in sorted(by.items()):
        if k == cls:
            w = v[-D:]
            print(f"{c} {k}: {len(v)} dispatches, window {len(w)}, mean {sum(w) / len(w):.1f} KiB per dispatch")
        elif "copyBuffer" in k and copy_bytes:
            print(f"{c} copy of {copy_bytes} bytes: {sum(v):.1f} KiB (scale {copy_bytes / 1024 / sum(v):.4f})")


def sources_sha256(paths: list[str], root: str) -> str:
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(root, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


if __name__ == "__main__":
    a = sys.argv[1:]
    if a and a[0] == "trace" and len(a) == 4:
        trace(a[1], a[2], a[3])
    elif a and a[0] == "pmc" and len(a) in (4, 5):
        pmc(a[1], a[2], int(a[3]), int(a[4]) if len(a) == 5 else 0)
    elif a and a[0] == "sha256":
        print(sources_sha256(a[1].split(","), os.path.dirname(os.path.abspath(__file__))))
    else:
        raise SystemExit(__doc__)
