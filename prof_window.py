"""Summaries of rocprofv3 CSV output for one kernel class over the timed window.

The benchmark's event-timed replay is the last part of its run, so the window
of a class is the last D dispatches of its kernel in the trace, D being the
dispatch count the benchmark line reports (``kernel_dispatches``).  Counter
runs (``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE``) are scaled by the same
counter read on a device copy of known size.

    python prof_window.py trace DIR CLASS BENCH_JSON
    python prof_window.py pmc DIR CLASS D [COPY_BYTES]
    python prof_window.py counters DIR NAME_PART [D]
    python prof_window.py sha256 FILE,FILE,...
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


def _workgroups(r: dict) -> int:
    """Workgroups of one traced dispatch (grid sizes are in threads)."""
    n = 1
    for ax in "XYZ":
        g = int(r.get(f"Grid_Size_{ax}", r.get("Grid_Size", 1)) if ax == "X" else r.get(f"Grid_Size_{ax}", 1))
        w = int(r.get(f"Workgroup_Size_{ax}", r.get("Workgroup_Size", 1)) if ax == "X" else
                r.get(f"Workgroup_Size_{ax}", 1))
        n *= max(1, -(-g // max(1, w)))
    return n


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
    shapes = collections.defaultdict(list)
    for i in win:
        shapes[_workgroups(rows[i])].append(int(rows[i]["End_Timestamp"]) - int(rows[i]["Start_Timestamp"]))
    print(f"\nworkgroups launched per dispatch in the window (grid x * y * z / workgroup size):")
    print("| workgroups | dispatches | avg us |")
    print("|---:|---:|---:|")
    for wg in sorted(shapes):
        v = shapes[wg]
        print(f"| {wg} | {len(v)} | {sum(v) / len(v) / 1e3:.3f} |")
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


def counters(dirname: str, pattern: str, D: int = 0) -> None:
    """Per-dispatch means of every collected counter for the kernels whose
    name contains `pattern`, grouped by instantiation, over the last D
    dispatches of each (all when D = 0).  The MFMA op counters
    (SQ_INSTS_VALU_MFMA_MOPS_*) count units of 512 flops; MfmaUtil is the busy
    share of the matrix cores, SQ_VALU_MFMA_BUSY_CYCLES summed over the SIMDs
    over the busy cycles of the device times the SIMD count (the CSV holds
    GRBM_GUI_ACTIVE summed over the XCDs: the device's cycles are that sum
    over the XCD count)."""
    f = _one(os.path.join(dirname, "**", "*counter_collection.csv"))
    simds, xcc = 0, 1
    agent = glob.glob(os.path.join(dirname, "**", "*agent_info.csv"), recursive=True)
    for r in (csv.DictReader(open(agent[0])) if agent else []):
        if r.get("Agent_Type") == "GPU":
            simds, xcc = int(r["Simd_Count"]), max(1, int(r["Num_Xcc"]))
    by = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in csv.DictReader(open(f)):
        name = r["Kernel_Name"]
        if pattern not in name:
            continue
        bare = name.replace("(anonymous namespace)::", "")
        key = bare.split("(")[0] if "<" not in bare else bare[:bare.rfind(">") + 1]
        by[key][r["Counter_Name"]].append(float(r["Counter_Value"]))
    for key, cs in sorted(by.items()):
        print(f"{key}")
        means = {}
        for c, v in sorted(cs.items()):
            w = v[-D:] if D > 0 else v
            means[c] = sum(w) / len(w)
            line = f"  {c}: {len(v)} dispatches, window {len(w)}, mean {means[c]:.4g} per dispatch"
            if "MFMA_MOPS" in c:
                line += f" ({means[c] * 512 / 1e9:.4g} GFLOP)"
            print(line)
        if simds and "SQ_VALU_MFMA_BUSY_CYCLES" in means and means.get("GRBM_GUI_ACTIVE"):
            cyc = means["GRBM_GUI_ACTIVE"] / xcc
            print(f"  device busy cycles {cyc:.4g} per dispatch; MfmaUtil over the window: "
                  f"{100 * means['SQ_VALU_MFMA_BUSY_CYCLES'] / (cyc * simds):.1f} % ({simds} SIMDs, {xcc} XCDs)")


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
    elif a and a[0] == "counters" and len(a) in (3, 4):
        counters(a[1], a[2], int(a[3]) if len(a) == 4 else 0)
    elif a and a[0] == "sha256":
        print(sources_sha256(a[1].split(","), os.path.dirname(os.path.abspath(__file__))))
    else:
        raise SystemExit(__doc__)
