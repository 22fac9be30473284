"""Summaries of rocprofv3 output for the committed profile notes.

    python -m paper_2407_05930_amd.profiling stats <kernel_stats.csv> <out.md> <command>
    python -m paper_2407_05930_amd.profiling traffic <fetch_counter_collection.csv>
        <write_counter_collection.csv> <kernel substring> <copy bytes> <out.md> <command...>

The traffic summary scales each counter of the named kernel by the ratio
between the known size of a plain device copy and what the same counter
reads for that copy (rocprofv3 reports FETCH_SIZE / WRITE_SIZE in KiB).
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def source_hash() -> str:
    h = hashlib.sha256()
    for name in sorted(os.listdir(os.path.join(HERE, "csrc"))):
        with open(os.path.join(HERE, "csrc", name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def stats(path, out, command):
    rows = list(csv.DictReader(open(path)))
    lines = [f"# rocprofv3 kernel statistics", "", f"Command: `{command}`", "",
             f"Library source hash: `{source_hash()}`", "",
             "Totals cover the whole command: the setup (upload, autotuning, the Lanczos runs of the low-rank "
             "corrections: `k_axpy_cols`, `k_dot<double, 8>`, copies) and every timed solve.", "",
             "| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
    for r in rows[:30]:
        name = r["Name"].replace("|", "/")
        if len(name) > 110:
            name = name[:110] + "..."
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    open(out, "w").write("\n".join(lines) + "\n")


def _counter_rows(path, counter):
    rows = list(csv.DictReader(open(path)))
    out = []
    for r in rows:
        name = r.get("Counter_Name") or r.get("Counter")
        if name != counter:
            continue
        out.append((r["Kernel_Name"], float(r.get("Counter_Value") or r.get("Value")),
                    int(r.get("Dispatch_Id", 0))))
    return out


def traffic(fetch_csv, write_csv, kernel, copy_bytes, out, command):
    res = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = _counter_rows(path, counter)
        # per-dispatch values summed over the counter's instances
        per = {}
        for name, val, did in rows:
            per.setdefault((name, did), 0.0)
            per[(name, did)] += val
        copy = [v for (nm, _), v in per.items() if "copy" in nm.lower() or "elementwise" in nm.lower()]
        kern = [v for (nm, _), v in per.items() if kernel in nm]
        if not copy or not kern:
            raise SystemExit(f"{counter}: copy or kernel dispatches not found")
        copy_kib = max(copy)
        factor = copy_bytes / (copy_kib * 1024.0)
        avg_kib = sum(kern) / len(kern)
        res[counter] = dict(copy_kib=copy_kib, factor=factor, kernel_avg_kib=avg_kib,
                            kernel_bytes=avg_kib * 1024.0 * factor, dispatches=len(kern))
    total = res["FETCH_SIZE"]["kernel_bytes"] + res["WRITE_SIZE"]["kernel_bytes"]
    info = dict(kernel=kernel, source_hash=source_hash(), traffic_bytes_per_launch=total, counters=res,
                command=command)
    json.dump(info, open(os.path.splitext(out)[0] + ".json", "w"), indent=1)
    lines = [f"# HBM traffic of `{kernel}` (rocprofv3 counters)", "", f"Command: `{command}`", "",
             f"Library source hash: `{source_hash()}`", ""]
    for cn, v in res.items():
        lines.append(f"- {cn}: kernel average {v['kernel_avg_kib']:.0f} KiB over {v['dispatches']} dispatches; "
                     f"copy of {copy_bytes} bytes reads {v['copy_kib']:.0f} KiB -> factor {v['factor']:.4f}; "
                     f"calibrated {v['kernel_bytes'] / 1e6:.1f} MB per launch")
    lines.append(f"- total: {total / 1e6:.1f} MB per launch")
    open(out, "w").write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3], " ".join(sys.argv[4:]))
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], float(sys.argv[5]), sys.argv[6], " ".join(sys.argv[7:]))
