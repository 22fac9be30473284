"""Summaries of rocprofv3 output for the committed profile notes.

    python -m paper_2407_05930_amd.profiling window <kernel_trace.csv> <out.md> [--what=<title>] <command...>
    python -m paper_2407_05930_amd.profiling traffic <fetch_counter_collection.csv>
        <write_counter_collection.csv> <kernel name> <copy bytes> <out.md> <command...>
    python -m paper_2407_05930_amd.profiling counters <counter_collection.csv> <out.md> <command...>
    python -m paper_2407_05930_amd.profiling vcycle <fetch.csv> <write.csv> <l2.csv> <copy bytes>
        <bench.json> <out.md> <command...>

``window`` keeps the dispatches between the two int16 fill kernels that
bench.py launches just before and just after the timed steps of the headline
solve (setup, autotuning and the other legs fall outside), and tabulates
them per kernel function.  ``traffic`` scales each counter of the named
kernel (dispatches inside the window) by the ratio between the known size of
a plain device copy and what the same counter reads for that copy (rocprofv3
reports FETCH_SIZE / WRITE_SIZE in KiB).  ``counters`` averages every counter
per kernel function inside the window.
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


MARKER = "FillFunctor<short>"   # the int16 fill bench.py launches around the timed steps


def short_name(name):
    """Kernel function as the library's timers name it: no return type,
    namespace or argument list ("void msp::k_op_dot<32>(long, ...)" ->
    "k_op_dot<32>")."""
    n = name.strip()
    if n.startswith("void "):
        n = n[5:]
    n = n.replace("msp::", "")
    depth = 0
    for i, ch in enumerate(n):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return n[:i]
    return n


def _in_window(rows, order_key):
    """Rows strictly between the first and the last marker dispatch (all rows
    when the markers are missing), in dispatch order; flag says which."""
    rows = sorted(rows, key=order_key)
    marks = [i for i, r in enumerate(rows) if MARKER in r["Kernel_Name"]]
    if len(marks) < 2:
        return rows, False
    return [r for r in rows[marks[0] + 1:marks[-1]] if MARKER not in r["Kernel_Name"]], True


def window(path, out, command, what="the timed headline solves"):
    rows = list(csv.DictReader(open(path)))
    rows, found = _in_window(rows, lambda r: int(r["Start_Timestamp"]))
    per = {}
    for r in rows:
        d = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        e = per.setdefault(short_name(r["Kernel_Name"]), [0, 0])
        e[0] += 1
        e[1] += d
    total = sum(v[1] for v in per.values()) or 1
    span = (int(rows[-1]["End_Timestamp"]) - int(rows[0]["Start_Timestamp"])) if rows else 0
    lines = [f"# rocprofv3 kernel statistics of {what}", "", f"Command: `{command}`", "",
             f"Library source hash: `{source_hash()}`", "",
             ("Only the dispatches between the two int16 fill markers that bench.py launches around its timed steps "
              "are counted (no setup, autotuning or Lanczos kernels)." if found else
              "The window markers were not found: every dispatch of the command is counted."), "",
             f"Dispatches: {len(rows)}; kernel busy time {total / 1e6:.3f} ms; window span {span / 1e6:.3f} ms.", "",
             "| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
    for name, (cnt, ns) in sorted(per.items(), key=lambda kv: -kv[1][1]):
        nm = name.replace("|", "/")
        if len(nm) > 140:
            nm = nm[:140] + "..."
        lines.append(f"| `{nm}` | {cnt} | {ns / 1e6:.3f} | {ns / cnt / 1e3:.2f} | {100.0 * ns / total:.2f} |")
    open(out, "w").write("\n".join(lines) + "\n")
    json.dump({name: dict(calls=c, total_ns=t, avg_ns=t / c) for name, (c, t) in per.items()},
              open(os.path.splitext(out)[0] + ".json", "w"), indent=1)


def _dispatches(path):
    """{(kernel, dispatch id): {counter: value summed over its instances}} for the
    dispatches inside the marker window, and the copy dispatches outside it."""
    rows = list(csv.DictReader(open(path)))
    per = {}
    for r in rows:
        name = r.get("Counter_Name") or r.get("Counter")
        key = (r["Kernel_Name"], int(r.get("Dispatch_Id", 0)))
        d = per.setdefault(key, {})
        d[name] = d.get(name, 0.0) + float(r.get("Counter_Value") or r.get("Value"))
    items = [dict(Kernel_Name=k[0], Dispatch_Id=k[1], values=v) for k, v in per.items()]
    inside, found = _in_window(items, lambda r: r["Dispatch_Id"])
    return items, inside, found


def traffic(fetch_csv, write_csv, kernel, copy_bytes, out, command):
    res = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        items, inside, found = _dispatches(path)
        copy = [r["values"][counter] for r in items if "copy" in r["Kernel_Name"].lower() and counter in r["values"]]
        kern = [r["values"][counter] for r in inside if short_name(r["Kernel_Name"]) == kernel and counter in r["values"]]
        if not copy or not kern:
            raise SystemExit(f"{counter}: copy or kernel dispatches not found")
        copy_kib = max(copy)
        factor = copy_bytes / (copy_kib * 1024.0)
        avg_kib = sum(kern) / len(kern)
        res[counter] = dict(copy_kib=copy_kib, factor=factor, kernel_avg_kib=avg_kib,
                            kernel_bytes=avg_kib * 1024.0 * factor, dispatches=len(kern), window=found)
    total = res["FETCH_SIZE"]["kernel_bytes"] + res["WRITE_SIZE"]["kernel_bytes"]
    info = dict(kernel=kernel, source_hash=source_hash(), traffic_bytes_per_launch=total, counters=res,
                command=command)
    json.dump(info, open(os.path.splitext(out)[0] + ".json", "w"), indent=1)
    lines = [f"# HBM traffic of `{kernel}` (rocprofv3 counters)", "", f"Command: `{command}`", "",
             f"Library source hash: `{source_hash()}`", "",
             "Dispatches of the timed headline solves only (between the bench's window markers)." if
             res["FETCH_SIZE"]["window"] else "All dispatches of the command (window markers not found).", ""]
    for cn, v in res.items():
        lines.append(f"- {cn}: kernel average {v['kernel_avg_kib']:.0f} KiB over {v['dispatches']} dispatches; "
                     f"copy of {copy_bytes:.0f} bytes reads {v['copy_kib']:.0f} KiB -> factor {v['factor']:.4f}; "
                     f"calibrated {v['kernel_bytes'] / 1e6:.1f} MB per launch")
    lines.append(f"- total: {total / 1e6:.1f} MB per launch")
    open(out, "w").write("\n".join(lines) + "\n")


def counters(path, out, command):
    """Average of every collected counter per kernel function inside the window."""
    items, inside, found = _dispatches(path)
    per = {}
    for r in inside:
        e = per.setdefault(short_name(r["Kernel_Name"]), dict(n=0, sums={}))
        e["n"] += 1
        for cn, v in r["values"].items():
            e["sums"][cn] = e["sums"].get(cn, 0.0) + v
    names = sorted({cn for e in per.values() for cn in e["sums"]})
    lines = ["# rocprofv3 counters per kernel function (timed headline solves)", "", f"Command: `{command}`", "",
             f"Library source hash: `{source_hash()}`", "",
             "Per-dispatch averages over the dispatches between the bench's window markers." if found else
             "Per-dispatch averages over every dispatch of the command (window markers not found).", "",
             "| kernel | dispatches | " + " | ".join(names) + " |", "|---|---|" + "---|" * len(names)]
    for name, e in sorted(per.items(), key=lambda kv: kv[0]):
        nm = name.replace("|", "/")
        if len(nm) > 110:
            nm = nm[:110] + "..."
        vals = " | ".join(f"{e['sums'].get(cn, 0.0) / e['n']:.0f}" for cn in names)
        lines.append(f"| `{nm}` | {e['n']} | {vals} |")
    open(out, "w").write("\n".join(lines) + "\n")


VCYCLE_KERNELS = ("k_spmm", "k_sell", "k_pack_sets", "k_dense_sets", "k_dense_part", "k_dense_sum")


def vcycle_order(nlev):
    """Classes of one V(1,1) cycle's dispatches in launch order with the
    explicit smoother: per level M, A, R on the way down, the two kernels of
    the coarsest solve, then P, A, M on the way up."""
    down = [f"L{l}.{k}" for l in range(nlev) for k in ("M", "A", "R")]
    up = [f"L{l}.{k}" for l in reversed(range(nlev)) for k in ("P", "A", "M")]
    return down + ["coarsest.1", "coarsest.2"] + up


def _label_vcycles(inside):
    """Label the dispatches of every V-cycle (a maximal run of V-cycle
    kernels between PCG kernels) by class; runs of another length stay
    unlabelled."""
    out, run = [], []

    def flush():
        if run and (len(run) - 2) % 6 == 0 and len(run) >= 8:
            for r, cls in zip(run, vcycle_order((len(run) - 2) // 6)):
                out.append((cls, r))
        run.clear()

    for r in inside:
        if short_name(r["Kernel_Name"]).startswith(VCYCLE_KERNELS):
            run.append(r)
        else:
            flush()
    flush()
    return out


def vcycle_classes(fetch_csv, write_csv, l2_csv, copy_bytes, bench_json, out, command):
    """Per V-cycle class: calibrated FETCH/WRITE bytes per launch against the
    bench's algorithmic bytes, and the L2 / L1 request counters."""
    per = {}
    factors = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv), (None, l2_csv)):
        items, inside, found = _dispatches(path)
        if counter:
            copy = [r["values"][counter] for r in items if "copy" in r["Kernel_Name"].lower() and counter in r["values"]]
            factors[counter] = copy_bytes / (max(copy) * 1024.0)
        for cls, r in _label_vcycles(inside):
            e = per.setdefault(cls, dict(kernel=short_name(r["Kernel_Name"]), n={}, sums={}))
            for cn, v in r["values"].items():
                if counter and cn == counter:
                    v = v * 1024.0 * factors[counter]
                e["sums"][cn] = e["sums"].get(cn, 0.0) + v
                e["n"][cn] = e["n"].get(cn, 0) + 1
    alg = {}
    if bench_json:
        d = json.loads(open(bench_json).read().strip().splitlines()[-1])
        for kind, v in d.get("kernel_breakdown_mixed", {}).items():
            if v.get("GBs") and v.get("launches"):
                alg[kind] = v["GBs"] * 1e9 * v["ms"] * 1e-3 / v["launches"]
    avg = lambda e, cn: e["sums"][cn] / e["n"][cn] if cn in e["sums"] else float("nan")  # noqa: E731
    lines = ["# V-cycle traffic and cache counters per class (timed headline solves)", "",
             f"Command: `{command}`", "", f"Library source hash: `{source_hash()}`", "",
             "Every dispatch of a V-cycle inside the bench's window markers is labelled by its position in the cycle "
             "(per level M, A, R down; the coarsest solve's two kernels; P, A, M up). FETCH_SIZE and WRITE_SIZE are "
             f"calibrated by a {copy_bytes:.0f}-byte device copy (factors {factors.get('FETCH_SIZE', 0):.4f}, "
             f"{factors.get('WRITE_SIZE', 0):.4f}); 'alg' is bench.py's algorithmic bytes per launch of the class. "
             "TCC_HIT / TCC_MISS count L2 requests (hit rate = hits / (hits + misses)); TCP_TCC_READ_REQ counts the "
             "read requests the vector L1 caches send to L2.", "",
             "| class | kernel | alg MB | fetch MB | write MB | (fetch+write)/alg | L2 hit % | L1->L2 reads (M) |",
             "|---|---|---|---|---|---|---|---|"]
    js = {}
    for cls in sorted(per, key=lambda c: (c.startswith("coarsest"), c)):
        e = per[cls]
        f, w = avg(e, "FETCH_SIZE"), avg(e, "WRITE_SIZE")
        h, m_ = avg(e, "TCC_HIT_sum"), avg(e, "TCC_MISS_sum")
        rq = avg(e, "TCP_TCC_READ_REQ_sum")
        # the coarsest solve's bytes are the second kernel's (the first packs the columns by subsystem)
        key = {"coarsest.1": None, "coarsest.2": "dense_coarse"}.get(cls, cls)
        a = alg.get(key) if key else None
        ratio = (f + w) / a if a else float("nan")
        hit = 100.0 * h / (h + m_) if h == h and m_ == m_ and h + m_ > 0 else float("nan")
        lines.append(f"| {cls} | `{e['kernel']}` | {a / 1e6 if a else float('nan'):.1f} | {f / 1e6:.1f} | "
                     f"{w / 1e6:.1f} | {ratio:.2f} | {hit:.0f} | {rq / 1e6:.2f} |")
        js[cls] = dict(kernel=e["kernel"], alg_bytes=a, fetch_bytes=f, write_bytes=w, l2_hit_pct=hit,
                       l1_l2_read_req=rq)
    open(out, "w").write("\n".join(lines) + "\n")
    json.dump(js, open(os.path.splitext(out)[0] + ".json", "w"), indent=1)


if __name__ == "__main__":
    if sys.argv[1] == "window":
        if sys.argv[4].startswith("--what="):
            window(sys.argv[2], sys.argv[3], " ".join(sys.argv[5:]), sys.argv[4][len("--what="):])
        else:
            window(sys.argv[2], sys.argv[3], " ".join(sys.argv[4:]))
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], float(sys.argv[5]), sys.argv[6], " ".join(sys.argv[7:]))
    elif sys.argv[1] == "counters":
        counters(sys.argv[2], sys.argv[3], " ".join(sys.argv[4:]))
    elif sys.argv[1] == "vcycle":
        vcycle_classes(sys.argv[2], sys.argv[3], sys.argv[4], float(sys.argv[5]), sys.argv[6], sys.argv[7],
                       " ".join(sys.argv[8:]))
    else:
        raise SystemExit(__doc__)
