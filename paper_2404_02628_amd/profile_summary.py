"""Summaries of rocprofv3 output for the profiles/ notes.

    python -m paper_2404_02628_amd.profile_summary trace DIR
        per-kernel launch statistics from DIR/run_kernel_trace.csv (--kernel-trace), grouped by
        kernel name and grid size (so launches of different batch sizes stay apart)

    python -m paper_2404_02628_amd.profile_summary counters FETCH_DIR WRITE_DIR --copy-mib 512 \
            --kernel k_pair_f32 --replicas 64 --precision mixed
        FETCH_SIZE / WRITE_SIZE per dispatch (KiB) from two --pmc runs of profile_run, the
        scale factors that map each counter onto the bytes of the run's plain device copy
        (copy-mib MiB read and written), and the traffic record of the named kernel (mean
        counter values, scales, and the SHA-256 of the sources that define the kernel, so a
        reader can tell whether the record still describes the current code).

    python -m paper_2404_02628_amd.profile_summary pmc DIR [--kernel PREFIX ...]
        mean value per dispatch of every counter of one --pmc run, for the kernels whose short
        name starts with a given prefix
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import statistics
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# Sources whose change invalidates a kernel's counter record.
KERNEL_SOURCES = {
    "k_pair_sym_f32": ["paper_2404_02628_amd/csrc/k_pair.hip", "paper_2404_02628_amd/csrc/device_util.h",
                       "paper_2404_02628_amd/csrc/pimd_internal.h"],
    "k_pair_sym_f64": ["paper_2404_02628_amd/csrc/k_pair.hip", "paper_2404_02628_amd/csrc/device_util.h",
                       "paper_2404_02628_amd/csrc/pimd_internal.h", "paper_2404_02628_amd/csrc/fast_exp.h"],
    "k_pair_f32": ["paper_2404_02628_amd/csrc/k_pair.hip", "paper_2404_02628_amd/csrc/device_util.h",
                   "paper_2404_02628_amd/csrc/pimd_internal.h"],
    "k_pair_f64": ["paper_2404_02628_amd/csrc/k_pair.hip", "paper_2404_02628_amd/csrc/device_util.h",
                   "paper_2404_02628_amd/csrc/pimd_internal.h"],
    "k_recursion": ["paper_2404_02628_amd/csrc/k_exchange.hip", "paper_2404_02628_amd/csrc/fast_exp.h",
                    "paper_2404_02628_amd/csrc/device_util.h", "paper_2404_02628_amd/csrc/pimd_internal.h"],
    "k_integrate": ["paper_2404_02628_amd/csrc/k_integrate.hip", "paper_2404_02628_amd/csrc/nhc.h",
                    "paper_2404_02628_amd/csrc/fast_exp.h", "paper_2404_02628_amd/csrc/pimd_internal.h"],
    "k_springs": ["paper_2404_02628_amd/csrc/k_springs.hip", "paper_2404_02628_amd/csrc/pimd_internal.h"],
}


def sources_sha256(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(p.encode() + b"\0" + f.read() + b"\0")
    return h.hexdigest()


def short_name(name: str) -> str:
    base = name.split("(")[0]
    return base.replace("void ", "").replace("pimd::", "")


def _dispatches(d: str):
    """(kernel name, grid threads, duration us) per dispatch, from the CSV or the SQLite output."""
    csv_path = os.path.join(d, "run_kernel_trace.csv")
    if os.path.exists(csv_path):
        for r in csv.DictReader(open(csv_path)):
            grid = (int(r["Grid_Size"]) if "Grid_Size" in r
                    else int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"]))
            yield r["Kernel_Name"], grid, (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        return
    import sqlite3
    con = sqlite3.connect(os.path.join(d, "run_results.db"))
    for name, gx, gy, gz, dur in con.execute("select name, grid_x, grid_y, grid_z, duration from kernels"):
        yield name, gx * gy * gz, dur / 1e3


def trace(d: str):
    groups = defaultdict(list)
    for name, grid, dur in _dispatches(d):
        groups[(short_name(name), grid)].append(dur)
    total = sum(sum(v) for v in groups.values())
    out = ["| kernel | grid (threads) | launches | mean us | min us | max us | share |",
           "|---|---:|---:|---:|---:|---:|---:|"]
    for (k, g), v in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
        out.append(f"| `{k}` | {g} | {len(v)} | {statistics.fmean(v):.1f} | {min(v):.1f} | {max(v):.1f} | "
                   f"{sum(v) / total * 100:.1f}% |")
    return "\n".join(out)


def _counter_rows(d: str):
    """(kernel name, grid threads, counter value) per dispatch, from the CSV or the SQLite output."""
    csv_path = os.path.join(d, "run_counter_collection.csv")
    if os.path.exists(csv_path):
        return [(r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"])) for r in csv.DictReader(open(csv_path))]
    import sqlite3
    con = sqlite3.connect(os.path.join(d, "run_results.db"))
    return [(n, int(g), float(v)) for n, g, v in con.execute("select kernel_name, grid_size, value from counters_collection")]


def counters(fetch_dir, write_dir, copy_mib, kernel, replicas, precision):
    fr, wr = _counter_rows(fetch_dir), _counter_rows(write_dir)

    def per_kernel(rows):
        g = defaultdict(list)
        for name, grid, value in rows:
            g[short_name(name)].append((value, grid))
        return g

    fk, wk = per_kernel(fr), per_kernel(wr)
    copy_kib = copy_mib * 1024.0

    def copy_value(g):
        # the plain copy: the copyBuffer dispatch with the largest value
        cand = [v for k, vals in g.items() if "copyBuffer" in k for v, _ in vals]
        return max(cand) if cand else None

    fc, wc = copy_value(fk), copy_value(wk)
    fs = copy_kib / fc if fc else None
    ws = copy_kib / wc if wc else None
    lines = [f"plain device copy of {copy_mib} MiB: FETCH_SIZE {fc:.1f} KiB, WRITE_SIZE {wc:.1f} KiB "
             f"-> scale FETCH x{fs:.4f}, WRITE x{ws:.4f}", "",
             "| kernel | grid | dispatches | FETCH_SIZE KiB (mean) | WRITE_SIZE KiB (mean) | scaled MB / launch |",
             "|---|---:|---:|---:|---:|---:|"]
    keys = sorted(set((k, g) for k, vals in fk.items() for _, g in vals))
    for k, g in keys:
        fv = [v for v, gg in fk.get(k, []) if gg == g]
        wv = [v for v, gg in wk.get(k, []) if gg == g]
        if not fv or not wv or "copyBuffer" in k or "fillBuffer" in k or "elementwise" in k:
            continue
        mb = (statistics.fmean(fv) * fs + statistics.fmean(wv) * ws) * 1024 / 1e6
        lines.append(f"| `{k}` | {g} | {len(fv)} | {statistics.fmean(fv):.1f} | {statistics.fmean(wv):.1f} | {mb:.2f} |")
    rec = None
    kf = [v for kk, vals in fk.items() if kk.split("<")[0] == kernel for v, _ in vals]
    kw = [v for kk, vals in wk.items() if kk.split("<")[0] == kernel for v, _ in vals]
    if kf and kw:
        srcs = KERNEL_SOURCES.get(kernel, [])
        rec = {"kernel": kernel, "replicas": replicas, "precision": precision,
               "fetch_kib": round(statistics.fmean(kf), 3), "write_kib": round(statistics.fmean(kw), 3),
               "fetch_scale": round(fs, 6), "write_scale": round(ws, 6),
               "sources": srcs, "sources_sha256": sources_sha256(srcs)}
    return "\n".join(lines), rec


def _named_counter_rows(d: str):
    """(kernel name, grid threads, counter name, value) per dispatch and counter."""
    import glob
    rows = []
    for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        rows += [(r["Kernel_Name"], int(r["Grid_Size"]), r["Counter_Name"], float(r["Counter_Value"]))
                 for r in csv.DictReader(open(path))]
    if not rows:
        import sqlite3
        for path in glob.glob(os.path.join(d, "**", "*.db"), recursive=True):
            con = sqlite3.connect(path)
            rows += [(n, int(g), c, float(v)) for n, g, c, v in
                     con.execute("select kernel_name, grid_size, counter_name, value from counters_collection")]
    return rows


def pmc(d: str, kernels):
    """Mean value per dispatch of every collected counter, for the kernels whose short name starts
    with one of `kernels`."""
    g = defaultdict(lambda: defaultdict(list))
    for name, grid, cname, value in _named_counter_rows(d):
        k = short_name(name)
        if any(k.startswith(p) for p in kernels):
            g[(k, grid)][cname].append(value)
    lines = []
    for (k, grid), cs in sorted(g.items()):
        lines += [f"`{k}` (grid {grid} threads)", "", "| counter | dispatches | mean per dispatch |", "|---|---:|---:|"]
        lines += [f"| {c} | {len(v)} | {statistics.fmean(v):.6g} |" for c, v in sorted(cs.items())]
        lines.append("")
    return "\n".join(lines)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    c = sub.add_parser("counters")
    c.add_argument("fetch_dir")
    c.add_argument("write_dir")
    c.add_argument("--copy-mib", type=float, default=512)
    c.add_argument("--kernel", default="k_pair_f32")
    c.add_argument("--replicas", type=int, default=64)
    c.add_argument("--precision", default="mixed")
    m = sub.add_parser("pmc")
    m.add_argument("dir")
    m.add_argument("--kernel", action="append", default=[])
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        print(trace(a.dir))
    elif a.cmd == "pmc":
        print(pmc(a.dir, a.kernel or ["k_"]))
    else:
        table, rec = counters(a.fetch_dir, a.write_dir, a.copy_mib, a.kernel, a.replicas, a.precision)
        print(table)
        if rec is not None:
            print("\n```json traffic-record\n" + json.dumps(rec, indent=1) + "\n```")
    return 0


if __name__ == "__main__":
    sys.exit(main())
