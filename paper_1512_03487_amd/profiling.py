"""Summaries of rocprofv3 output for the hopping kernels (HBM traffic per launch, kernel times).

rocprofv3's FETCH_SIZE and WRITE_SIZE counters are in KiB per dispatch; on gfx950 they are
calibrated here against a plain device copy of known size run in the same command (a 256 MiB copy:
the bytes it must read and write divided by what the counters report).

Usage:
  python -m paper_1512_03487_amd.profiling traffic FETCH_DIR WRITE_DIR KERNEL_SUBSTR OUT.txt [--grid N] [--cmd "..."]
  python -m paper_1512_03487_amd.profiling stats KT_DIR OUT.txt [--focus SUBSTR ...] [--cmd "..."]
  python -m paper_1512_03487_amd.profiling counters DIR[,DIR...] KERNEL_SUBSTR OUT.txt [--grid N] [--cmd "..."]
  python -m paper_1512_03487_amd.profiling table DIR OUT.txt --focus SUBSTR [--focus ...] [--cmd "..."]

--grid N keeps only dispatches of N work-items (one launch shape of a kernel that several
workloads share). The stats summary lists each kernel per launch shape as well.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import os
import sys

COPY_BYTES = 256 << 20
COPY_KERNEL = "copyBuffer"
TOP = 40   # rows per table of the stats summary


def _rows(d):
    out = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        out += list(csv.DictReader(open(f)))
    return out


def _per_kernel(rows, counter, substr, grid=None):
    return [float(r["Counter_Value"]) for r in rows if r["Counter_Name"] == counter and substr in r["Kernel_Name"]
            and (grid is None or int(r["Grid_Size"]) == grid)]


def _calibration_copies(rows, counter, n=3):
    """Counter values of the calibration copy: the command's last n copy dispatches (bench.py
    --calibrate-copy runs a 256 MiB device copy three times after everything else; the fields'
    own copies come earlier and have other sizes)."""
    rows = [r for r in rows if r["Counter_Name"] == counter and COPY_KERNEL in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return [float(r["Counter_Value"]) for r in rows[-n:]]


def kernel_source_hash(root):
    h = hashlib.sha256()
    for f in ("dhop.hip", "device.h"):
        with open(os.path.join(root, "paper_1512_03487_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic(fetch_dir, write_dir, kernel, out, cmd="", grid=None):
    fr, wr = _rows(fetch_dir), _rows(write_dir)
    fk, wk = _per_kernel(fr, "FETCH_SIZE", kernel, grid), _per_kernel(wr, "WRITE_SIZE", kernel, grid)
    fc, wc = _calibration_copies(fr, "FETCH_SIZE"), _calibration_copies(wr, "WRITE_SIZE")
    if not fk or not wk or not fc or not wc:
        raise SystemExit("missing kernel or copy dispatches in the counter output")
    f_factor = COPY_BYTES / (sum(fc) / len(fc) * 1024)
    w_factor = COPY_BYTES / (sum(wc) / len(wc) * 1024)
    f_b = sum(fk) / len(fk) * 1024 * f_factor
    w_b = sum(wk) / len(wk) * 1024 * w_factor
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    with open(out, "w") as fh:
        fh.write(f"# HBM traffic per dispatch of kernels matching '{kernel}'"
                 + (f" launched with {grid} work-items" if grid else "") + " (rocprofv3 --pmc)\n")
        if cmd:
            fh.write(f"# command: {cmd}\n")
        fh.write(f"dispatches_fetch: {len(fk)}\ndispatches_write: {len(wk)}\n")
        fh.write(f"fetch_kib_per_dispatch_raw: {sum(fk) / len(fk):.1f}\n")
        fh.write(f"write_kib_per_dispatch_raw: {sum(wk) / len(wk):.1f}\n")
        fh.write(f"copy_calibration_fetch_factor: {f_factor:.4f}\n")
        fh.write(f"copy_calibration_write_factor: {w_factor:.4f}\n")
        fh.write(f"hbm_read_bytes_per_launch: {f_b:.0f}\n")
        fh.write(f"hbm_write_bytes_per_launch: {w_b:.0f}\n")
        fh.write(f"hbm_bytes_per_launch: {f_b + w_b:.0f}\n")
        fh.write(f"source_sha256: {kernel_source_hash(root)}\n")
    print(open(out).read())


def counters(dirs, kernel, out, cmd="", grid=None):
    """Median per dispatch of every counter found under the given output directories (one
    rocprofv3 --pmc pass each, comma-separated) for the kernels matching `kernel`."""
    vals = {}
    for d in dirs.split(","):
        for r in _rows(d):
            if kernel in r["Kernel_Name"] and (grid is None or int(r["Grid_Size"]) == grid):
                vals.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    if not vals:
        raise SystemExit("no dispatches of " + kernel)
    with open(out, "w") as fh:
        fh.write(f"# counters per dispatch (median) of kernels matching '{kernel}'"
                 + (f" launched with {grid} work-items" if grid else "") + " (rocprofv3 --pmc)\n")
        if cmd:
            fh.write(f"# command: {cmd}\n")
        for k in sorted(vals):
            v = sorted(vals[k])
            fh.write(f"{k}: {v[len(v) // 2]:.6g}   (dispatches {len(v)})\n")
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        fh.write(f"source_sha256: {kernel_source_hash(root)}\n")
    print(open(out).read())


def table(d, out, cmd="", focus=()):
    """One row per (kernel, launch shape) matching any of `focus`: the median per dispatch of every
    counter in the pass under `d`."""
    groups = {}
    for r in _rows(d):
        if any(f in r["Kernel_Name"] for f in focus):
            key = (r["Kernel_Name"], int(r["Grid_Size"]))
            groups.setdefault(key, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    if not groups:
        raise SystemExit("no dispatches of " + str(focus))
    names = sorted({c for v in groups.values() for c in v})
    with open(out, "w") as fh:
        fh.write("# counters per dispatch (median) by kernel and launch shape (rocprofv3 --pmc)\n")
        if cmd:
            fh.write(f"# command: {cmd}\n")
        fh.write("\n| kernel | work-items | dispatches | " + " | ".join(names) + " |\n")
        fh.write("|---|---|---|" + "---|" * len(names) + "\n")
        for (name, n), v in sorted(groups.items()):
            short = name if len(name) <= 90 else name[:90] + "..."
            cells = []
            for c in names:
                x = sorted(v.get(c, []))
                cells.append(f"{x[len(x) // 2]:.4g}" if x else "")
            fh.write(f"| `{short}` | {n} | {len(next(iter(v.values())))} | " + " | ".join(cells) + " |\n")
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        fh.write(f"\nsource_sha256: {kernel_source_hash(root)}\n")
    print(open(out).read())


def stats(kt_dir, out, cmd="", focus=()):
    files = glob.glob(os.path.join(kt_dir, "**", "*kernel_stats.csv"), recursive=True)
    if not files:
        raise SystemExit("no kernel_stats.csv under " + kt_dir)
    rows = list(csv.DictReader(open(files[0])))
    with open(out, "w") as fh:
        fh.write("# rocprofv3 --kernel-trace --stats summary\n")
        if cmd:
            fh.write(f"# command: {cmd}\n")
        fh.write(f"Top {min(len(rows), TOP)} of {len(rows)} kernels by total time:\n\n")
        fh.write("| kernel | calls | avg us | min us | max us | total % |\n|---|---|---|---|---|---|\n")
        for r in rows[:TOP]:
            name = r["Name"]
            if len(name) > 110:
                name = name[:110] + "..."
            fh.write(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                     f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.1f} |\n")
        traces = glob.glob(os.path.join(kt_dir, "**", "*kernel_trace.csv"), recursive=True)
        if traces:
            groups = {}
            for r in csv.DictReader(open(traces[0])):
                key = (r["Kernel_Name"], int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"]))
                groups.setdefault(key, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
            ranked = sorted(groups.items(), key=lambda kv: -sum(kv[1]))
            picked = [kv for kv in ranked if any(f in kv[0][0] for f in focus)]
            picked += [kv for kv in ranked[:TOP] if kv not in picked]
            fh.write(f"\nPer launch shape (work-items per dispatch): the kernels matching {list(focus)}, then the top "
                     f"{min(len(groups), TOP)} of {len(groups)} by total time:\n\n")
            fh.write("| kernel | work-items | calls | avg us | min us | max us |\n|---|---|---|---|---|---|\n")
            for (name, n), v in picked:
                if len(name) > 110:
                    name = name[:110] + "..."
                fh.write(f"| `{name}` | {n} | {len(v)} | {sum(v) / len(v):.2f} | {min(v):.2f} | {max(v):.2f} |\n")
    print(open(out).read())


if __name__ == "__main__":
    args = sys.argv[1:]
    cmd = ""
    if "--cmd" in args:
        i = args.index("--cmd")
        cmd = args[i + 1]
        args = args[:i] + args[i + 2:]
    grid = None
    if "--grid" in args:
        i = args.index("--grid")
        grid = int(args[i + 1])
        args = args[:i] + args[i + 2:]
    focus = []
    while "--focus" in args:
        i = args.index("--focus")
        focus.append(args[i + 1])
        args = args[:i] + args[i + 2:]
    if args and args[0] == "traffic":
        traffic(*args[1:5], cmd=cmd, grid=grid)
    elif args and args[0] == "counters":
        counters(*args[1:4], cmd=cmd, grid=grid)
    elif args and args[0] == "table":
        table(*args[1:3], cmd=cmd, focus=tuple(focus))
    elif args and args[0] == "stats":
        stats(*args[1:3], cmd=cmd, focus=tuple(focus))
    else:
        print(__doc__)
