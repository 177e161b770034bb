"""Profile summaries of the Gauss-Seidel colour pass from rocprofv3 output.

Usage:

    python -m paper_1410_2153_amd.counters traffic <fetch counter_collection.csv> \
        <write counter_collection.csv> [out.json]
    python -m paper_1410_2153_amd.counters stats <kernel_stats.csv> [top]
    python -m paper_1410_2153_amd.counters phases <kernel_trace.csv> [kernel]
    python -m paper_1410_2153_amd.counters markers <marker_api_trace.csv>

traffic: HBM bytes per launch from the two `rocprofv3 --pmc` runs of bench.py named in the
output record. FETCH_SIZE and WRITE_SIZE are read in KiB per dispatch. Each is scaled by the
ratio of the bytes a plain device copy moves to what the same counter reads for that copy: the
bench's `--copy-calibration` runs a 512 MiB copy, whose dispatch is the largest
`__amd_rocclr_copyBuffer` in the run. The counter runs use `--autotune 0` (every launch site in
the default shape), so that the autotuner's trial launches in other shapes are not averaged in.
The record is keyed by the SHA-256 of the kernel sources with comments and whitespace removed
(`source_key`), so bench.py reports it only for the kernel code it was measured on.

stats: markdown table of a `--stats` kernel summary.

markers: the library's named ranges (roctx, `--marker-trace`) in the order they opened, with
their durations: setup phases, device layout, autotuning, solves.

phases: splits a `--kernel-trace` timeline at idle gaps over 200 us (host work between the
bench's phases: autotuning, timed solves, per-launch timing, B_co loops) and gives the kernel's
launch count and mean duration per phase.
"""
from __future__ import annotations

import collections
import csv
import hashlib
import json
import os
import re
import sys

KERNEL = "asmg::k_sell<0, double>"
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SRCS = [os.path.join(ROOT, "paper_1410_2153_amd", "csrc", f) for f in ("device.hip", "common.hpp")]
COPY_BYTES = 64 * 2 ** 20 * 8


def source_key(paths=KERNEL_SRCS):
    """SHA-256 of C++/HIP sources with comments and whitespace removed (code changes only)."""
    h = hashlib.sha256()
    for path in paths:
        text = open(path, encoding="utf-8").read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(re.sub(r"\s+", "", text).encode())
    return h.hexdigest()


def _name(kernel_name):
    return kernel_name.split("(")[0].replace("void ", "")


def _per_dispatch(path, counter):
    vals, copies = [], []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        name = _name(r["Kernel_Name"])
        v = float(r["Counter_Value"])
        if name == KERNEL:
            vals.append(v)
        elif name.startswith("__amd_rocclr_copyBuffer"):
            copies.append((int(r["Grid_Size"]), v))
    if not vals or not copies:
        raise SystemExit(f"{path}: no {KERNEL} or copy dispatches with {counter}")
    copy = max(copies)[1]  # the 512 MiB calibration copy has the largest grid
    return sum(vals) / len(vals), len(vals), copy


def _bco_kernel(name, prec):
    """True for the kernels of one B_co application in precision prec ("double" or "float"):
    colour passes, residuals, transfers, the bottom GEMV and a first pass run on its own."""
    if not name.startswith("asmg::"):
        return False
    k = name[len("asmg::"):]
    if k == "k_gs_first_cvt":
        return prec == "float"
    # position of the value type among the template arguments
    pos = {"k_sell": 1, "k_sell_spmv": 2, "k_gemv": 0, "k_gs_first": 0}
    base, _, args = k.partition("<")
    if base not in pos or not args:
        return False
    targs = args.rstrip(">").replace(" ", "").split(",")
    return len(targs) > pos[base] and targs[pos[base]] == prec


def bco_traffic(fetch_csv, write_csv, f_scale, w_scale):
    """HBM bytes per B_co application from the counter runs (FP64 and FP32 V-cycle kernels; the
    number of applications is the number of bottom GEMV dispatches in that precision)."""
    out = {}
    for prec, key in (("double", "fp64"), ("float", "fp32")):
        tot = {}
        for path, counter, scale in ((fetch_csv, "FETCH_SIZE", f_scale), (write_csv, "WRITE_SIZE", w_scale)):
            s, napp = 0.0, 0
            for r in csv.DictReader(open(path)):
                if r["Counter_Name"] != counter:
                    continue
                name = _name(r["Kernel_Name"])
                if _bco_kernel(name, prec):
                    s += float(r["Counter_Value"]) * 1024.0 * scale
                if name == f"asmg::k_gemv<{prec}>":
                    napp += 1
            tot[counter] = (s, napp)
        napp = tot["FETCH_SIZE"][1]
        if napp:
            fb, wb = tot["FETCH_SIZE"][0] / napp, tot["WRITE_SIZE"][0] / napp
            out[key] = {"applications": napp, "fetch_bytes": fb, "write_bytes": wb, "traffic_bytes": fb + wb}
    return out


def record(fetch_csv, write_csv):
    f_kib, n, f_copy = _per_dispatch(fetch_csv, "FETCH_SIZE")
    w_kib, n2, w_copy = _per_dispatch(write_csv, "WRITE_SIZE")
    f_scale = COPY_BYTES / (f_copy * 1024.0)
    w_scale = COPY_BYTES / (w_copy * 1024.0)
    fb = f_kib * 1024.0 * f_scale
    wb = w_kib * 1024.0 * w_scale
    cmd = ("cd /tmp && rocprofv3 --pmc {c} --output-format csv -d <out>/pmc_{d} -o run -- python3 <repo>/bench.py "
           "--steps 1 --warmup 0 --no-cpu --batch-meshes 0 --no-extra --no-kernel-timing --copy-calibration "
           "--autotune 0")
    return {
        "kernel": KERNEL,
        "workload": "graded 2-D Delaunay mesh, 1002722 vertices, FP64 solve",
        "launch_shape": "256 threads per block, XCD-contiguous block order at every launch site",
        "kernel_code_key": source_key(),
        "dispatches": n,
        "fetch_kib_per_dispatch_raw": f_kib,
        "write_kib_per_dispatch_raw": w_kib,
        "copy_reference_bytes": COPY_BYTES,
        "copy_fetch_kib_raw": f_copy,
        "copy_write_kib_raw": w_copy,
        "fetch_scale": f_scale,
        "write_scale": w_scale,
        "fetch_bytes_per_launch": fb,
        "write_bytes_per_launch": wb,
        "traffic_bytes_per_launch": fb + wb,
        "bco_per_application": bco_traffic(fetch_csv, write_csv, f_scale, w_scale),
        "commands": [cmd.format(c="FETCH_SIZE", d="fetch"), cmd.format(c="WRITE_SIZE", d="write"),
                     "python -m paper_1410_2153_amd.counters traffic <out>/pmc_fetch/run_counter_collection.csv "
                     "<out>/pmc_write/run_counter_collection.csv profiles/traffic_k_sell_gs.json"],
    }


def stats_table(stats_csv, top=25):
    """Markdown table of a rocprofv3 `--stats` kernel summary (kernel, calls, total, average, share)."""
    rows = list(csv.DictReader(open(stats_csv)))
    out = ["| kernel | calls | total ms | avg us | % |", "|---|---:|---:|---:|---:|"]
    for r in rows[:top]:
        out.append(f"| `{_name(r['Name'])}` | {int(r['Calls'])} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['Percentage']):.1f} |")
    return "\n".join(out)


def trace_phases(trace_csv, kernel=KERNEL, gap_us=200.0):
    """Per phase of a kernel trace (split at idle gaps): launches of `kernel`, their mean
    duration in us, their block sizes, and the phase's wall span in ms."""
    rows = sorted(csv.DictReader(open(trace_csv)), key=lambda r: int(r["Start_Timestamp"]))
    phases, cur = [], []
    for r in rows:
        if cur and int(r["Start_Timestamp"]) - int(cur[-1]["End_Timestamp"]) > gap_us * 1e3:
            phases.append(cur)
            cur = []
        cur.append(r)
    if cur:
        phases.append(cur)
    out = []
    for ph in phases:
        ks = [r for r in ph if _name(r["Kernel_Name"]) == kernel]
        if not ks:
            continue
        dur = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in ks]
        out.append({"launches": len(ks), "mean_us": sum(dur) / len(dur),
                    "block_sizes": dict(collections.Counter(int(r["Workgroup_Size_X"]) for r in ks)),
                    "span_ms": (int(ph[-1]["End_Timestamp"]) - int(ph[0]["Start_Timestamp"])) / 1e6})
    return out


def phases_table(trace_csv, kernel=KERNEL):
    out = [f"| phase | `{kernel}` launches | mean us | block sizes | span ms |", "|---:|---:|---:|---|---:|"]
    for i, p in enumerate(trace_phases(trace_csv, kernel)):
        sizes = ", ".join(f"{k}: {v}" for k, v in sorted(p["block_sizes"].items()))
        out.append(f"| {i} | {p['launches']} | {p['mean_us']:.2f} | {sizes} | {p['span_ms']:.1f} |")
    return "\n".join(out)


def markers_table(marker_csv):
    rows = sorted(csv.DictReader(open(marker_csv)), key=lambda r: int(r["Start_Timestamp"]))
    out = ["| range | ms |", "|---|---:|"]
    for r in rows:
        out.append(f"| `{r['Function']}` | {(int(r['End_Timestamp']) - int(r['Start_Timestamp'])) / 1e6:.2f} |")
    return "\n".join(out)


def main(argv):
    if len(argv) >= 3 and argv[0] == "traffic":
        out = json.dumps(record(argv[1], argv[2]), indent=1)
        if len(argv) > 3:
            open(argv[3], "w").write(out + "\n")
        print(out)
    elif len(argv) >= 2 and argv[0] == "stats":
        print(stats_table(argv[1], int(argv[2]) if len(argv) > 2 else 25))
    elif len(argv) >= 2 and argv[0] == "phases":
        print(phases_table(argv[1], argv[2] if len(argv) > 2 else KERNEL))
    elif len(argv) >= 2 and argv[0] == "markers":
        print(markers_table(argv[1]))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
