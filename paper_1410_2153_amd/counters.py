"""HBM traffic per launch of the Gauss-Seidel colour pass from two rocprofv3 counter runs.

Usage (after the two `rocprofv3 --pmc` runs of bench.py named in the output record):

    python -m paper_1410_2153_amd.counters <fetch counter_collection.csv> <write counter_collection.csv> \
        [out.json]

FETCH_SIZE and WRITE_SIZE are read in KiB per dispatch. Each is scaled by the ratio of the
bytes a plain device copy moves to what the same counter reads for that copy: the bench's
`--copy-calibration` runs a 512 MiB copy, whose dispatch is the largest `__amd_rocclr_copyBuffer`
in the run. The record is keyed by the SHA-256 of device.hip with comments and whitespace
removed (`source_key`), so bench.py reports it only for the kernel code it was measured on.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys

KERNEL = "asmg::k_sell<0, double>"
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DEVICE_SRC = os.path.join(ROOT, "paper_1410_2153_amd", "csrc", "device.hip")


def source_key(path=DEVICE_SRC):
    """SHA-256 of a C++/HIP source with comments and whitespace removed (code changes only)."""
    import re
    text = open(path, encoding="utf-8").read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    text = re.sub(r"\s+", "", text)
    return hashlib.sha256(text.encode()).hexdigest()
COPY_BYTES = 64 * 2 ** 20 * 8


def _per_dispatch(path, counter):
    vals, copies = [], []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        name = r["Kernel_Name"]
        v = float(r["Counter_Value"])
        if name.startswith("void " + KERNEL) or name.startswith(KERNEL):
            vals.append(v)
        elif name.startswith("__amd_rocclr_copyBuffer"):
            copies.append((int(r["Grid_Size"]), v))
    if not vals or not copies:
        raise SystemExit(f"{path}: no {KERNEL} or copy dispatches with {counter}")
    copy = max(copies)[1]  # the 512 MiB calibration copy has the largest grid
    return sum(vals) / len(vals), len(vals), copy


def record(fetch_csv, write_csv):
    f_kib, n, f_copy = _per_dispatch(fetch_csv, "FETCH_SIZE")
    w_kib, n2, w_copy = _per_dispatch(write_csv, "WRITE_SIZE")
    f_scale = COPY_BYTES / (f_copy * 1024.0)
    w_scale = COPY_BYTES / (w_copy * 1024.0)
    fb = f_kib * 1024.0 * f_scale
    wb = w_kib * 1024.0 * w_scale
    cmd = ("cd /tmp && rocprofv3 --pmc {c} --output-format csv -d <out>/pmc_{d} -o run -- python3 <repo>/bench.py "
           "--steps 1 --warmup 0 --no-cpu --batch-meshes 0 --no-extra --no-kernel-timing --copy-calibration")
    return {
        "kernel": KERNEL,
        "workload": "graded 2-D Delaunay mesh, 1002722 vertices, FP64 solve",
        "device_hip_code_key": source_key(),
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
        "commands": [cmd.format(c="FETCH_SIZE", d="fetch"), cmd.format(c="WRITE_SIZE", d="write"),
                     "python -m paper_1410_2153_amd.counters <out>/pmc_fetch/run_counter_collection.csv "
                     "<out>/pmc_write/run_counter_collection.csv profiles/traffic_k_sell_gs.json"],
    }


def main(argv):
    if len(argv) < 2:
        raise SystemExit(__doc__)
    rec = record(argv[0], argv[1])
    out = json.dumps(rec, indent=1)
    if len(argv) > 2:
        open(argv[2], "w").write(out + "\n")
    print(out)


if __name__ == "__main__":
    main(sys.argv[1:])


def stats_table(stats_csv, top=25):
    """Markdown table of a rocprofv3 `--stats` kernel summary (kernel, calls, total, average, share)."""
    rows = list(csv.DictReader(open(stats_csv)))
    out = ["| kernel | calls | total ms | avg us | % |", "|---|---:|---:|---:|---:|"]
    for r in rows[:top]:
        name = r["Name"].split("(")[0].replace("void ", "")
        out.append(f"| `{name}` | {int(r['Calls'])} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['Percentage']):.1f} |")
    return "\n".join(out)
