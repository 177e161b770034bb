"""Profile summaries of the solver's kernels from rocprofv3 output.

Usage:

    python -m paper_1410_2153_amd.counters traffic <workload> <fetch counter_collection.csv> \
        <write counter_collection.csv> [out.json]
    python -m paper_1410_2153_amd.counters kernels <fetch csv> <write csv> [top]
    python -m paper_1410_2153_amd.counters stats <kernel_stats.csv> [top]
    python -m paper_1410_2153_amd.counters phases <kernel_trace.csv> [kernel]
    python -m paper_1410_2153_amd.counters markers <marker_api_trace.csv>

traffic: HBM bytes per launch of a workload's dominant kernel (WORKLOADS: the graded 2-D mesh,
the 3-D Kuhn cube, the batched 256-mesh workload) from two `rocprofv3 --pmc` runs of bench.py,
the commands named in the output record. FETCH_SIZE and WRITE_SIZE are read in KiB per
dispatch. Each is scaled by the ratio of the bytes a plain device copy moves to what the same
counter reads for that copy: the bench's `--copy-calibration` runs a 512 MiB copy, whose
dispatch is the largest `__amd_rocclr_copyBuffer` in the run. The counter runs use
`--autotune 0` (every launch site in the default shape), so that the autotuner's trial launches
in other shapes are not averaged in. The record is keyed by the SHA-256 of the kernel's sources
with comments and whitespace removed (`source_key`), so bench.py reports it only for the kernel
code it was measured on. It also gives the HBM bytes of one whole B_co application (every
V-cycle kernel of one precision, per application).

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

KERNEL = "asmg::k_sell<0, double, 0>"
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 64 * 2 ** 20 * 8


def _srcs(*names):
    return [os.path.join(ROOT, "paper_1410_2153_amd", "csrc", f) for f in names]


KERNEL_SRCS = _srcs("device.hip", "common.hpp")

# workload -> dominant kernel, the sources that define it, the bench selection of the counter runs
WORKLOADS = {
    "graded1M": dict(kernel="asmg::k_sell<0, double, 0>", sources=("device.hip", "common.hpp"),
                     bench="--only graded --no-extra", engine="single",
                     desc="graded 2-D Delaunay mesh, 1002722 vertices, FP64 and mixed solves"),
    "cube2M": dict(kernel="asmg::k_sell<0, double, 0>", sources=("device.hip", "common.hpp"),
                   bench="--only cube3d", engine="single",
                   desc="Kuhn cube 128^3 x 6 tetrahedra, 2048383 unknowns, FP64 and mixed solves"),
    "batched256x4": dict(kernel=("asmg::kb_sell<0, 4, double, 0>", "asmg::kb_sell<3, 4, double, 0>"),
                         sources=("batch.hip", "common.hpp"),
                         bench="--only batched", engine="batch",
                         desc="256 jittered squares (sides 32..512) x 4 right-hand sides, FP64 and mixed solves"),
}


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


def _per_dispatch(path, counter, kernel):
    """Mean counter value over the dispatches of `kernel` (a name, or a tuple of names averaged
    together), and the value for the calibration copy."""
    names = kernel if isinstance(kernel, tuple) else (kernel,)
    vals, copies = [], []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        name = _name(r["Kernel_Name"])
        v = float(r["Counter_Value"])
        if name in names:
            vals.append(v)
        elif name.startswith("__amd_rocclr_copyBuffer"):
            copies.append((int(r["Grid_Size"]), v))
    if not vals or not copies:
        raise SystemExit(f"{path}: no {kernel} or copy dispatches with {counter}")
    copy = max(copies)[1]  # the 512 MiB calibration copy has the largest grid
    return sum(vals) / len(vals), len(vals), copy


def _targs(name):
    base, _, args = name.partition("<")
    return base, [a for a in args.rstrip(">").replace(" ", "").split(",") if a]


def _bco_kernel(name, prec, engine="single"):
    """True for the kernels of one B_co application in precision prec ("double" or "float"):
    colour passes, residuals, transfers, bottom GEMVs and a first pass run on its own."""
    if not name.startswith("asmg::"):
        return False
    base, targs = _targs(name[len("asmg::"):])
    if engine == "batch":
        if base == "kb_first_cvt":
            return prec == "float"
        pos = {"kb_sell": 2, "kb_sell_spmv": 3, "kb_gemv": 1, "kb_first": 1}
    else:
        if base == "k_gs_first_cvt":
            return prec == "float"
        pos = {"k_sell": 1, "k_sell_spmv": 2, "k_gemv": 0, "k_gs_first": 0}
    return base in pos and len(targs) > pos[base] and targs[pos[base]] == prec


def _bco_application(name, prec, engine):
    """One dispatch per B_co application: the bottom GEMV (single mesh) or r.z (batched)."""
    if engine == "batch":
        base, targs = _targs(name[len("asmg::"):]) if name.startswith("asmg::") else ("", [])
        return base == "kb_cg_rz" and len(targs) > 1 and targs[1] == prec
    return name == f"asmg::k_gemv<{prec}>"


def bco_traffic(fetch_csv, write_csv, f_scale, w_scale, engine="single"):
    """HBM bytes per B_co application from the counter runs (FP64 and FP32 V-cycle kernels)."""
    out = {}
    for prec, key in (("double", "fp64"), ("float", "fp32")):
        tot = {}
        for path, counter, scale in ((fetch_csv, "FETCH_SIZE", f_scale), (write_csv, "WRITE_SIZE", w_scale)):
            s, napp = 0.0, 0
            for r in csv.DictReader(open(path)):
                if r["Counter_Name"] != counter:
                    continue
                name = _name(r["Kernel_Name"])
                if _bco_kernel(name, prec, engine):
                    s += float(r["Counter_Value"]) * 1024.0 * scale
                if _bco_application(name, prec, engine):
                    napp += 1
            tot[counter] = (s, napp)
        napp = tot["FETCH_SIZE"][1]
        if napp:
            fb, wb = tot["FETCH_SIZE"][0] / napp, tot["WRITE_SIZE"][0] / napp
            out[key] = {"applications": napp, "fetch_bytes": fb, "write_bytes": wb, "traffic_bytes": fb + wb}
    return out


def record(workload, fetch_csv, write_csv):
    wl = WORKLOADS[workload]
    kernel = wl["kernel"]
    f_kib, n, f_copy = _per_dispatch(fetch_csv, "FETCH_SIZE", kernel)
    w_kib, n2, w_copy = _per_dispatch(write_csv, "WRITE_SIZE", kernel)
    f_scale = COPY_BYTES / (f_copy * 1024.0)
    w_scale = COPY_BYTES / (w_copy * 1024.0)
    fb = f_kib * 1024.0 * f_scale
    wb = w_kib * 1024.0 * w_scale
    cmd = ("cd /tmp && timeout -s KILL 600 rocprofv3 --pmc {c} --output-format csv -d <out>/pmc_{d} -o run -- "
           "python3 <repo>/bench.py --steps 1 --warmup 0 " + wl["bench"] +
           " --no-kernel-timing --copy-calibration --autotune 0")
    return {
        "kernel": " and ".join(kernel) if isinstance(kernel, tuple) else kernel,
        "workload": wl["desc"],
        "launch_shape": "256 threads per block, XCD-contiguous block order at every launch site",
        "kernel_code_key": source_key(_srcs(*wl["sources"])),
        "kernel_sources": list(wl["sources"]),
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
        "bco_per_application": bco_traffic(fetch_csv, write_csv, f_scale, w_scale, wl["engine"]),
        "commands": [cmd.format(c="FETCH_SIZE", d="fetch"), cmd.format(c="WRITE_SIZE", d="write"),
                     f"python -m paper_1410_2153_amd.counters traffic {workload} "
                     "<out>/pmc_fetch/run_counter_collection.csv <out>/pmc_write/run_counter_collection.csv "
                     f"profiles/traffic_{workload}.json"],
    }


def per_kernel_traffic(fetch_csv, write_csv, top=20):
    """Markdown table: mean scaled HBM bytes (fetch + write) per dispatch of every kernel."""
    tabs = {}
    for path, counter in ((fetch_csv, "FETCH_SIZE"), (write_csv, "WRITE_SIZE")):
        copies, per = [], collections.defaultdict(list)
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            name = _name(r["Kernel_Name"])
            if name.startswith("__amd_rocclr_copyBuffer"):
                copies.append((int(r["Grid_Size"]), float(r["Counter_Value"])))
            else:
                per[name].append(float(r["Counter_Value"]))
        scale = COPY_BYTES / (max(copies)[1] * 1024.0)
        tabs[counter] = {k: (sum(v) / len(v) * 1024.0 * scale, len(v), sum(v) * 1024.0 * scale) for k, v in per.items()}
    names = sorted(tabs["FETCH_SIZE"], key=lambda k: -tabs["FETCH_SIZE"][k][2])[:top]
    out = ["| kernel | dispatches | fetch MB/dispatch | write MB/dispatch |", "|---|---:|---:|---:|"]
    for k in names:
        f = tabs["FETCH_SIZE"][k]
        w = tabs["WRITE_SIZE"].get(k, (0.0, 0, 0.0))
        out.append(f"| `{k}` | {f[1]} | {f[0] / 1e6:.3f} | {w[0] / 1e6:.3f} |")
    return "\n".join(out)


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
    if len(argv) >= 4 and argv[0] == "traffic":
        out = json.dumps(record(argv[1], argv[2], argv[3]), indent=1)
        if len(argv) > 4:
            open(argv[4], "w").write(out + "\n")
        print(out)
    elif len(argv) >= 3 and argv[0] == "kernels":
        print(per_kernel_traffic(argv[1], argv[2], int(argv[3]) if len(argv) > 3 else 20))
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
