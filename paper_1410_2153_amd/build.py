"""Build the HIP/C++ shared library libasmg.so for gfx950 (in-tree, under _lib/).

Sources: csrc/setup.cpp (host setup), csrc/domain.cpp (general-domain predicates),
csrc/api.cpp (C ABI), csrc/device.hip and csrc/batch.hip (kernels and PCG drivers),
csrc/tree.hip, csrc/assemble.hip, csrc/levels.hip and csrc/colour.hip (setup steps built on the
device, option setup_device: cluster tree, fine and level matrices, prolongations, level meshes,
hash-order colourings).
The host setup is compiled without floating-point contraction, so barycenters, box
keys and the exact orientation predicates are plain IEEE operations.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(OUT_DIR, "libasmg.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
COMMON = ["-std=c++17", "-O3", "-fPIC", "-Wall", "-Wno-unused-function", "-Wno-unused-result",
          "-I" + os.path.join(ROCM, "include")]
# packed FP32 instructions are disabled for device code (hipcc makes them from plain float code)
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = True) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    jobs = []
    for src, extra in (("setup.cpp", ["-ffp-contract=off"]), ("domain.cpp", ["-ffp-contract=off"]),
                       ("nearbnd.cpp", []), ("api.cpp", [])):
        obj = os.path.join(OUT_DIR, src.replace(".cpp", ".o"))
        jobs.append([HIPCC, "-x", "c++", *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", obj])
    # the device setup reproduces the host setup's IEEE operations: no contraction there either
    for src, extra in (("device.hip", []), ("batch.hip", []), ("tree.hip", ["-ffp-contract=off"]),
                       ("assemble.hip", ["-ffp-contract=off"]), ("colour.hip", []), ("levels.hip", []),
                       ("transfer.hip", ["-ffp-contract=off"])):
        obj = os.path.join(OUT_DIR, src.replace(".hip", ".o"))
        jobs.append([HIPCC, "-x", "hip", *COMMON, *DEVICE, *extra, "-c", os.path.join(CSRC, src), "-o", obj])
    objs = [j[-1] for j in jobs]
    # independent translation units compile in parallel (bounded by the host's cores)
    workers = max(1, min(len(jobs), len(os.sched_getaffinity(0)), 16))
    with ThreadPoolExecutor(workers) as ex:
        list(ex.map(_run, jobs))
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs, "-lpthread", "-lrocprofiler-sdk-roctx"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
