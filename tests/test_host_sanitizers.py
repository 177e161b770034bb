"""The host setup (setup.cpp, domain.cpp) built with AddressSanitizer and UndefinedBehaviorSanitizer
(g++, host code only; no HIP code is part of this build) and run through the whole pipeline on a
2-D graded mesh, a 3-D cube, an L-shape with Dirichlet grids on the mesh domain, an annulus
with the mixed Dirichlet/Neumann grids and a pure Neumann annulus, each with the near-boundary
sets and their exact solvers: no sanitizer report, no leak."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads as W
from oracle.domain import boundary_vertices

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1410_2153_amd", "csrc")


def _write(path, coords, elems, kappa, domain=0, mask=None):
    with open(path, "wb") as f:
        np.array([coords.shape[1]], np.int32).tofile(f)
        np.array([len(coords), len(elems)], np.int64).tofile(f)
        np.array([domain, 0 if mask is None else 1], np.int32).tofile(f)
        np.ascontiguousarray(coords, np.float64).tofile(f)
        np.ascontiguousarray(elems, np.int32).tofile(f)
        np.ascontiguousarray(kappa, np.float64).tofile(f)
        if mask is not None:
            np.ascontiguousarray(mask, np.uint8).tofile(f)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_setup_under_sanitizers(tmp_path):
    flags = ["-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
             "-ffp-contract=off", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    here = os.path.dirname(os.path.abspath(__file__))
    srcs = [os.path.join(CSRC, "setup.cpp"), os.path.join(CSRC, "domain.cpp"), os.path.join(CSRC, "nearbnd.cpp"),
            os.path.join(here, "setup_check_main.cpp")]
    procs = [subprocess.Popen(["g++", *flags, "-c", s, "-o", str(tmp_path / (os.path.basename(s) + ".o"))])
             for s in srcs]
    assert all(p.wait() == 0 for p in procs)
    exe = str(tmp_path / "setup_check")
    subprocess.run(["g++", *flags, *[str(tmp_path / (os.path.basename(s) + ".o")) for s in srcs], "-o", exe,
                    "-lpthread"], check=True)

    cases = []
    c = W.make_config(1, scale=0.004)
    cases.append(("graded", (c["coords"], c["elems"], c["kappa"]), {}))
    c = W.make_config(2, scale=1 / 16)
    cases.append(("cube", (c["coords"], c["elems"], c["kappa"]), {}))
    X, T, _ = W.lshape_mesh(24, 0.3)
    cases.append(("lshape", (X, T, np.ones(len(T))), dict(domain=1)))
    X, T, _ = W.annulus_mesh(64)
    m = boundary_vertices(T, len(X)) & (np.hypot(X[:, 0] - 0.5, X[:, 1] - 0.5) > 0.35)
    cases.append(("annulus_mixed", (X, T, np.ones(len(T))), dict(domain=2, mask=m)))
    cases.append(("annulus_neumann", (X, T, np.ones(len(T))), dict(domain=2, mask=np.zeros(len(X), bool))))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    for name, args, kw in cases:
        path = str(tmp_path / f"{name}.bin")
        _write(path, *args, **kw)
        r = subprocess.run([exe, path], capture_output=True, text=True, env=env, timeout=600)
        assert r.returncode == 0, (name, r.stderr[-2000:])
        assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, (name, r.stderr[-2000:])
        assert r.stdout.startswith("n "), (name, r.stdout)
