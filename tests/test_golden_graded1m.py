"""Full-size parity on the graded 2-D mesh (about 1.0 M unknowns) against stored oracle values.

The expected values in ``tests/golden/graded1m.npz`` were written by
``tests/golden/make_graded1m.py``, which calls only the oracle and the input generators.
At this size the oracle's setup takes about half an hour, so the values are stored:
  * the hierarchy's index maps, bit-exact (SHA-256 of canonical int64 forms): keys,
    refined set, leaves, level sizes, level vertices/simplices/unknowns, patterns of A,
    A_l, P_l and Pi, colourings (CPU test, host-only handle; the device solves use the
    same host setup);
  * one FP64 B_co application (Algorithm 1) at 4096 seeded unknowns:
    |z_gpu - z| <= 1e-12 |z|_inf element by element;
  * the FP64 PCG solve to 1e-8: the same iteration count and |u_gpu - u| <= 1e-10 |u|_inf
    element by element on the samples;
  * the mixed-precision solve (FP32 B_co inside FP64 CG) to 1e-8: within 1e-6 |u|_inf of the
    oracle's solve to 1e-12.
Each GPU case runs in the launch configuration bench.py uses (default reduction grid,
autotuned launch shapes), so the kernels' full-size paths (grid-stride loops, every slice
width) are the ones compared.
"""
import importlib.util
import json
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "graded1m.npz")

A = pytest.importorskip("paper_1410_2153_amd")

pytestmark = [pytest.mark.slow,
              pytest.mark.skipif(not os.path.exists(GOLDEN), reason="stored oracle values not written")]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _golden_script():
    spec = importlib.util.spec_from_file_location("make_graded1m", os.path.join(HERE, "golden", "make_graded1m.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def library_digests(S):
    """The library's exports in the canonical forms of the stored digests."""
    G = _golden_script()
    cat = np.concatenate
    out = {"keys": G.digest(S.export("keys")), "refined": G.digest(S.export("refined")),
           "leaves": G.digest(S.export("leaves")), "level_n": G.digest(S.export("level_n")),
           "A_pattern": G.digest(cat([S.export("A_rowptr"), S.export("A_col")])),
           "Pi_pattern": G.digest(cat([S.export("Pi_rowptr"), S.export("Pi_col")])),
           "colour_fine": G.digest(S.export("colour_fine"))}
    info = S.info()
    for l in range(info["lc"], info["J"] + 1):
        out[f"level_verts_{l}"] = G.digest(S.export("level_verts", l))
        out[f"level_simp_{l}"] = G.digest(S.export("level_simp", l))
        out[f"level_dofs_{l}"] = G.digest(S.export("level_dofs", l))
        out[f"Al_pattern_{l}"] = G.digest(cat([S.export("Al_rowptr", l), S.export("Al_col", l)]))
    for l in range(info["lc"] + 1, info["J"] + 1):
        out[f"P_pattern_{l}"] = G.digest(cat([S.export("P_rowptr", l), S.export("P_col", l)]))
        out[f"colour_aux_{l}"] = G.digest(S.export("colour_aux", l))
    return out


@pytest.fixture(scope="module")
def golden():
    z = np.load(GOLDEN)
    g = {k: z[k] for k in z.files}
    g["digests"] = json.loads(str(g["hierarchy_digests"]))
    return g


@pytest.fixture(scope="module")
def mesh(golden):
    import bench
    _say("[golden graded1m] loading the graded mesh")
    c = bench.load_workload(float(golden["scale"]))
    return c


def test_digest_forms_agree_on_a_small_mesh():
    # the canonical forms of the stored digests, computed from the oracle and from the library's
    # exports, agree on a small mesh of the same family (so a full-size mismatch is a real one)
    import workloads as W
    from oracle.hierarchy import Hierarchy
    c = W.make_config(1, scale=0.004)
    H = Hierarchy(c["coords"], c["elems"], c["kappa"])
    S = A.Solver(c["coords"], c["elems"], c["kappa"], device=-1)
    assert _golden_script().hierarchy_digests(H) == library_digests(S)


def test_hierarchy_bit_exact_at_full_size(golden, mesh):
    S = A.Solver(mesh["coords"], mesh["elems"], mesh["kappa"], device=-1)
    info = S.info()
    assert (S.n, info["J"], info["lc"]) == (int(golden["n"]), int(golden["J"]), int(golden["lc"]))
    lib = library_digests(S)
    bad = sorted(k for k, v in golden["digests"].items() if lib.get(k) != v)
    assert not bad, bad
    assert set(lib) == set(golden["digests"])


@pytest.fixture(scope="module")
def gpu_solver(golden, mesh):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    S = A.Solver(mesh["coords"], mesh["elems"], mesh["kappa"])
    f = np.ascontiguousarray(mesh["f_vertex"][S.dof_vertex()])
    _say(f"[golden graded1m] device handle: {S.n} unknowns")
    return S, torch.from_numpy(f).cuda()


@pytest.mark.gpu
def test_preconditioner_fp64_elementwise(golden, gpu_solver):
    S, fd = gpu_solver
    idx = golden["idx"]
    z = S.apply_preconditioner(fd, A.PREC_FP64).cpu().numpy()
    err = np.abs(z[idx] - golden["z"]).max() / float(golden["z_inf"])
    _say(f"[golden graded1m] B_co f: max |dz| / |z|_inf = {err:.3e} on {len(idx)} unknowns")
    assert err <= 1e-12
    assert abs(np.abs(z).max() - float(golden["z_inf"])) <= 1e-12 * float(golden["z_inf"])


@pytest.mark.gpu
def test_solve_fp64_elementwise(golden, gpu_solver):
    S, fd = gpu_solver
    idx = golden["idx"]
    S.set_precision(A.PREC_FP64)
    u, it, tr = S.solve_device(fd, 1e-8)
    u = u.cpu().numpy()
    err = np.abs(u[idx] - golden["u"]).max() / float(golden["u_inf"])
    _say(f"[golden graded1m] FP64 solve: {it} iterations (oracle {int(golden['iters'])}), "
         f"max |du| / |u|_inf = {err:.3e}, true residual {tr:.3e}")
    assert it == int(golden["iters"])
    assert err <= 1e-10
    assert tr <= 1e-8 * (1 + 1e-6)


@pytest.mark.gpu
def test_solve_mixed_elementwise(golden, gpu_solver):
    S, fd = gpu_solver
    idx = golden["idx"]
    S.set_precision(A.PREC_MIXED)
    try:
        u, it, tr = S.solve_device(fd, 1e-8)
    finally:
        S.set_precision(A.PREC_FP64)
    u = u.cpu().numpy()
    err = np.abs(u[idx] - golden["u12"]).max() / float(golden["u12_inf"])
    _say(f"[golden graded1m] mixed solve: {it} iterations, max |u - u(1e-12)| / |u|_inf = {err:.3e}")
    assert err <= 1e-6
    assert tr <= 1e-8 * (1 + 1e-6)
