"""The C-ABI library loads, exports every function include/asmg.h declares, and rejects bad input (CPU only)."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
A = pytest.importorskip("paper_1410_2153_amd")


def _declared():
    hdr = open(os.path.join(ROOT, "include", "asmg.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*\**(asmg_\w+)\s*\(", hdr, re.M)))


def test_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 14
    lib = ctypes.CDLL(A.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(A.EXPORTED)


def test_rejects_invalid_input():
    coords, elems, _ = W.square_mesh(6, 0.2)
    k = np.ones(len(elems))
    with pytest.raises(A.AsmgError) as e:
        A.Solver(coords, elems, -k, device=-1)
    assert e.value.code == A.EINVAL
    bad = elems.copy()
    bad[3, 1] = 10 ** 6
    with pytest.raises(A.AsmgError):
        A.Solver(coords, bad, k, device=-1)
    deg = elems.copy()
    deg[0] = [0, 0, 1]
    with pytest.raises(A.AsmgError) as e:
        A.Solver(coords, deg, k, device=-1)
    assert e.value.code == A.EINVAL
    with pytest.raises(A.AsmgError):
        A.Solver(coords, elems, k, device=-1, nu_aux=0)
    with pytest.raises(A.AsmgError) as e:
        A.Solver(coords, elems, k, device=-1, smoothing=2)
    assert e.value.code == A.EINVAL
    with pytest.raises(A.AsmgError) as e:
        A.Solver(coords, elems, k, device=-1, domain=3)
    assert e.value.code == A.EINVAL
    for bad_nested in (-1, 17):
        with pytest.raises(A.AsmgError) as e:
            A.Solver(coords, elems, k, device=-1, nested=bad_nested)
        assert e.value.code == A.EINVAL
    with pytest.raises(A.AsmgError) as e:   # the nested iteration needs whole-level smoothing
        A.Solver(coords, elems, k, device=-1, nested=1, smoothing=1)
    assert e.value.code == A.EINVAL
    A.Solver(coords, elems, k, device=-1, nested=2)
    for bad in (dict(setup_device=1), dict(setup_device=2, device=0)):   # the device tree needs a device
        with pytest.raises(A.AsmgError) as e:
            A.Solver(coords, elems, k, **{"device": -1, **bad})
        assert e.value.code == A.EINVAL
    c3, e3, _ = W.kuhn_cube_mesh(3, 0.0)
    with pytest.raises(A.AsmgError) as e:   # general domains are 2-D
        A.Solver(c3, e3, np.ones(len(e3)), device=-1, domain=1)
    assert e.value.code == A.EINVAL
    with pytest.raises(A.AsmgError) as e:   # so are the mixed grids
        A.Solver(c3, e3, np.ones(len(e3)), device=-1, domain=2)
    assert e.value.code == A.EINVAL


def test_host_only_handle_refuses_device_calls():
    coords, elems, _ = W.square_mesh(6, 0.2)
    S = A.Solver(coords, elems, np.ones(len(elems)), device=-1)
    with pytest.raises(A.AsmgError) as e:
        S.solve(np.ones(S.n))
    assert e.value.code == A.EDEVICE
    with pytest.raises(A.AsmgError) as e:
        S.export("nonsense")
    assert e.value.code == A.EINVAL
    with pytest.raises(A.AsmgError):
        S.export("level_verts", level=99)


def test_update_coefficient_host_only():
    from oracle import fem
    coords, elems, _ = W.square_mesh(10, 0.2)
    S = A.Solver(coords, elems, np.ones(len(elems)), device=-1)
    k2 = np.random.default_rng(0).uniform(0.5, 2.0, len(elems))
    S.update_coefficient(k2)
    ref, _ = fem.assemble(coords, elems, k2)
    got = S.export_csr("A", shape=ref.shape)
    assert abs(got - ref).max() <= 1e-13 * abs(ref).max()
    with pytest.raises(A.AsmgError):
        S.update_coefficient(np.zeros(len(elems)))


def test_batch_setup_host_only():
    meshes = W.batched_config(n_meshes=5, side_lo=4, side_hi=20, n_rhs=1, item=3)
    B = A.BatchSolver([(m["coords"], m["elems"], m["kappa"]) for m in meshes], device=-1)
    for m, nm in zip(meshes, B.n_per_mesh):
        S = A.Solver(m["coords"], m["elems"], m["kappa"], device=-1)
        assert S.n == nm
    with pytest.raises(A.AsmgError) as e:
        A.lib.asmg_solve(B.h, None, 1e-8, None, None, None)
        A._check(A.lib.asmg_solve(B.h, None, 1e-8, None, None, None))
    bad = [(m["coords"], m["elems"], -m["kappa"]) for m in meshes]
    with pytest.raises(A.AsmgError):
        A.BatchSolver(bad, device=-1)
    # local smoothing is a single-mesh option
    with pytest.raises(A.AsmgError) as e:
        A.BatchSolver([(m["coords"], m["elems"], m["kappa"]) for m in meshes], device=-1, smoothing=1)
    assert e.value.code == A.EINVAL
    with pytest.raises(A.AsmgError) as e:   # so is the nested iteration
        A.BatchSolver([(m["coords"], m["elems"], m["kappa"]) for m in meshes], device=-1, nested=1)
    assert e.value.code == A.EINVAL


def test_binding_rejects_wrong_sizes():
    coords, elems, _ = W.square_mesh(6, 0.2)
    S = A.Solver(coords, elems, np.ones(len(elems)), device=-1)
    with pytest.raises(ValueError):
        S.solve(np.ones(S.n + 3))
    with pytest.raises(ValueError):
        S.update_coefficient(np.ones(len(elems) - 1))
    with pytest.raises(ValueError):
        A.Solver(coords, elems, np.ones(len(elems) + 1), device=-1)
    with pytest.raises(ValueError):
        A.Solver(coords, elems, np.ones(len(elems)), np.zeros(3, dtype=bool), device=-1)


def test_python_shape_list_matches_the_library():
    # the binding's list of autotuner candidates (used to label the tuning table) is the library's
    import os
    import re
    src = open(os.path.join(os.path.dirname(A.__file__), "csrc", "common.hpp")).read()
    body = re.search(r"kShapes\[\] = \{(.*?)\};", src, re.S).group(1)
    triples = [tuple(int(v) for v in t) for t in re.findall(r"\{(\d+),\s*(\d+),\s*(\d+)\}", body)]
    assert triples == [tuple(t) for t in A.SHAPES]
