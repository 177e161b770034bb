"""Batched solves (many meshes x several right-hand sides) against the oracle, system by system."""
import numpy as np
import pytest

import workloads as W
from oracle.hierarchy import Hierarchy

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
A = pytest.importorskip("paper_1410_2153_amd")


@pytest.fixture(scope="module")
def batch():
    meshes = W.batched_config(n_meshes=6, side_lo=6, side_hi=48, n_rhs=4, item=7)
    # one graded mesh too: deep, uneven hierarchy next to shallow ones
    g = W.make_config(1, scale=0.004)
    meshes.append(dict(coords=g["coords"], elems=g["elems"], kappa=g["kappa"],
                       f_vertex=np.stack([g["f_vertex"]] * 4) * np.array([[1.0], [-2.0], [0.5], [3.0]])))
    print("[gpu batch] sides", [m.get("n") for m in meshes], flush=True)
    H = [Hierarchy(m["coords"], m["elems"], m["kappa"]) for m in meshes]
    return meshes, H


def _pack(meshes, H, nr):
    return np.concatenate([m["f_vertex"][:nr, h.dofs].ravel() for m, h in zip(meshes, H)])


@pytest.mark.parametrize("nr", [1, 4])
def test_batched_fp64_matches_oracle(batch, nr):
    meshes, H = batch
    B = A.BatchSolver([(m["coords"], m["elems"], m["kappa"]) for m in meshes])
    assert list(B.n_per_mesh) == [h.n for h in H]
    F = _pack(meshes, H, nr)
    U, its, tr = B.solve(torch.from_numpy(F).cuda(), nr, 1e-8)
    U = U.cpu().numpy()
    off = B.offsets(nr)
    for m, h in enumerate(H):
        blk = U[off[m]:off[m + 1]].reshape(nr, h.n)
        for r in range(nr):
            f = meshes[m]["f_vertex"][r, h.dofs]
            uo, ito, info = h.solve(f, 1e-8, record=True)
            err = np.linalg.norm(blk[r] - uo) / np.linalg.norm(uo)
            near = any(abs(x - 1e-8) < 1e-3 * 1e-8 for x in info["history"][-2:])
            assert its[m, r] == ito or near, (m, r, its[m, r], ito)
            assert err <= 1e-10, (m, r, err)
            assert tr[m, r] <= 1e-8 * (1 + 1e-6)
    # the launch-shape autotuner ran on the first solve and picked a shape for every site
    shapes = B.tuned_shapes(nr, A.PREC_FP64)
    assert len(shapes) > 10
    assert set(shapes[:, 0].tolist()) <= {128, 256, 512} and set(shapes[:, 1].tolist()) <= {0, 1}
    assert set(shapes[:, 2].tolist()) <= {0, 1}


def test_batched_mixed(batch):
    meshes, H = batch
    B = A.BatchSolver([(m["coords"], m["elems"], m["kappa"]) for m in meshes], precision=A.PREC_MIXED)
    F = _pack(meshes, H, 4)
    U, its, tr = B.solve(torch.from_numpy(F).cuda(), 4, 1e-8)
    U = U.cpu().numpy()
    off = B.offsets(4)
    for m, h in enumerate(H):
        blk = U[off[m]:off[m + 1]].reshape(4, h.n)
        for r in range(4):
            ref = h.solve(meshes[m]["f_vertex"][r, h.dofs], 1e-12)[0]
            assert np.linalg.norm(blk[r] - ref) <= 1e-6 * np.linalg.norm(ref)
            assert tr[m, r] <= 1e-8


def test_batched_zero_rhs_systems(batch):
    meshes, H = batch
    B = A.BatchSolver([(m["coords"], m["elems"], m["kappa"]) for m in meshes])
    F = _pack(meshes, H, 2)
    off = B.offsets(2)
    F[off[1]:off[2]] = 0.0          # every system of mesh 1 has f = 0
    U, its, tr = B.solve(torch.from_numpy(F).cuda(), 2, 1e-8)
    U = U.cpu().numpy()
    assert np.all(U[off[1]:off[2]] == 0) and np.all(its[1] == 0)
    assert np.all(its[0] > 0)


def test_batched_rhs_count_switch(batch):
    # one handle solving with 4, 1, 2 and again 4 right-hand sides gives bit for bit what a fresh
    # handle gives for each count (the residual kernel leaves rows unwritten whose zeros depend
    # on the [row][NR] layout)
    meshes, H = batch
    mk = lambda: A.BatchSolver([(m["coords"], m["elems"], m["kappa"]) for m in meshes])
    B = mk()
    fresh = {}
    for nr in (4, 1, 2, 4):
        F = torch.from_numpy(_pack(meshes, H, nr)).cuda()
        U, its, tr = B.solve(F, nr, 1e-8)
        if nr not in fresh:
            fresh[nr] = mk().solve(F, nr, 1e-8)
        U0, its0, tr0 = fresh[nr]
        assert np.array_equal(its, its0), nr
        assert torch.equal(U, U0), nr
