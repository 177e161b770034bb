"""The full-size batched workload on the GPU (256 jittered squares, sides ~ U{32..512}, 4
right-hand sides each, every system to 1e-8), in the launch configuration bench.py times.

The oracle cannot solve 1024 systems of up to 263k unknowns. Checked here:
* every system's true residual, recomputed with the oracle's own FP64 assembly of its mesh's A,
  is <= 1e-8 (FP64 and mixed), and agrees with the residual the library reports;
* on the smallest meshes the batched solution equals the oracle's PCG solution element-wise
  (1e-10) with the same iteration count;
* on a sample (smallest, median and largest mesh) the batched engine equals the single-mesh
  engine element-wise: the same algorithm in a different data layout (interleaved right-hand
  sides, merged levels), differing only in the order of reduction sums.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import fem
from oracle.hierarchy import Hierarchy

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
torch = pytest.importorskip("torch")
A = pytest.importorskip("paper_1410_2153_amd")

NR = 4
TOL = 1e-8


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def full():
    _say("[batched full size] generating 256 meshes")
    ms = W.batched_config()
    B = A.BatchSolver([(m["coords"], m["elems"], m["kappa"]) for m in ms], precision=A.PREC_FP64)
    dofs = [fem.dof_vertices(W.boundary_vertices(m["coords"])) for m in ms]
    F = np.concatenate([m["f_vertex"][:NR, d].ravel() for m, d in zip(ms, dofs)])
    assert list(B.n_per_mesh) == [len(d) for d in dofs]
    _say(f"[batched full size] {B.n_total} unknowns per right-hand side")
    Fd = torch.from_numpy(F).cuda()
    out = {}
    for name, prec in (("fp64", A.PREC_FP64), ("mixed", A.PREC_MIXED)):
        B.set_precision(prec)
        B.solve(Fd, NR, TOL)                        # first solve: autotuning
        U, its, tr = B.solve(Fd, NR, TOL)           # the configuration bench.py times
        out[name] = (U.cpu().numpy(), its.copy(), tr.copy())
        _say(f"[batched full size] {name}: iterations {its.min()}..{its.max()}")
    return ms, dofs, B, F, out


def _block(B, U, m, n):
    off = B.offsets(NR)
    return U[off[m]:off[m + 1]].reshape(NR, n)


def test_true_residual_of_every_system(full):
    ms, dofs, B, F, out = full
    worst = {p: 0.0 for p in out}
    for m, mesh in enumerate(ms):
        Am, dm = fem.assemble(mesh["coords"], mesh["elems"], mesh["kappa"])
        assert np.array_equal(dm, dofs[m])
        for prec, (U, its, tr) in out.items():
            u = _block(B, U, m, len(dm))
            for r in range(NR):
                f = mesh["f_vertex"][r, dm]
                res = np.linalg.norm(f - Am @ u[r]) / np.linalg.norm(f)
                worst[prec] = max(worst[prec], res)
                assert res <= TOL * (1 + 1e-6), (prec, m, r, res)
                assert abs(res - tr[m, r]) <= 1e-3 * tr[m, r] + 1e-15, (prec, m, r, res, tr[m, r])
    for prec, (U, its, tr) in out.items():
        _say(f"{prec}: worst true residual over {len(ms) * NR} systems {worst[prec]:.3e}, "
             f"iterations <= {its.max()}")
        assert its.max() <= 30


def test_smallest_meshes_match_the_oracle(full):
    ms, dofs, B, F, out = full
    U, its, tr = out["fp64"]
    for m in np.argsort([len(d) for d in dofs])[:3]:
        mesh = ms[m]
        H = Hierarchy(mesh["coords"], mesh["elems"], mesh["kappa"])
        u = _block(B, U, m, H.n)
        for r in range(NR):
            uo, ito, info = H.solve(mesh["f_vertex"][r, H.dofs], TOL, record=True)
            near = any(abs(h - TOL) < 1e-3 * TOL for h in info["history"][-2:])
            err = np.abs(u[r] - uo).max() / np.abs(uo).max()
            _say(f"mesh {m} (side {mesh['n']}) rhs {r}: iterations {its[m, r]} oracle {ito}, element-wise {err:.2e}")
            assert its[m, r] == ito or near
            assert err <= 1e-10


def test_sample_matches_the_single_mesh_engine(full):
    ms, dofs, B, F, out = full
    U, its, tr = out["fp64"]
    order = np.argsort([len(d) for d in dofs])
    for m in (order[0], order[len(order) // 2], order[-1]):
        mesh = ms[m]
        S = A.Solver(mesh["coords"], mesh["elems"], mesh["kappa"])
        u = _block(B, U, m, S.n)
        for r in range(NR):
            f = np.ascontiguousarray(mesh["f_vertex"][r, dofs[m]])
            us, its_s, _ = S.solve(f, TOL)
            err = np.abs(u[r] - us).max() / np.abs(us).max()
            _say(f"mesh {m} (side {mesh['n']}) rhs {r}: batched {its[m, r]} single {its_s} iterations, "
                 f"element-wise {err:.2e}")
            assert its[m, r] == its_s
            assert err <= 1e-12
        S.close()
