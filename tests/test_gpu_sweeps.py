"""Gauss-Seidel sweep counts other than the defaults (two auxiliary sweeps, one fine sweep per
side of Algorithms 1 and 2): B_co and PCG through the C ABI against the oracle run with the same
counts, on the single-mesh and the batched engines.

After a single forward sweep from zero a level's residual kernel adds only each row's later
colours' terms (the fine level by default; the auxiliary levels with one sweep); after two or more
sweeps, with local smoothing and on levels with a near-boundary set it computes b - A x in full.
The cases run both forms on every kind of level.

Bars as in the other parity tests: B_co element-wise within 1e-12 (FP64) and 1e-5 (FP32 V-cycle)
of the oracle's; FP64 solves take the oracle's iteration count and agree element-wise to 1e-10.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle.hierarchy import Hierarchy

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
A = pytest.importorskip("paper_1410_2153_amd")

SWEEPS = [(1, 1), (1, 2), (3, 1), (2, 3)]   # (nu_aux, nu_fine)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel_inf(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _annulus_neumann_hole():
    from oracle.domain import boundary_vertices
    X, T, _ = W.annulus_mesh(200)
    dm = boundary_vertices(T, len(X)) & (np.hypot(X[:, 0] - 0.5, X[:, 1] - 0.5) > 0.35)
    return dict(coords=X, elems=T, kappa=np.exp(np.random.default_rng(2).normal(0, 0.5, len(T))), dirichlet=dm,
                f_vertex=W.rhs_per_vertex(len(X), 5, 1))


# name -> (workload, solver options; the oracle takes the same colouring, smoothing, domain, layers)
CASES = {
    "graded20k": (lambda: W.make_config(1, scale=0.01), dict(colouring=2)),
    "cube16": (lambda: W.make_config(2, scale=1 / 8), dict(colouring=2)),
    "graded20k_local": (lambda: W.make_config(1, scale=0.01), dict(colouring=2, smoothing=1)),
    "annulus_mixed_nb2": (_annulus_neumann_hole, dict(colouring=2, domain=2, nb_layers=2)),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    _say(f"[gpu sweeps] case {request.param}")
    make, kw = CASES[request.param]
    c = make()
    dm = c.get("dirichlet")
    H = Hierarchy(c["coords"], c["elems"], c["kappa"], dirichlet=dm,
                  colouring={0: "natural", 2: "smallest_last"}[kw.get("colouring", 0)],
                  domain=["box", "mesh", "mixed"][kw.get("domain", 0)])
    okw = dict(smoothing=["full", "local"][kw.get("smoothing", 0)], nb_layers=kw.get("nb_layers", 0))
    return request.param, c, dm, kw, H, okw, c["f_vertex"][H.dofs]


@pytest.mark.parametrize("nu", SWEEPS, ids=[f"aux{a}_fine{b}" for a, b in SWEEPS])
def test_preconditioner_and_solve(case, nu):
    name, c, dm, kw, H, okw, f = case
    nu_aux, nu_fine = nu
    S = A.Solver(c["coords"], c["elems"], c["kappa"], dm, nu_aux=nu_aux, nu_fine=nu_fine, **kw)
    r = np.random.default_rng(5).standard_normal(H.n)
    zo = H.preconditioner(nu_aux=nu_aux, nu_fine=nu_fine, **okw)(r)
    rd = torch.from_numpy(r).cuda()
    z64 = S.apply_preconditioner(rd).cpu().numpy()
    z32 = S.apply_preconditioner(rd, precision=A.PREC_MIXED).cpu().numpy()
    _say(name, nu, f"B_co fp64 {_rel_inf(z64, zo):.2e}, fp32 {_rel_inf(z32, zo):.2e}")
    assert _rel_inf(z64, zo) <= 1e-12
    assert _rel_inf(z32, zo) <= 1e-5
    uo, ito, info = H.solve(f, 1e-8, record=True, nu_aux=nu_aux, nu_fine=nu_fine, **okw)
    u, it, tr = S.solve(f, 1e-8)
    near = any(abs(h - 1e-8) < 1e-3 * 1e-8 for h in info["history"][-2:])
    _say(name, nu, f"iterations gpu {it} oracle {ito}, element-wise {_rel_inf(u, uo):.2e}")
    assert it == ito or near
    assert tr <= 1e-8 * (1 + 1e-6)
    assert _rel_inf(u, uo) <= 1e-10
    S.close()


@pytest.mark.parametrize("nu", SWEEPS, ids=[f"aux{a}_fine{b}" for a, b in SWEEPS])
def test_batched(nu):
    nu_aux, nu_fine = nu
    meshes = W.batched_config(n_meshes=4, side_lo=8, side_hi=40, n_rhs=2, item=11)
    H = [Hierarchy(m["coords"], m["elems"], m["kappa"]) for m in meshes]
    B = A.BatchSolver([(m["coords"], m["elems"], m["kappa"]) for m in meshes], nu_aux=nu_aux, nu_fine=nu_fine)
    F = np.concatenate([m["f_vertex"][:2, h.dofs].ravel() for m, h in zip(meshes, H)])
    U, its, tr = B.solve(torch.from_numpy(F).cuda(), 2, 1e-8)
    U = U.cpu().numpy()
    off = B.offsets(2)
    for m, h in enumerate(H):
        blk = U[off[m]:off[m + 1]].reshape(2, h.n)
        for q in range(2):
            uo, ito, info = h.solve(meshes[m]["f_vertex"][q, h.dofs], 1e-8, record=True, nu_aux=nu_aux,
                                    nu_fine=nu_fine)
            near = any(abs(x - 1e-8) < 1e-3 * 1e-8 for x in info["history"][-2:])
            _say(f"batched {nu} mesh {m} rhs {q}: iterations {its[m, q]} oracle {ito}, "
                 f"element-wise {_rel_inf(blk[q], uo):.2e}")
            assert its[m, q] == ito or near
            assert _rel_inf(blk[q], uo) <= 1e-10
            assert tr[m, q] <= 1e-8 * (1 + 1e-6)
    B.close()
