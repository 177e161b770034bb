"""Pins of the PCG solve (oracle.pcg, oracle.hierarchy; Section 5.2) and the adjoint (oracle.adjoint)."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as sla

import workloads as W
from oracle import adjoint, fem
from oracle.hierarchy import Hierarchy


def test_matches_dense_solve(graded_small):
    c, H = graded_small
    f = c["f_vertex"][H.dofs]
    u, it, info = H.solve(f, tol=1e-13)
    ref = np.linalg.solve(H.A.toarray(), f)
    assert np.linalg.norm(u - ref) <= 1e-10 * np.linalg.norm(ref)
    assert info["true_rel_residual"] <= 1e-12


def test_zero_rhs():
    coords, elems, _ = W.square_mesh(8, 0.3, cfg=0, item=2)
    H = Hierarchy(coords, elems, np.ones(len(elems)))
    u, it, info = H.solve(np.zeros(H.n))
    assert it == 0 and np.all(u == 0)


def test_p1_reproduction_through_solver():
    coords, elems, _ = W.square_mesh(32, 0.3, cfg=0, item=4)
    H = Hierarchy(coords, elems, np.ones(len(elems)))
    A_full = fem.assemble_full(coords, elems, np.ones(len(elems)))
    bnd = fem.default_dirichlet(coords)
    g = 0.25 + 1.5 * coords[:, 0] - 0.5 * coords[:, 1]
    B = np.nonzero(bnd)[0]
    f = -(A_full[H.dofs][:, B] @ g[B])
    u, it, _ = H.solve(f, tol=1e-13)
    np.testing.assert_allclose(u, g[H.dofs], atol=1e-10)


def test_iterations_grow_logarithmically():
    its = {}
    for n in (8, 16, 32, 64, 128):
        coords, elems, _ = W.square_mesh(n, 0.3, cfg=0, item=n)
        H = Hierarchy(coords, elems, np.ones(len(elems)))
        f = W.rhs_per_vertex(len(coords), 0, n)[H.dofs]
        its[n] = H.solve(f, 1e-8)[1]
    # kappa(BA) <~ log N: no power-law growth; a + b log N with a small b
    assert its[128] <= its[16] + 3
    assert max(its.values()) <= 14


def test_mixed_precision_accuracy(graded_small):
    c, H = graded_small
    f = c["f_vertex"][H.dofs]
    ref = sla.spsolve(H.A.tocsc(), f)
    u, it, info = H.solve(f, 1e-8, mixed=True)
    u64, it64, _ = H.solve(f, 1e-8)
    assert info["true_rel_residual"] <= 1e-8
    assert abs(it - it64) <= 1
    assert np.linalg.norm(u - ref) <= 1e-6 * np.linalg.norm(ref)


def test_adjoint_gradient_finite_differences():
    coords, elems, _ = W.square_mesh(12, 0.3, cfg=4, item=7)
    rng = np.random.default_rng(5)
    m = rng.normal(0, 0.3, len(elems))
    dofs = fem.dof_vertices(fem.default_dirichlet(coords))
    f = rng.uniform(-1, 1, len(dofs))
    u_obs = rng.normal(0, 0.01, len(dofs))
    J0, g, _ = adjoint.loss_and_gradient(coords, elems, m, f, u_obs)
    for _ in range(5):
        d = rng.standard_normal(len(elems))
        eps = 1e-6
        Jp = adjoint.loss_and_gradient(coords, elems, m + eps * d, f, u_obs)[0]
        Jm = adjoint.loss_and_gradient(coords, elems, m - eps * d, f, u_obs)[0]
        fd = (Jp - Jm) / (2 * eps)
        assert fd == pytest.approx(g @ d, rel=1e-6, abs=1e-12)


_HIER = {}  # (cfg, scale) -> (workload, hierarchy), shared by the precision cases below


@pytest.mark.parametrize("cfg,scale", [(0, 1.0), (1, 0.01)])
@pytest.mark.parametrize("mixed", [False, True])
def test_restart_from_true_residual_at_the_fp64_floor(cfg, scale, mixed):
    # Below the FP64 floor of the true residual (about 1.5e-15 relative here) the recursively
    # updated residual still meets tol = 1e-15 while f - A u cannot: CG restarts from the true
    # residual at most 3 times, then returns "ok" with the true residual above tol.
    if (cfg, scale) not in _HIER:
        c = W.make_config(cfg, scale=scale)
        _HIER[(cfg, scale)] = (c, Hierarchy(c["coords"], c["elems"], c["kappa"]))
    c, H = _HIER[(cfg, scale)]
    f = c["f_vertex"][H.dofs]
    u, it, info = H.solve(f, 1e-15, mixed=mixed, record=True)
    assert info["status"] == "ok" and info["restarts"] == 3
    assert info["true_rel_residual"] > 1e-15
    # each restart takes at least one product with A
    first = next(k for k, h in enumerate(info["history"]) if h <= 1e-15) + 1
    assert it >= first + 3
    # the iterate is still the solution to the floor: the error is far below the 1e-8 solve's
    ref = np.linalg.solve(H.A.toarray(), f) if H.n <= 5000 else None
    if ref is not None:
        assert np.linalg.norm(u - ref) <= 1e-12 * np.linalg.norm(ref)


def test_restart_with_the_iteration_budget_spent_is_noconv():
    # converged on the updated residual exactly at max_iter with the true residual above tol:
    # the restart cannot take a step, so the solve ends unconverged
    c = W.make_config(0)
    H = Hierarchy(c["coords"], c["elems"], c["kappa"])
    f = c["f_vertex"][H.dofs]
    _, _, info = H.solve(f, 1e-15, record=True)
    first = next(k for k, h in enumerate(info["history"]) if h <= 1e-15) + 1
    u, it, info2 = H.solve(f, 1e-15, max_iter=first)
    assert info2["status"] == "noconv" and it == first
