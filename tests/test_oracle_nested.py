"""Pins of the nested iteration (oracle.asmg.ASMGPreconditioner.nested_guess) and of PCG from a
nonzero initial guess (oracle.pcg)."""
import numpy as np
import pytest
import scipy.sparse.linalg as sla

import workloads as W
from oracle import pcg
from oracle.hierarchy import Hierarchy


def _exact(p):
    return np.sin(np.pi * p[..., 0]) * np.sin(np.pi * p[..., 1])


def _load(X, T, F):
    """Consistent P1 load vector, edge-midpoint rule (exact for quadratic integrands)."""
    P = X[T]
    area = 0.5 * np.abs((P[:, 1, 0] - P[:, 0, 0]) * (P[:, 2, 1] - P[:, 0, 1])
                        - (P[:, 2, 0] - P[:, 0, 0]) * (P[:, 1, 1] - P[:, 0, 1]))
    mids = [(P[:, 0] + P[:, 1]) / 2, (P[:, 1] + P[:, 2]) / 2, (P[:, 2] + P[:, 0]) / 2]
    touch = {0: (0, 2), 1: (0, 1), 2: (1, 2)}   # midpoints of the edges through vertex a
    f = np.zeros(len(X))
    for a in range(3):
        np.add.at(f, T[:, a], sum(0.5 * F(mids[k]) for k in touch[a]) * area / 3)
    return f


def _setup(n, jitter=0.0, diagonals="random"):
    X, T, _ = W.square_mesh(n, jitter=jitter, diagonals=diagonals)
    H = Hierarchy(X, T, np.ones(len(T)))
    f = _load(X, T, lambda p: 2 * np.pi ** 2 * _exact(p))[H.dofs]
    return X, T, H, f


def test_bottom_is_finest_gives_the_discrete_solution():
    # 32^2: the finest auxiliary grid is the bottom level and carries the fine grid's vertices, so
    # the guess is Pi A_J^-1 Pi^T f = A^-1 f, and PCG stops before its first iteration
    X, T, H, f = _setup(32)
    assert H.aux.J == H.aux.lc
    uh = sla.spsolve(H.A.tocsc(), f)
    u0 = H.preconditioner().nested_guess(f, 1)
    assert np.abs(u0 - uh).max() <= 1e-12 * np.abs(uh).max()
    u, its, info = H.solve(f, 1e-8, nested=1)
    assert its == 0 and info["true_rel_residual"] <= 1e-8


def test_many_cycles_reach_the_auxiliary_solution():
    # with the V-cycles iterated to convergence on every level, e_J = A_J^-1 g_J exactly
    X, T, H, f = _setup(64, jitter=0.3)
    B = H.preconditioner()
    ref = B.Pi @ sla.spsolve(H.aux.A[H.aux.J].tocsc(), B.PiT @ f)
    u40 = B.nested_guess(f, 40)
    assert np.linalg.norm(u40 - ref) <= 1e-11 * np.linalg.norm(ref)


def test_restricted_load_vectors_are_the_level_load_vectors():
    # F = 1 on a uniform grid with every cell split the same way: every interior vertex has 6
    # triangles, so the fine load entry is h^2; on these meshes Pi is the identity at level J, and
    # P_l^T carries the load vector of level l to that of level l-1: g_l = h_l^2 with
    # h_l = 2^-(l-1), on every level down to the bottom
    X, T, _ = W.square_mesh(128, jitter=0.0, diagonals="ur")
    H = Hierarchy(X, T, np.ones(len(T)))
    f = _load(X, T, lambda p: np.ones(p.shape[:-1]))[H.dofs]
    np.testing.assert_allclose(f, 1.0 / 128 ** 2, rtol=1e-12)
    u0, g, e = H.preconditioner().nested_guess(f, 1, levels=True)
    assert H.aux.J == 8 and H.aux.lc < H.aux.J - 1
    for l in range(H.aux.lc, H.aux.J + 1):
        np.testing.assert_allclose(g[l], 4.0 ** -(l - 1), rtol=1e-12)


def test_one_cycle_per_level_is_below_the_discretisation_error():
    # full multigrid: one V-cycle per level leaves an algebraic error far below the discretisation
    # error max|u_h - u| of the smooth solution u = sin(pi x) sin(pi y); without the cycles the
    # guess only carries the coarse grid's error
    X, T, H, f = _setup(128)
    uh = sla.spsolve(H.A.tocsc(), f)
    disc = np.abs(uh - _exact(X[H.dofs])).max()
    B = H.preconditioner()
    err = {k: np.abs(B.nested_guess(f, k) - uh).max() for k in (0, 1, 2)}
    assert err[1] < 0.1 * disc
    assert err[2] < err[1]
    assert err[0] > disc


def test_nested_start_saves_iterations_and_agrees(graded_small):
    c, H = graded_small
    f = c["f_vertex"][H.dofs] if "f_vertex" in c else np.random.default_rng(3).uniform(-1, 1, H.n)
    u, its, _ = H.solve(f, 1e-10)
    u1, its1, info = H.solve(f, 1e-10, nested=1)
    assert info["status"] == "ok" and its1 <= its
    assert np.linalg.norm(u1 - u) <= 1e-8 * np.linalg.norm(u)
    um, itsm, infom = H.solve(f, 1e-10, nested=1, mixed=True)
    assert infom["true_rel_residual"] <= 1e-10


def test_pcg_from_a_guess():
    X, T, H, f = _setup(32, jitter=0.3)
    uh = sla.spsolve(H.A.tocsc(), f)
    B = H.preconditioner()
    # the exact solution as the guess: zero iterations
    u, its, info = pcg.pcg(H.A, f, B, 1e-8, u0=uh)
    assert its == 0 and np.array_equal(u, uh)
    # any guess: the same solution to the tolerance, and the rule stays relative to ||f||
    g = np.random.default_rng(4).standard_normal(H.n)
    u, its, info = pcg.pcg(H.A, f, B, 1e-10, u0=g)
    assert info["status"] == "ok"
    assert np.linalg.norm(H.A @ u - f) <= 1e-10 * np.linalg.norm(f) * (1 + 1e-6)
