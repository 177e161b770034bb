"""Pins of the near-boundary correction (oracle.nearbnd; Section 3.5, Algorithm 3) and of the pure
Neumann problems it is meant for.

* J_{l,j} against a brute-force construction by the definition (facets counted per kept simplex,
  layers grown simplex by simplex), and Gamma_l on the root box against the box's faces;
* the correction zeroes the residual on J; the regularised exact solve is the minimum-norm
  solution (numpy's pseudo-inverse) on right-hand sides with zero sum;
* B_co with the correction is symmetric positive definite (dense, small meshes), also on a pure
  Neumann problem; the pure Neumann solve equals the pseudo-inverse solution of the projected f;
* the transfer Pi reproduces linear functions at every fine vertex on Neumann grids (boundary
  vertices included: a facet on the root box's boundary belongs to one simplex only);
* the Neumann problems converge at a level-independent rate below 1/2, and the correction does
  not slow the stationary iteration down.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import nearbnd
from oracle.hierarchy import Hierarchy


def _neumann(X, T, seed=2, sigma=0.5):
    k = np.exp(np.random.default_rng(seed).normal(0, sigma, len(T)))
    return Hierarchy(X, T, k, dirichlet=np.zeros(len(X), dtype=bool), domain="mixed")


@pytest.fixture(scope="module")
def square_neumann():
    X, T, _ = W.square_mesh(24, 0.3, cfg=0, item=1)
    return X, T, _neumann(X, T)


@pytest.fixture(scope="module")
def annulus_neumann():
    X, T, _ = W.annulus_mesh(48)
    return X, T, _neumann(X, T)


def _levels(H):
    return range(H.aux.lc + 1, H.tree.J + 1)


@pytest.mark.parametrize("case", ["square_dirichlet", "annulus_mixed", "lshape_mesh", "cube"])
@pytest.mark.parametrize("j", [0, 1, 2])
def test_near_boundary_set_matches_brute_force(case, j):
    if case == "square_dirichlet":
        X, T, _ = W.square_mesh(16, 0.3, cfg=0, item=2)
        H = Hierarchy(X, T, np.ones(len(T)))
    elif case == "annulus_mixed":
        X, T, _ = W.annulus_mesh(40)
        outer = np.hypot(X[:, 0] - 0.5, X[:, 1] - 0.5) > 0.45
        from oracle.domain import boundary_vertices
        H = Hierarchy(X, T, np.ones(len(T)), dirichlet=boundary_vertices(T, len(X)) & outer, domain="mixed")
    elif case == "lshape_mesh":
        X, T, _ = W.lshape_mesh(16, 0.3)
        H = Hierarchy(X, T, np.ones(len(T)), domain="mesh")
    else:
        X, T, _ = W.kuhn_cube_mesh(4, 0.2, cfg=2, item=4)
        H = Hierarchy(X, T, np.ones(len(T)))
    for l in _levels(H):
        lm = H.meshes.level(l)
        J = nearbnd.near_boundary_set(lm, j)
        assert J.tolist() == nearbnd.brute_force_layers(lm, j), (l, j)
        assert np.all(np.diff(J) > 0)


def test_boundary_of_the_root_box_grid():
    # On the root box every simplex of sigma^(l) is kept: Gamma_l is the box's boundary, and the
    # layers are the vertices within j + 1 cells of it (Kuhn triangles: a vertex shares a triangle
    # with each of its 8 lattice neighbours except two diagonal ones, so the layers grow by one
    # cell per step in the max-norm, up to the missing diagonal)
    X, T, _ = W.square_mesh(32, 0.0, cfg=0, item=3)
    H = Hierarchy(X, T, np.ones(len(T)))
    lm = H.meshes.level(H.tree.J)
    top = lm.verts.max()
    on = nearbnd.grid_boundary_vertices(lm)
    geo = np.any((lm.verts == 0) | (lm.verts == top), axis=1)
    assert np.array_equal(on, geo)
    J0 = nearbnd.near_boundary_set(lm, 0)
    V = lm.verts[lm.dof_vert[J0]]
    step = top // (1 << (H.tree.J - 1))
    dist = np.minimum(V, top - V).min(axis=1)
    assert dist.max() <= step and dist.min() == step      # interior unknowns of the first cell ring
    allv = lm.verts[lm.dof_vert]
    ring = np.minimum(allv, top - allv).min(axis=1) == step
    assert set(np.nonzero(ring)[0]) <= set(J0.tolist())


def test_correction_zeroes_the_residual_on_J(annulus_neumann):
    X, T, H = annulus_neumann
    rng = np.random.default_rng(1)
    for l in _levels(H):
        J = nearbnd.near_boundary_set(H.meshes.level(l), 2)
        A = H.aux.A[l]
        nb = nearbnd.NearBoundary(A, J)
        g = rng.standard_normal(A.shape[0])
        e = rng.standard_normal(A.shape[0])
        Jc = np.setdiff1d(np.arange(A.shape[0]), J)
        e0 = e.copy()
        nb.correct(e, g)
        r = g - A @ e
        if len(J) == A.shape[0]:
            # the whole level (singular, regularised): the residual is left in the constants
            assert abs(r.sum() - g.sum()) <= 1e-10 * np.abs(g).sum()
            r = r - r.mean()
        assert np.abs(r[J]).max() <= 1e-9 * np.abs(g).max(), l
        assert np.array_equal(e[Jc], e0[Jc])


def test_regularised_solve_is_the_minimum_norm_solution(annulus_neumann):
    X, T, H = annulus_neumann
    A = H.aux.A[H.aux.lc]
    assert np.abs(np.asarray(A.sum(axis=1))).max() <= 1e-12 * A.diagonal().max()   # singular
    b = np.random.default_rng(3).standard_normal(A.shape[0])
    b -= b.mean()
    x = nearbnd.ExactSolve(A)(b)
    ref = np.linalg.pinv(A.toarray()) @ b
    assert np.abs(x - ref).max() <= 1e-9 * np.abs(ref).max()
    # two components, one singular and one not: each is solved on its own
    B = sp.block_diag([A, A + sp.eye(A.shape[0])]).tocsr()
    b2 = np.concatenate([b, np.random.default_rng(4).standard_normal(A.shape[0])])
    x2 = nearbnd.ExactSolve(B)(b2)
    assert np.abs(x2[:len(b)] - ref).max() <= 1e-9 * np.abs(ref).max()
    y = np.linalg.solve((A + sp.eye(A.shape[0])).toarray(), b2[len(b):])
    assert np.abs(x2[len(b):] - y).max() <= 1e-10 * np.abs(y).max()


@pytest.mark.parametrize("case", ["dirichlet", "neumann"])
def test_bco_with_correction_is_spd(case):
    X, T, _ = W.square_mesh(12, 0.3, cfg=0, item=5)
    k = np.exp(np.random.default_rng(6).normal(0, 0.5, len(T)))
    # a small bottom level, so that there are levels above it to correct on
    if case == "dirichlet":
        H = Hierarchy(X, T, k, coarse_max_dofs=16)
    else:
        H = Hierarchy(X, T, k, dirichlet=np.zeros(len(X), dtype=bool), domain="mixed", coarse_max_dofs=16)
    B = H.preconditioner(nb_layers=1)
    assert B.nb, "no level with a near-boundary set"
    M = np.column_stack([B(e) for e in np.eye(H.n)])
    assert np.abs(M - M.T).max() <= 1e-12 * np.abs(M).max()
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0


@pytest.mark.parametrize("nb", [0, 2])
def test_pure_neumann_solve_is_the_pseudo_inverse_solution(square_neumann, nb):
    X, T, H = square_neumann
    assert H.pure_neumann and H.n == len(X)
    f = np.random.default_rng(7).standard_normal(H.n)
    u, it, info = H.solve(f, 1e-12, nb_layers=nb)
    assert info["status"] == "ok"
    ref = np.linalg.pinv(H.A.toarray()) @ (f - f.mean())
    assert abs(u.mean()) <= 1e-14 * np.abs(u).max()
    assert np.linalg.norm(u - ref) <= 1e-9 * np.linalg.norm(ref)


@pytest.mark.parametrize("mesh", ["square", "annulus"])
def test_transfer_reproduces_linear_functions_on_neumann_grids(mesh):
    if mesh == "square":
        X, T, _ = W.square_mesh(24, 0.3, cfg=0, item=6)
    else:
        X, T, _ = W.annulus_mesh(48)
    H = _neumann(X, T)
    lm = H.meshes.level(H.tree.J)
    unit = H.tree.L * 2.0 ** (-H.tree.J)
    Y = H.tree.a + lm.verts[lm.dof_vert] * unit
    d = X.shape[1]
    lin = lambda Z: 0.7 + Z @ np.array([1.3, -2.1, 0.4][:d])
    np.testing.assert_allclose(H.Pi @ lin(Y), lin(X[H.dofs]), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(H.Pi @ np.ones(H.Pi.shape[1]), 1.0, atol=1e-13)


def _seminorm_rate(H, nb, its=14):
    # contraction of e <- (I - B_co A) e in the A-(semi)norm (constants are invisible to it)
    B, A = H.preconditioner(nb_layers=nb), H.A
    e = np.random.default_rng(0).standard_normal(H.n)
    norm = lambda v: float(np.sqrt(max(v @ (A @ v), 0.0)))
    ns = [norm(e)]
    for _ in range(its):
        e = e - B(A @ e)
        ns.append(norm(e))
    return (ns[-1] / ns[4]) ** (1.0 / (its - 4))


def test_neumann_rates_are_small_level_independent_and_not_slowed_by_the_correction():
    hs = [_neumann(*W.square_mesh(n, 0.3, cfg=0, item=7)[:2]) for n in (32, 64)]
    r0 = [_seminorm_rate(H, 0) for H in hs]
    r2 = [_seminorm_rate(H, 2) for H in hs]
    assert all(r < 0.5 for r in r0 + r2), (r0, r2)
    assert r0[1] <= r0[0] + 0.1, r0
    assert all(b <= a + 0.01 for a, b in zip(r0, r2)), (r0, r2)
