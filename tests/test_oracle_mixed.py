"""Pins of the mixed Dirichlet/Neumann auxiliary grids (oracle.domain.Domain.mixed; the remark of
Section 3.5): T^M_l keeps the simplices of sigma^(l) that meet the domain and not its Dirichlet
boundary Gamma_D; the vertices of simplices meeting Gamma_D carry essential conditions."""
import numpy as np
import pytest

import workloads as W
from oracle.domain import boundary_vertices
from oracle.hierarchy import Hierarchy


@pytest.fixture(scope="module")
def left_dirichlet():
    # uniform 64^2 square, Dirichlet only on x = 0 (Neumann on the three other sides); a bottom
    # level of at most 256 unknowns keeps three auxiliary levels (l = 5, 6, 7) under test
    X, T, _ = W.square_mesh(64, jitter=0.0)
    return X, T, Hierarchy(X, T, np.ones(len(T)), dirichlet=X[:, 0] == 0.0, domain="mixed", coarse_max_dofs=256)


def test_closed_form_counts_on_the_square(left_dirichlet):
    # Omega is the root box, so every simplex meets it; the simplices that meet Gamma_D = {x = 0}
    # are the 2n of the first column of cells (every triangle of a cell has a vertex on its left
    # side). Their vertices (x = 0 and x = h) are Dirichlet; every other vertex, on the Neumann
    # sides too, is an unknown: (n - 1)(n + 1) on a level with n = 2^(l-1) cells per side
    X, T, H = left_dirichlet
    assert H.aux.J - H.aux.lc >= 2
    for l in range(H.aux.lc, H.aux.J + 1):
        lm = H.meshes.level(l)
        n = 1 << (l - 1)
        assert lm.kept.sum() == 2 * n * n - 2 * n
        assert lm.n == (n - 1) * (n + 1)
        xs = lm.verts[lm.dof_vert, 0]
        top = 1 << H.aux.J
        assert xs.min() == 2 * (top // n) and xs.max() == top      # x = 2h .. 1
        # natural conditions on y = 0, y = 1 and x = 1: those vertices are unknowns
        assert np.any(lm.verts[lm.dof_vert, 1] == 0) and np.any(lm.verts[lm.dof_vert, 1] == top)


def test_mixed_grids_precondition_the_mixed_problem(left_dirichlet):
    # B_co stays SPD (small case, dense) and, on a problem with Neumann sides, the mixed grids
    # need far fewer iterations than Dirichlet grids on the root box (the reason for them)
    X, T, H = left_dirichlet
    f = np.random.default_rng(0).uniform(-1, 1, H.n)
    u, it, info = H.solve(f, 1e-8)
    Hb = Hierarchy(X, T, np.ones(len(T)), dirichlet=X[:, 0] == 0.0, domain="box", coarse_max_dofs=256)
    ub, itb, _ = Hb.solve(f, 1e-8)
    assert info["status"] == "ok" and it < 0.75 * itb, (it, itb)
    assert np.linalg.norm(u - ub) <= 1e-6 * np.linalg.norm(ub)
    Xs, Ts, _ = W.square_mesh(16, jitter=0.2)
    Hs = Hierarchy(Xs, Ts, np.ones(len(Ts)), dirichlet=Xs[:, 0] == 0.0, domain="mixed")
    B = Hs.preconditioner()
    M = np.column_stack([B(e) for e in np.eye(Hs.n)])
    assert np.abs(M - M.T).max() <= 1e-12 * np.abs(M).max()
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0


def test_annulus_kept_set_by_sampling():
    # Neumann hole, Dirichlet outer circle. A simplex with a sampled point inside the domain is
    # kept unless it meets Gamma_D; a kept simplex meets the domain or a boundary edge; a vertex
    # of a simplex whose samples all sit near the outer circle is never an unknown
    X, T, _ = W.annulus_mesh(60)
    r = np.hypot(X[:, 0] - 0.5, X[:, 1] - 0.5)
    outer = boundary_vertices(T, len(X)) & (r > 0.35)
    H = Hierarchy(X, T, np.ones(len(T)), dirichlet=outer, domain="mixed")
    dom = H.meshes.domain
    lm = H.meshes.level(H.aux.J)
    ts = np.array([[a, b, 1 - a - b] for a in np.linspace(0.02, 0.96, 9) for b in np.linspace(0.02, 0.96, 9)
                   if a + b <= 0.98])
    checked = 0
    for s in range(len(lm.simp)):
        P = np.array([dom.aux_point(H.tree, lm.verts[v]) for v in lm.simp[s]])
        pts = ts @ P
        if not lm.kept[s]:
            inside = [p for p in pts if 0.21 < np.hypot(p[0] - 0.5, p[1] - 0.5) < 0.49]
            if inside:   # safely inside the annulus: dropped only for meeting Gamma_D
                assert np.hypot(*(P.mean(axis=0) - 0.5)) > 0.4
                checked += 1
        else:
            rr = np.hypot(pts[:, 0] - 0.5, pts[:, 1] - 0.5)
            assert rr.min() < 0.51 and rr.max() > 0.19    # meets the closed annulus (polygonal)
    assert checked > 0
    # the hole's boundary is natural: unknowns lie on the hole side of the inner circle too
    rv = np.array([np.hypot(*(dom.aux_point(H.tree, lm.verts[v]) - 0.5)) for v in lm.dof_vert])
    assert rv.min() < 0.2 and rv.max() < 0.5
