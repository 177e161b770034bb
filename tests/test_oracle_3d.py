"""Pins of the oracle's 3-D path (tetrahedra): the auxiliary operators of Section 4.1 on the
Kuhn/cone templates of the octree (Section 3.3), the Scott-Zhang face rule of the transfer
(Section 4.1), B_co (Algorithm 1) and its convergence (Section 5.2).

Each pin checks against something independent of the function it pins: an exact identity
(Galerkin, B_co's closed form), a second construction (the fine float assembly, point location
and barycentric evaluation, a brute-force face search), or the behaviour the paper reports.
"""
import itertools

import numpy as np
import pytest

import workloads as W
from oracle import auxgrid, auxops, cluster, fem, transfer
from oracle.hierarchy import Hierarchy


def _graded_cube(n=8, item=3):
    # jittered Kuhn cube squeezed towards the corner (0,0,0): with n_min = 3 the tree is graded,
    # the closure adds boxes, and the level meshes carry cone (fan) boxes
    coords, elems, _ = W.kuhn_cube_mesh(n, 0.1, cfg=2, item=item)
    kappa = np.random.default_rng(item).uniform(0.5, 2.0, len(elems))
    return coords ** 2, elems, kappa


@pytest.fixture(scope="module")
def graded_cube_ops():
    coords, elems, kappa = _graded_cube()
    tree = cluster.BoxTree(coords, elems, n_min=3)
    m = auxgrid.AuxMeshes(tree)
    ops = auxops.AuxOperators(tree, m, kappa, coarse_max_dofs=20)
    return tree, m, ops


def test_graded_cube_has_cone_boxes(graded_cube_ops):
    tree, m, ops = graded_cube_ops
    assert ops.J - ops.lc >= 3
    fans = sum(int(np.count_nonzero(m.level(l).box_fan)) for l in range(ops.lc, ops.J + 1))
    assert fans > 0


def test_galerkin_identity_3d(graded_cube_ops):
    # A_(l-1) = P_l^T A_l P_l: the coarse gradients are constant on the coarse simplices, so the
    # coefficient means over the child Kuhn simplices give exactly the Galerkin product
    tree, m, ops = graded_cube_ops
    for l in range(ops.J, ops.lc, -1):
        P = ops.P[l]
        G = (P.T @ ops.A[l] @ P).toarray()
        Ac = ops.A[l - 1].toarray()
        assert np.abs(G - Ac).max() <= 1e-13 * np.abs(Ac).max(), l


def test_prolongation_is_nodal_interpolation_3d(graded_cube_ops):
    """P_l v equals the coarse P1 function evaluated at the fine unknowns, with the coarse simplex
    found by brute-force point location and barycentric coordinates from a 3 x 3 inverse."""
    tree, m, ops = graded_cube_ops
    rng = np.random.default_rng(0)
    for l in range(ops.J, ops.lc, -1):
        fine, coarse = m.level(l), m.level(l - 1)
        vc = rng.standard_normal(coarse.n)
        vv = np.zeros(len(coarse.verts))
        vv[coarse.dof_vert] = vc
        Wc = coarse.verts[coarse.simp].astype(float)          # (s, 4, 3)
        T0 = Wc[:, 0]
        Einv = np.linalg.inv(np.transpose(Wc[:, 1:] - Wc[:, :1], (0, 2, 1)))
        got = ops.P[l] @ vc
        sample = rng.choice(fine.n, size=min(fine.n, 300), replace=False)   # every level, any row kind
        for i in sample:
            X = fine.verts[fine.dof_vert[i]].astype(float)
            lam = np.einsum("sij,sj->si", Einv, X - T0)
            lam = np.concatenate([1 - lam.sum(1, keepdims=True), lam], 1)
            s = np.nonzero(np.all(lam >= -1e-12, axis=1))[0][0]
            assert got[i] == pytest.approx(lam[s] @ vv[coarse.simp[s]], rel=1e-12, abs=1e-12)


def test_aux_matrix_equals_fine_kuhn_matrix():
    # unjittered Kuhn cube: with n_min = 7 every finest box holds its cell's 6 barycenters, the
    # finest auxiliary grid is the original mesh (same main diagonal), so A_J (exact integer
    # assembly) equals the fine float assembly, with kappa constant per cell
    n = 8
    coords, elems, cells = W.kuhn_cube_mesh(n, 0.0)
    kc = np.random.default_rng(4).uniform(0.5, 2.0, n ** 3)
    kappa = kc[cells[:, 0] + n * (cells[:, 1] + n * cells[:, 2])]
    A, dofs = fem.assemble(coords, elems, kappa)
    tree = cluster.BoxTree(coords, elems)
    m = auxgrid.AuxMeshes(tree)
    ops = auxops.AuxOperators(tree, m, kappa, coarse_max_dofs=10)
    lm = m.level(tree.J)
    unit = tree.L * 2.0 ** (-tree.J)
    pos = {tuple(np.round(coords[v] / unit).astype(int)): i for i, v in enumerate(dofs)}
    perm = np.array([pos[tuple(lm.verts[v])] for v in lm.dof_vert])
    AJ = ops.A[tree.J].toarray()
    Af = A.toarray()[np.ix_(perm, perm)]
    assert np.abs(AJ - Af).max() <= 1e-13 * np.abs(Af).max()
    # a stiffness matrix annihilates constants away from the boundary rows
    interior = np.array([np.all((lm.verts[v] > 2) & (lm.verts[v] < 2 ** tree.J - 2)) for v in lm.dof_vert])
    assert np.abs(AJ[interior].sum(1)).max() <= 1e-13 * np.abs(AJ).max()


def test_sz_face_is_lexicographically_smallest():
    # brute force over every tetrahedron: the smallest (j, k), j < k, among the faces (i, j, k)
    # of the mesh that contain the unknown's vertex i
    coords, elems, _ = W.kuhn_cube_mesh(5, 0.2, cfg=2, item=1)
    elems = np.random.default_rng(0).permuted(elems, axis=1)     # any vertex order inside a tet
    A, dofs = fem.assemble(coords, elems, np.ones(len(elems)))
    best = {}
    for t in elems.tolist():
        for face in itertools.combinations(t, 3):
            for i in face:
                jk = tuple(sorted(x for x in face if x != i))
                if i not in best or jk < best[i]:
                    best[i] = jk
    got = transfer.sz_simplices(elems, dofs, 3)
    for row in got.tolist():
        assert tuple(row[1:]) == best[row[0]]


@pytest.fixture(scope="module")
def tiny_cube():
    coords, elems, kappa = _graded_cube(n=6, item=5)
    H = Hierarchy(coords, elems, kappa, n_min=3, coarse_max_dofs=20)
    assert H.n <= 200 and H.aux.J - H.aux.lc >= 2
    return H


def _dense(op, n):
    return np.column_stack([op(e) for e in np.eye(n)])


def _gs_dense(A, col):
    n = A.shape[0]
    order = np.lexsort((np.arange(n), col))
    Ap = A.toarray()[np.ix_(order, order)]
    Sp = np.linalg.inv(np.tril(Ap))
    S = np.zeros_like(Sp)
    S[np.ix_(order, order)] = Sp
    return S


def test_preconditioner_3d_symmetric_positive_definite(tiny_cube):
    H = tiny_cube
    Bd = _dense(H.preconditioner(), H.n)
    assert np.abs(Bd - Bd.T).max() <= 1e-13 * np.abs(Bd).max()
    assert np.linalg.eigvalsh(0.5 * (Bd + Bd.T)).min() > 0


def test_preconditioner_3d_closed_form(tiny_cube):
    # B_co = S^T D S + (I - S^T A) Pi B~ Pi^T (I - A S)
    H = tiny_cube
    B = H.preconditioner()
    n = H.n
    A = H.A.toarray()
    S = _gs_dense(H.A, H.colour_fine)
    D = np.diag(np.diag(A))
    Bt = _dense(lambda g: B.vcycle(H.aux.J, g), H.Pi.shape[1])
    Pi = H.Pi.toarray()
    I = np.eye(n)
    closed = S.T @ D @ S + (I - S.T @ A) @ Pi @ Bt @ Pi.T @ (I - A @ S)
    np.testing.assert_allclose(_dense(B, n), closed, rtol=1e-11, atol=1e-11 * np.abs(closed).max())


def _rate(H, its=12):
    B, A = H.preconditioner(), H.A
    e = np.random.default_rng(0).standard_normal(H.n)
    norm = lambda v: float(np.sqrt(v @ (A @ v)))
    ns = [norm(e)]
    for _ in range(its):
        e = e - B(A @ e)
        ns.append(norm(e))
    return (ns[-1] / ns[4]) ** (1.0 / (its - 4))


def test_stationary_rate_3d_small_and_level_independent():
    # the jittered checkerboard cube of the 3-D workload at 8^3 and 16^3 cells, V-cycles down to
    # at most 30 unknowns (2 and 3 auxiliary levels): the contraction of e <- (I - B_co A) e stays
    # well below the paper's ~0.4 and does not grow with the number of levels
    hs = []
    for scale in (1 / 16, 1 / 8):
        c = W.make_config(2, scale=scale)
        hs.append(Hierarchy(c["coords"], c["elems"], c["kappa"], coarse_max_dofs=30))
    assert hs[1].aux.J - hs[1].aux.lc > hs[0].aux.J - hs[0].aux.lc
    rates = [_rate(H) for H in hs]
    assert all(r < 0.45 for r in rates), rates
    assert rates[1] <= rates[0] + 0.1, rates
