"""Pins of the auxiliary operators A_l, P_l (oracle.auxops; Algorithm 2, Section 5.1)."""
import numpy as np
import pytest

import workloads as W
from oracle import auxgrid, auxops, cluster


@pytest.fixture(scope="module")
def graded_ops():
    c = W.make_config(1, scale=0.003)
    tree = cluster.BoxTree(c["coords"], c["elems"])
    m = auxgrid.AuxMeshes(tree)
    ops = auxops.AuxOperators(tree, m, c["kappa"], coarse_max_dofs=50)
    return tree, m, ops


def test_galerkin_identity(graded_ops):
    tree, m, ops = graded_ops
    assert ops.J - ops.lc >= 3
    for l in range(ops.J, ops.lc, -1):
        P = ops.P[l]
        G = (P.T @ ops.A[l] @ P).toarray()
        Ac = ops.A[l - 1].toarray()
        assert np.abs(G - Ac).max() <= 1e-13 * np.abs(Ac).max()


def test_prolongation_midpoint_structure(graded_ops):
    tree, m, ops = graded_ops
    for l in range(ops.J, ops.lc, -1):
        fine, coarse = m.level(l), m.level(l - 1)
        cvert = {tuple(v): i for i, v in enumerate(coarse.verts.tolist())}
        P = ops.P[l].tocsr()
        for i in range(P.shape[0]):
            X = fine.verts[fine.dof_vert[i]]
            cols = P.indices[P.indptr[i]:P.indptr[i + 1]]
            vals = P.data[P.indptr[i]:P.indptr[i + 1]]
            if tuple(X) in cvert:
                j = coarse.dof_of_vert[cvert[tuple(X)]]
                assert list(cols) == [j] and list(vals) == [1.0]
            else:
                assert set(vals.tolist()) <= {0.5}
                # the two endpoints of the split coarse edge, reflected through X
                for j in cols:
                    Y = coarse.verts[coarse.dof_vert[j]]
                    assert tuple(2 * X - Y) in cvert


def test_prolongation_is_nodal_interpolation(graded_ops):
    """P v equals the coarse P1 function v evaluated at the fine unknowns (independent point location)."""
    tree, m, ops = graded_ops
    rng = np.random.default_rng(0)
    for l in range(ops.J, ops.lc, -1):
        fine, coarse = m.level(l), m.level(l - 1)
        vc = rng.standard_normal(coarse.n)
        vv = np.zeros(len(coarse.verts))
        vv[coarse.dof_vert] = vc
        Wc = coarse.verts[coarse.simp].astype(float)
        T0 = Wc[:, 0]
        E = np.transpose(Wc[:, 1:] - Wc[:, :1], (0, 2, 1))
        Einv = np.linalg.inv(E)
        got = ops.P[l] @ vc
        for i, v in enumerate(fine.dof_vert):
            X = fine.verts[v].astype(float)
            lam = np.einsum("sij,sj->si", Einv, X - T0)
            lam = np.concatenate([1 - lam.sum(1, keepdims=True), lam], 1)
            s = np.nonzero(np.all(lam >= -1e-12, axis=1))[0][0]
            exp = lam[s] @ vv[coarse.simp[s]]
            assert got[i] == pytest.approx(exp, rel=1e-12, abs=1e-12)


def test_square64_textbook_five_point():
    c = W.make_config(0)
    tree = cluster.BoxTree(c["coords"], c["elems"])
    m = auxgrid.AuxMeshes(tree)
    ops = auxops.AuxOperators(tree, m, c["kappa"], coarse_max_dofs=10)
    for l in range(ops.lc, ops.J + 1):
        A = ops.A[l]
        n = 2 ** (l - 1) - 1
        assert A.shape == (n * n, n * n)
        D = A.diagonal()
        assert np.all(D == 4.0)
        off = A - np.diag(D) if False else A.copy()
        off.setdiag(0)
        off.eliminate_zeros()
        assert set(off.data.tolist()) == {-1.0}
        assert off.nnz == 4 * n * n - 4 * n


def test_aux_matrix_equals_fine_matrix_on_matching_mesh():
    # unjittered square with lower-left to upper-right diagonals: the original mesh is sigma^(J),
    # so A_J (integer assembly) must equal the fine matrix (float assembly), up to the numbering
    from oracle import fem
    coords, elems, _ = W.square_mesh(32, 0.0, diagonals="ur")
    kappa = np.random.default_rng(3).uniform(0.5, 2.0, len(elems))
    # constant per 2x2-element block = per leaf box of level 6 (cluster of 2 barycenters)
    kappa = np.repeat(kappa[0::2], 2)
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
    np.testing.assert_allclose(AJ, Af, rtol=1e-13, atol=1e-14)


def test_kuhn_aux_seven_point():
    c = W.make_config(2, scale=1 / 16)
    tree = cluster.BoxTree(c["coords"], c["elems"])
    m = auxgrid.AuxMeshes(tree)
    ops = auxops.AuxOperators(tree, m, np.ones(len(c["elems"])), coarse_max_dofs=10)
    A = ops.A[tree.J]
    n = c["n"] - 1
    assert A.nnz == 7 * n ** 3 - 6 * n ** 2
