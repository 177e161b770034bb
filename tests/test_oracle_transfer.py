"""Pins of the Scott-Zhang transfer Pi (oracle.transfer; Section 4.1)."""
import numpy as np
import pytest

import workloads as W
from oracle import auxgrid, cluster, fem, transfer


def _setup(coords, elems):
    tree = cluster.BoxTree(coords, elems)
    m = auxgrid.AuxMeshes(tree)
    dofs = fem.dof_vertices(fem.default_dirichlet(coords))
    return tree, m, dofs


@pytest.mark.parametrize("kind", ["square", "graded", "cube"])
def test_p1_reproduction(kind):
    if kind == "square":
        coords, elems, _ = W.square_mesh(24, 0.3, cfg=0, item=9)
    elif kind == "graded":
        c = W.make_config(1, scale=0.003)
        coords, elems = c["coords"], c["elems"]
    else:
        coords, elems, _ = W.kuhn_cube_mesh(4, 0.2, cfg=2, item=9)
    tree, m, dofs = _setup(coords, elems)
    Pi = transfer.transfer(tree, m, coords, elems, dofs, all_aux_vertices=True)
    lm = m.level(tree.J)
    unit = tree.L * 2.0 ** (-tree.J)
    X = tree.a + lm.verts * unit
    d = coords.shape[1]
    lin = lambda Y: 0.7 + Y @ np.array([1.3, -2.1, 0.4][:d])
    np.testing.assert_allclose(Pi @ lin(X), lin(coords[dofs]), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(Pi @ np.ones(Pi.shape[1]), 1.0, atol=1e-13)


def test_identity_when_fine_mesh_is_finest_aux_mesh():
    coords, elems, _ = W.square_mesh(64, 0.0, diagonals="ur")
    tree, m, dofs = _setup(coords, elems)
    Pi = transfer.transfer(tree, m, coords, elems, dofs)
    lm = m.level(tree.J)
    unit = tree.L * 2.0 ** (-tree.J)
    pos = {tuple(v): i for i, v in enumerate(lm.verts[lm.dof_vert].tolist())}
    D = Pi.toarray()
    for i, v in enumerate(dofs):
        j = pos[tuple(np.round(coords[v] / unit).astype(int).tolist())]
        row = D[i]
        assert row[j] == 1.0
        assert np.count_nonzero(row) == 1


def test_sz_edge_choice():
    coords, elems, _ = W.square_mesh(6, 0.2, cfg=0, item=1)
    dofs = fem.dof_vertices(fem.default_dirichlet(coords))
    sig = transfer.sz_simplices(elems, dofs, 2)
    for (i, j) in sig:
        nb = set(elems[np.any(elems == i, axis=1)].ravel().tolist()) - {i}
        assert j == min(nb)
