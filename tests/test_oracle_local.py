"""Pins of local smoothing on N~_l (oracle.auxops.local_set, oracle.asmg smoothing="local").

N~_l (Section 4.3, the decomposition V_J = sum_l sum_{k in N~_l} V_{l,k}) holds the unknowns
of level l that are new or whose nodal basis function changed between levels l-1 and l. The
oracle reads it off P_l; these tests count it independently from the level meshes: a basis
function phi_k changes exactly when some edge of sigma^(l-1) at k is bisected, i.e. its
midpoint is a new vertex of sigma^(l).
"""
import numpy as np
import pytest

import workloads as W
from oracle import asmg, auxops
from oracle.hierarchy import Hierarchy


def _geometric_local_set(meshes, l):
    fine, coarse = meshes.level(l), meshes.level(l - 1)
    cset = {tuple(v) for v in coarse.verts.tolist()}
    fidx = {tuple(v): i for i, v in enumerate(fine.verts.tolist())}
    new = np.array([tuple(fine.verts[v]) not in cset for v in fine.dof_vert])
    changed = np.zeros(fine.n, dtype=bool)
    d = fine.d
    for s in coarse.simp:
        for a in range(d + 1):
            for b in range(a + 1, d + 1):
                pa, pb = coarse.verts[s[a]], coarse.verts[s[b]]
                mid = tuple(((pa + pb) // 2).tolist())
                if np.any((pa + pb) % 2) or mid in cset or mid not in fidx:
                    continue
                for p in (pa, pb):   # the edge (a, b) is bisected: both end functions change
                    j = fine.dof_of_vert[fidx[tuple(p.tolist())]]
                    if j >= 0:
                        changed[j] = True
    return new | changed


@pytest.mark.parametrize("which", ["graded2d", "graded_cube"])
def test_local_set_matches_bisected_edges(which, graded_small):
    if which == "graded2d":
        H = graded_small[1]
    else:
        coords, elems, _ = W.kuhn_cube_mesh(6, 0.1, cfg=2, item=3)
        H = Hierarchy(coords ** 2, elems, np.ones(len(elems)), n_min=3, coarse_max_dofs=20)
    partial = False
    for l in range(H.aux.lc + 1, H.aux.J + 1):
        m = auxops.local_set(H.aux.P[l])
        g = _geometric_local_set(H.meshes, l)
        assert np.array_equal(m, g), l
        partial |= bool(m.sum() < len(m))
    if which == "graded2d":
        assert partial  # the graded hierarchy has levels where only part of the unknowns move


def test_uniform_hierarchy_local_equals_full(cfg0_hier):
    _, H = cfg0_hier
    for l in range(H.aux.lc + 1, H.aux.J + 1):
        assert auxops.local_set(H.aux.P[l]).all()
    r = np.random.default_rng(4).standard_normal(H.n)
    zf = H.preconditioner()(r)
    zl = H.preconditioner(smoothing="local")(r)
    assert np.array_equal(zf, zl)


@pytest.fixture(scope="module")
def tiny():
    c = W.make_config(1, scale=0.0004)
    H = Hierarchy(c["coords"], c["elems"], c["kappa"], coarse_max_dofs=30)
    return c, H


def test_local_preconditioner_spd(tiny):
    _, H = tiny
    B = H.preconditioner(smoothing="local")
    assert any(not m.all() for m in B.masks.values())
    Bd = np.column_stack([B(e) for e in np.eye(H.n)])
    assert np.abs(Bd - Bd.T).max() <= 1e-13 * np.abs(Bd).max()
    assert np.linalg.eigvalsh(0.5 * (Bd + Bd.T)).min() > 0


def test_local_smoothing_solve(graded_small):
    c, H = graded_small
    f = c["f_vertex"][H.dofs]
    u, it, info = H.solve(f, 1e-10, smoothing="local")
    ref = np.linalg.solve(H.A.toarray(), f)
    assert np.linalg.norm(u - ref) <= 1e-7 * np.linalg.norm(ref)
    uf, itf, _ = H.solve(f, 1e-10)
    assert it <= itf + 2
