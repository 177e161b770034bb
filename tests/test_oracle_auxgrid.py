"""Pins of the auxiliary level meshes (oracle.auxgrid; Section 3.3)."""
import math
from collections import Counter

import numpy as np
import pytest

import workloads as W
from oracle import auxgrid, cluster


def _tree_2d(seed):
    rng = np.random.default_rng(seed)
    pts = np.vstack([rng.uniform(0, 1, (40, 2)), 1e-3 * rng.standard_normal((40, 2)) + rng.uniform(0.1, 0.9, 2),
                     [[0, 0], [1, 1]]])
    pts = np.clip(pts, 0, 1)
    return cluster.BoxTree(pts, np.stack([np.arange(len(pts))] * 3, 1))


def _tree_3d(seed):
    rng = np.random.default_rng(seed)
    pts = np.vstack([rng.uniform(0, 1, (12, 3)), 2e-2 * rng.standard_normal((12, 3)) + rng.uniform(0.2, 0.8, 3),
                     [[0, 0, 0], [1, 1, 1]]])
    pts = np.clip(pts, 0, 1)
    return cluster.BoxTree(pts, np.stack([np.arange(len(pts))] * 4, 1), n_min=3)


def _volumes(lm):
    V = lm.verts[lm.simp].astype(np.int64)
    E = V[:, 1:] - V[:, :1]
    if lm.d == 2:
        det = E[:, 0, 0] * E[:, 1, 1] - E[:, 0, 1] * E[:, 1, 0]
    else:
        det = (E[:, 0, 0] * (E[:, 1, 1] * E[:, 2, 2] - E[:, 1, 2] * E[:, 2, 1])
               - E[:, 0, 1] * (E[:, 1, 0] * E[:, 2, 2] - E[:, 1, 2] * E[:, 2, 0])
               + E[:, 0, 2] * (E[:, 1, 0] * E[:, 2, 1] - E[:, 1, 1] * E[:, 2, 0]))
    return np.abs(det)


def _check_conforming(lm):
    d = lm.d
    top = 1 << lm.J
    vol = _volumes(lm)
    assert np.all(vol > 0)
    assert vol.sum() == math.factorial(d) * top ** d
    facets = Counter()
    for s in lm.simp:
        for k in range(d + 1):
            facets[tuple(sorted(np.delete(s, k).tolist()))] += 1
    for f, c in facets.items():
        X = lm.verts[list(f)]
        on_bnd = any(np.all(X[:, k] == 0) or np.all(X[:, k] == top) for k in range(d))
        assert c == (1 if on_bnd else 2), (f, c)
    # no vertex inside an edge (2-D) / no vertex in an edge or face (3-D): edge midpoint test on all edges
    vset = {tuple(v) for v in lm.verts.tolist()}
    for s in lm.simp:
        for a in range(d + 1):
            for b in range(a + 1, d + 1):
                P, Q = lm.verts[s[a]], lm.verts[s[b]]
                if np.all((P + Q) % 2 == 0):
                    assert tuple(((P + Q) // 2).tolist()) not in vset, "hanging node on an edge"


def _det(E):
    """Integer determinants of (m, d, d) edge matrices (rows = edges)."""
    if E.shape[-1] == 2:
        return E[..., 0, 0] * E[..., 1, 1] - E[..., 0, 1] * E[..., 1, 0]
    return (E[..., 0, 0] * (E[..., 1, 1] * E[..., 2, 2] - E[..., 1, 2] * E[..., 2, 1])
            - E[..., 0, 1] * (E[..., 1, 0] * E[..., 2, 2] - E[..., 1, 2] * E[..., 2, 0])
            + E[..., 0, 2] * (E[..., 1, 0] * E[..., 2, 1] - E[..., 1, 1] * E[..., 2, 0]))


def _inside_all(W_, X):
    """Which simplices W_ (m, d+1, d) contain point X (d,) (closed), exact int64 sign tests."""
    d = W_.shape[2]
    tot = _det(W_[:, 1:] - W_[:, :1])
    ok = np.ones(len(W_), dtype=bool)
    for k in range(d + 1):
        Q = W_.copy()
        Q[:, k] = X
        sub = _det(Q[:, 1:] - Q[:, :1])
        ok &= (sub * np.sign(tot)) >= 0
    return ok


def _check_nested(fine, coarse):
    d = fine.d
    Wc = coarse.verts[coarse.simp].astype(np.int64) * (d + 1)
    for s in fine.simp:
        V = fine.verts[s].astype(np.int64)
        hits = np.nonzero(_inside_all(Wc, V.sum(axis=0)))[0]
        assert len(hits) == 1
        for v in V:
            assert _inside_all(Wc[hits] // (d + 1) * 1, v)[0] or _inside_all(Wc[hits], v * (d + 1))[0]


@pytest.mark.parametrize("seed", [0, 1])
def test_levels_conforming_nested_2d(seed):
    tree = _tree_2d(seed)
    m = auxgrid.AuxMeshes(tree)
    assert any(m.level(l).box_fan.any() for l in range(1, tree.J + 1))
    prev = None
    for l in range(1, tree.J + 1):
        lm = m.level(l)
        _check_conforming(lm)
        if prev is not None:
            _check_nested(lm, prev)
        prev = lm


def test_levels_conforming_nested_3d():
    tree = _tree_3d(0)
    m = auxgrid.AuxMeshes(tree)
    assert any(m.level(l).box_fan.any() for l in range(1, tree.J + 1))
    prev = None
    for l in range(1, tree.J + 1):
        lm = m.level(l)
        _check_conforming(lm)
        if prev is not None:
            _check_nested(lm, prev)
        prev = lm


def test_min_angle_45_degrees_2d():
    tree = _tree_2d(2)
    m = auxgrid.AuxMeshes(tree)
    for l in range(1, tree.J + 1):
        lm = m.level(l)
        P = lm.verts[lm.simp].astype(float)
        for k in range(3):
            u = P[:, (k + 1) % 3] - P[:, k]
            v = P[:, (k + 2) % 3] - P[:, k]
            ang = np.degrees(np.arccos((u * v).sum(1) / np.linalg.norm(u, axis=1) / np.linalg.norm(v, axis=1)))
            assert np.all(np.isclose(ang, 45) | np.isclose(ang, 90))


def test_square64_finest_level_is_uniform_kuhn_grid():
    c = W.make_config(0)
    tree = cluster.BoxTree(c["coords"], c["elems"])
    m = auxgrid.AuxMeshes(tree)
    lm = m.level(7)
    assert not lm.box_fan.any()
    assert len(lm.simp) == 2 * 64 * 64
    assert lm.n == 63 * 63
    # Section 5.1: uniform hierarchy, dim V_l = (2^l - 1)^2 with the index shifted by one level here
    for l in range(2, 8):
        assert m.level(l).n == (2 ** (l - 1) - 1) ** 2


def test_morton_order():
    X = np.array([[0, 0], [1, 0], [0, 1], [1, 1], [2, 0], [0, 2]])
    order = auxgrid.morton_order(X)
    # key: x bit above y bit: (0,0)=0, (0,1)=1, (1,0)=2, (1,1)=3, (0,2)=4, (2,0)=8
    assert [tuple(X[i]) for i in order] == [(0, 0), (0, 1), (1, 0), (1, 1), (0, 2), (2, 0)]
