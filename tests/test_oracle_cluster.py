"""Pins of the cluster tree and closure (oracle.cluster; Sections 3.1-3.2)."""
import itertools
import math

import numpy as np
import pytest

import workloads as W
from oracle import cluster


def _geometric_box(x, a, L, level):
    """Index of the half-open level box containing x, by direct comparison (no keys)."""
    n = 1 << (level - 1)
    side = L / n
    out = []
    for k in range(len(x)):
        i = 0
        while i + 1 < n and a[k] + (i + 1) * side <= x[k]:
            i += 1
        out.append(i)
    return tuple(out)


def test_keys_match_geometric_boxes_on_dyadic_points():
    # barycenters exactly on split lines must go to the upper/right child (half-open boxes)
    rng = np.random.default_rng(0)
    a = np.array([0.0, 0.0])
    L = 1.0
    pts = rng.integers(0, 64, (300, 2)) / 64.0          # many on split lines
    pts = np.vstack([pts, rng.uniform(0, 1, (300, 2))])
    keys = cluster.axis_keys(pts, a, L, 2)
    for lev in range(1, 9):
        bx = cluster.box_of(keys, lev, 2)
        for p, b in zip(pts, bx):
            assert tuple(b) == _geometric_box(p, a, L, lev)


def test_barycenter_rounding_order():
    c = np.array([[0.1, 0.7], [0.2, 0.3], [0.3, 0.9]])
    xi = cluster.barycenters(c, np.array([[0, 1, 2]]))[0]
    assert xi[0] == ((0.1 + 0.2) + 0.3) / 3.0
    assert xi[1] == ((0.7 + 0.3) + 0.9) / 3.0


def _brute_counts(xi, a, L, level):
    cnt = {}
    for p in xi:
        b = (level,) + _geometric_box(p, a, L, level)
        cnt[b] = cnt.get(b, 0) + 1
    return cnt


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_refined_set_brute_force(seed):
    rng = np.random.default_rng(seed)
    # clustered points: refinement to several levels
    pts = np.vstack([rng.uniform(0, 1, (60, 2)), 0.02 * rng.standard_normal((60, 2)) + 0.3])
    pts = np.clip(pts, 0, 1)
    pts = np.vstack([pts, [[0, 0], [1, 1]]])
    # one "element" per point: degenerate triangles are fine for the tree
    coords = pts
    elems = np.stack([np.arange(len(pts))] * 3, 1)
    xi = cluster.barycenters(coords, elems)
    a, L = cluster.root_box(coords)
    keys = cluster.axis_keys(xi, a, L, 2)
    R0 = cluster.refined_by_count(keys, 2, 3)
    brute = set()
    for lev in range(1, 31):
        cnt = _brute_counts(xi, a, L, lev)
        sel = {b for b, c in cnt.items() if c > 3}
        if not sel:
            break
        brute |= sel
    assert R0 == brute


def _touch(b1, b2, d):
    """Closed boxes b1, b2 share a facet or (3-D) an edge: intersection of dimension >= d-1 (2-D), >= 1 (3-D)."""
    L1 = 1 << (30 - b1[0] + 1)
    L2 = 1 << (30 - b2[0] + 1)
    dims = 0
    for k in range(d):
        lo = max(b1[1 + k] * L1, b2[1 + k] * L2)
        hi = min((b1[1 + k] + 1) * L1, (b2[1 + k] + 1) * L2)
        if hi < lo:
            return False
        if hi > lo:
            dims += 1
    return dims >= (d - 1 if d == 2 else 1)


def _check_tree(tree):
    d = tree.d
    R = tree.R
    # R contains R0, every refined box is in the tree
    assert tree.R0 <= R
    for b in R:
        assert cluster.in_tree(b, R)
    # leaves hold at most n_min
    for lf in tree.leaves:
        lev = lf[0]
        bx = cluster.box_of(tree.keys, lev, d)
        cnt = int(np.all(bx == np.array(lf[1:]), axis=1).sum())
        assert cnt <= tree.n_min
    # balance, brute force over leaf pairs
    lv = tree.leaves
    for i in range(len(lv)):
        for j in range(i + 1, len(lv)):
            if abs(lv[i][0] - lv[j][0]) > 1 and _touch(lv[i], lv[j], d):
                raise AssertionError(f"unbalanced {lv[i]} {lv[j]}")
    # minimality: every closure box is forced
    offs = cluster.touch_offsets(d)
    for b in R - tree.R0:
        desc = {c for c in R if c[0] > b[0] and all((c[1 + k] >> (c[0] - b[0])) == b[1 + k] for k in range(d))}
        Rm = R - {b} - desc
        assert cluster.violates(b, Rm, offs), f"closure box {b} is not forced"


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_closure_balance_minimality_and_literal_2d(seed):
    rng = np.random.default_rng(seed)
    pts = np.vstack([rng.uniform(0, 1, (40, 2)), 1e-3 * rng.standard_normal((40, 2)) + rng.uniform(0.1, 0.9, 2),
                     [[0, 0], [1, 1]]])
    pts = np.clip(pts, 0, 1)
    elems = np.stack([np.arange(len(pts))] * 3, 1)
    tree = cluster.BoxTree(pts, elems, check_literal=True)
    assert len(tree.R) > len(tree.R0)
    _check_tree(tree)


@pytest.mark.parametrize("seed", [0, 1])
def test_closure_balance_minimality_and_literal_3d(seed):
    rng = np.random.default_rng(seed)
    pts = np.vstack([rng.uniform(0, 1, (60, 3)), 2e-3 * rng.standard_normal((60, 3)) + rng.uniform(0.2, 0.8, 3),
                     [[0, 0, 0], [1, 1, 1]]])
    pts = np.clip(pts, 0, 1)
    elems = np.stack([np.arange(len(pts))] * 4, 1)
    tree = cluster.BoxTree(pts, elems, n_min=3, check_literal=True)
    assert len(tree.R) > len(tree.R0)
    _check_tree(tree)


def test_depth_bound_lemma():
    # Section 3.1 lemma: a refined box has diameter >= h, so (level-1) <= log2(sqrt(d) L / h)
    c = W.make_config(1, scale=0.002)
    tree = cluster.BoxTree(c["coords"], c["elems"])
    xi = tree.xi
    import scipy.spatial
    dd, _ = scipy.spatial.cKDTree(xi).query(xi, k=2)
    h = dd[:, 1].min()
    bound = math.log2(math.sqrt(2) * tree.L / h)
    assert max(b[0] for b in tree.R) - 1 <= bound
    assert tree.J <= bound + 2


def test_worked_example_square64_uniform_level7():
    c = W.make_config(0)
    tree = cluster.BoxTree(c["coords"], c["elems"], check_literal=True)
    assert tree.J == 7
    expect = {(lev, i, j) for lev in range(1, 7) for i in range(1 << (lev - 1)) for j in range(1 << (lev - 1))}
    assert tree.R == expect
    assert len(tree.leaves) == 64 * 64


def test_worked_example_kuhn_cube_uniform():
    c = W.make_config(2, scale=1 / 16)   # 8^3 cells
    tree = cluster.BoxTree(c["coords"], c["elems"])
    n = c["n"]
    assert tree.n_min == 7
    assert tree.J == int(math.log2(n)) + 1
    assert len(tree.leaves) == n ** 3
    assert tree.R == tree.R0


@pytest.mark.parametrize("cfg,scale", [(1, 0.002), (2, 1 / 16)])
def test_leaf_kappa_means(cfg, scale):
    c = W.make_config(cfg, scale=scale)
    d = c["coords"].shape[1]
    tree = cluster.BoxTree(c["coords"], c["elems"])
    lk = tree.leaf_kappa(c["kappa"])
    for lf, v in list(lk.items())[:300]:
        q = lf
        while True:
            bx = cluster.box_of(tree.keys, q[0], d)
            m = np.all(bx == np.array(q[1:]), axis=1)
            if m.any():
                assert v == pytest.approx(c["kappa"][m].mean(), rel=1e-14)
                break
            q = cluster.parent(q)
