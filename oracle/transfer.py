"""Scott-Zhang transfer Pi from the finest auxiliary space to the original space (oracle).

Section 4.1 uses the Scott-Zhang quasi-interpolation as the transfer Pi: V -> the
original P1 space, with Pi^t its transpose. The displayed formula is garbled (its
dual function has no index and it integrates over Omega). The reading used is
Scott and Zhang's (d-1)-simplex construction.

* For every unknown i of the original mesh, sigma_i is a (d-1)-simplex of the
  original mesh that contains p_i. In 2-D it is the edge (i, j*), with j* the
  smallest vertex id among the neighbours of i. In 3-D it is the face (i, j, k),
  j < k, that is lexicographically smallest among the faces containing i.
* (Pi v)(p_i) = integral over sigma_i of psi_i v, where psi_i is the
  L2(sigma_i)-dual basis function of the vertex i: (6 lambda_i - 2) / |sigma_i|
  on an edge, (12 lambda_i - 3) / |sigma_i| on a triangle. It reproduces P1
  functions, as the section states.
* The integral is exact. sigma_i is clipped against every auxiliary simplex of
  sigma^(J) that it meets, and the integrand (a quadratic) is integrated exactly
  on each piece: Simpson on segments, and the edge-midpoint rule on the
  triangles of a fan of each polygon. A piece lying in a facet of an auxiliary
  simplex is met by the two simplices sharing that facet, and counts 1/2 from
  each; a facet on the boundary of the root box belongs to one simplex, and a piece
  there counts fully (this matters where boundary vertices are unknowns: the
  mixed and Neumann grids).

Pins: P1 reproduction (with the nodal values of a linear function on all
auxiliary vertices, the result equals its values at the original vertices,
1e-13); rows sum to 1 on the full auxiliary vertex set; on the unjittered
64 x 64 square whose diagonals all run lower-left to upper-right, the original
mesh is sigma^(J) and Pi = I exactly.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def sz_simplices(elems: np.ndarray, dof_vertices: np.ndarray, d: int) -> np.ndarray:
    """sigma_i for every unknown: (n, d) vertex ids with the unknown's vertex first."""
    elems = np.asarray(elems, dtype=np.int64)
    nv = int(elems.max()) + 1
    out = np.empty((len(dof_vertices), d), dtype=np.int64)
    if d == 2:
        best = np.full(nv, np.iinfo(np.int64).max)
        for a in range(3):
            for b in range(3):
                if a != b:
                    np.minimum.at(best, elems[:, a], elems[:, b])
        out[:, 0] = dof_vertices
        out[:, 1] = best[dof_vertices]
    else:
        vs, js, ks = [], [], []
        for a in range(4):
            others = [c for c in range(4) if c != a]
            for x in range(3):
                for y in range(x + 1, 3):
                    vs.append(elems[:, a])
                    js.append(np.minimum(elems[:, others[x]], elems[:, others[y]]))
                    ks.append(np.maximum(elems[:, others[x]], elems[:, others[y]]))
        vs, js, ks = np.concatenate(vs), np.concatenate(js), np.concatenate(ks)
        order = np.lexsort((ks, js, vs))      # by vertex, then (j, k) ascending
        vs, js, ks = vs[order], js[order], ks[order]
        first = np.ones(len(vs), dtype=bool)
        first[1:] = vs[1:] != vs[:-1]
        bj = np.full(nv, -1, dtype=np.int64)
        bk = np.full(nv, -1, dtype=np.int64)
        bj[vs[first]] = js[first]
        bk[vs[first]] = ks[first]
        out[:, 0] = dof_vertices
        out[:, 1] = bj[dof_vertices]
        out[:, 2] = bk[dof_vertices]
    return out


def _bary2(T, x):
    """Barycentric coordinates of points x (m, 2) in triangle T (3, 2)."""
    def cross(u, v):
        return u[..., 0] * v[..., 1] - u[..., 1] * v[..., 0]
    a2 = cross(T[1] - T[0], T[2] - T[0])
    l0 = cross(T[1] - x, T[2] - x) / a2
    l1 = cross(T[2] - x, T[0] - x) / a2
    l2 = cross(T[0] - x, T[1] - x) / a2
    return np.stack([l0, l1, l2], axis=-1)


def _det3(u, v, w):
    return (u[..., 0] * (v[..., 1] * w[..., 2] - v[..., 2] * w[..., 1])
            - u[..., 1] * (v[..., 0] * w[..., 2] - v[..., 2] * w[..., 0])
            + u[..., 2] * (v[..., 0] * w[..., 1] - v[..., 1] * w[..., 0]))


def _bary3(T, x):
    """Barycentric coordinates of points x (m, 3) in tetrahedron T (4, 3)."""
    vol = _det3(T[1] - T[0], T[2] - T[0], T[3] - T[0])
    out = []
    for m in range(4):
        Q = [T[k] if k != m else x for k in range(4)]
        out.append(_det3(Q[1] - Q[0], Q[2] - Q[0], Q[3] - Q[0]) / vol)
    return np.stack(out, axis=-1)


def _clip_interval(c0, c1):
    """t-interval in [0,1] where all affine functions c0 + t (c1 - c0) >= 0."""
    lo, hi = 0.0, 1.0
    for a, b in zip(c0, c1):
        s = b - a
        if s == 0.0:
            if a < 0.0:
                return None
            continue
        t = -a / s
        if s > 0:
            lo = max(lo, t)
        else:
            hi = min(hi, t)
    if hi <= lo:
        return None
    return lo, hi


def _clip_polygon(poly, coef):
    """Clip a convex polygon in (s, t) by half-planes c0 + s (c1-c0) + t (c2-c0) >= 0."""
    for c0, c1, c2 in coef:
        def f(p):
            return c0 + p[0] * (c1 - c0) + p[1] * (c2 - c0)
        out = []
        n = len(poly)
        for k in range(n):
            P = poly[k]
            Q = poly[(k + 1) % n]
            fp = f(P)
            fq = f(Q)
            if fp >= 0:
                out.append(P)
            if (fp > 0 and fq < 0) or (fp < 0 and fq > 0):
                t = fp / (fp - fq)
                out.append((P[0] + t * (Q[0] - P[0]), P[1] + t * (Q[1] - P[1])))
        poly = out
        if len(poly) < 3:
            return []
    return poly


class LeafIndex:
    """Leaf boxes of the closed tree and their simplices in sigma^(J)."""

    def __init__(self, tree, lmJ):
        self.tree = tree
        self.lm = lmJ
        self.box_simps = {}
        for s, bi in enumerate(lmJ.simp_box):
            self.box_simps.setdefault(lmJ.boxes[bi], []).append(s)

    def simplices_in_bbox(self, lo, hi):
        t = self.tree
        d = t.d
        out = []
        for k in range(1, t.J + 1):
            n = 1 << (k - 1)
            # closed boxes: a coordinate on a box boundary selects the boxes on both sides
            r0 = np.clip(np.ceil((lo - t.a) / t.L * n).astype(np.int64) - 1, 0, n - 1)
            r1 = np.clip(np.floor((hi - t.a) / t.L * n).astype(np.int64), 0, n - 1)
            for idx in np.ndindex(*tuple(int(r1[q] - r0[q] + 1) for q in range(d))):
                b = (k,) + tuple(int(r0[q] + idx[q]) for q in range(d))
                sl = self.box_simps.get(b)
                if sl is not None:
                    out.extend(sl)
        return out


def _facet_weight(lm, s, m):
    """Weight of a piece of sigma_i lying in the facet of simplex s opposite its vertex m: 1/2 for
    a facet shared by two simplices (each counts half), 1 for a facet on the boundary of the root
    box (one simplex has it)."""
    F = np.delete(lm.verts[lm.simp[s]], m, axis=0)
    top = 1 << lm.J
    on_root = any(np.all(F[:, q] == 0) or np.all(F[:, q] == top) for q in range(lm.d))
    return 1.0 if on_root else 0.5


def transfer(tree, meshes, coords, elems, dof_vertices, all_aux_vertices=False):
    """Pi as a sparse matrix (n_fine_unknowns x n_aux), n_aux = unknowns of sigma^(J).

    With ``all_aux_vertices`` the columns are every vertex of sigma^(J) (used by
    the P1-reproduction pin).
    """
    d = tree.d
    lm = meshes.level(tree.J)
    unit = tree.L * 2.0 ** (-tree.J)
    vphys = tree.a + lm.verts.astype(np.float64) * unit
    col_of_vert = np.arange(len(lm.verts)) if all_aux_vertices else lm.dof_of_vert
    ncols = len(lm.verts) if all_aux_vertices else lm.n
    leaf = LeafIndex(tree, lm)
    sig = sz_simplices(elems, dof_vertices, d)
    rows, cols, vals = [], [], []
    for i in range(len(dof_vertices)):
        P = coords[sig[i]]
        lo = P.min(axis=0)
        hi = P.max(axis=0)
        acc = {}
        for s in leaf.simplices_in_bbox(lo, hi):
            T = vphys[lm.simp[s]]
            if d == 2:
                lam = _bary2(T, P)                 # (2, 3): at t = 0 and t = 1
                iv = _clip_interval(lam[0], lam[1])
                if iv is None:
                    continue
                t0, t1 = iv
                on = [m for m in range(3) if lam[0][m] == 0.0 and lam[1][m] == 0.0]
                wgt = _facet_weight(lm, s, on[0]) if on else 1.0
                tm = 0.5 * (t0 + t1)
                for m in range(3):
                    def f(t):
                        return (4.0 - 6.0 * t) * (lam[0][m] + t * (lam[1][m] - lam[0][m]))
                    val = (t1 - t0) / 6.0 * (f(t0) + 4.0 * f(tm) + f(t1)) * wgt
                    c = col_of_vert[lm.simp[s][m]]
                    if c >= 0 and val != 0.0:
                        acc[c] = acc.get(c, 0.0) + val
            else:
                lam = _bary3(T, P)                 # (3, 4): at the face corners
                coef = [(lam[0][m], lam[1][m], lam[2][m]) for m in range(4)]
                poly = _clip_polygon([(0.0, 0.0), (1.0, 0.0), (0.0, 1.0)], coef)
                if len(poly) < 3:
                    continue
                on = [m for m in range(4) if coef[m][0] == 0.0 and coef[m][1] == 0.0 and coef[m][2] == 0.0]
                wgt = _facet_weight(lm, s, on[0]) if on else 1.0
                for m in range(4):
                    c = col_of_vert[lm.simp[s][m]]
                    if c < 0:
                        continue
                    c0, c1, c2 = coef[m]

                    def f(p):
                        return (18.0 - 24.0 * (p[0] + p[1])) * (c0 + p[0] * (c1 - c0) + p[1] * (c2 - c0))
                    val = 0.0
                    for q in range(1, len(poly) - 1):
                        A, B, C = poly[0], poly[q], poly[q + 1]
                        area = 0.5 * abs((B[0] - A[0]) * (C[1] - A[1]) - (B[1] - A[1]) * (C[0] - A[0]))
                        if area == 0.0:
                            continue
                        mab = ((A[0] + B[0]) / 2, (A[1] + B[1]) / 2)
                        mbc = ((B[0] + C[0]) / 2, (B[1] + C[1]) / 2)
                        mca = ((C[0] + A[0]) / 2, (C[1] + A[1]) / 2)
                        val += area * (f(mab) + f(mbc) + f(mca)) / 3.0
                    val *= wgt
                    if val != 0.0:
                        acc[c] = acc.get(c, 0.0) + val
        for c, v in acc.items():
            rows.append(i)
            cols.append(c)
            vals.append(v)
    Pi = sp.csr_matrix((vals, (rows, cols)), shape=(len(dof_vertices), ncols))
    Pi.sort_indices()
    return Pi
