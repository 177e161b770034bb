"""Dirichlet auxiliary grids on a general polygonal domain in 2-D (Section 3.4; oracle).

Section 3.4 keeps on level l only the simplices of sigma^(l) that lie in the domain:
T^D_l = {tau in sigma^(l) : tau in Omega}. The auxiliary space of level l is the P1 space on
T^D_l with homogeneous Dirichlet values on the boundary of their union.

Readings:
* Omega is the union of the closed fine triangles; "tau in Omega" is tau inside that closed set.
* Auxiliary vertex positions are the doubles x_k = a_k + L * (X_k * 2^-J) (integer coordinate
  X_k on the finest box grid, root corner a, root side L; IEEE round to nearest, the product
  first). Every predicate below is evaluated exactly on these doubles and on the mesh's own
  coordinates (rational arithmetic), so the kept set is unique.
* tau is kept iff no boundary edge of the mesh (an edge of a single triangle) meets the
  interior of tau, and the interior point (2 v0 + v1 + v2) / 4 of tau lies in a closed fine
  triangle. The first condition puts the connected set int(tau) entirely inside Omega or
  entirely outside its closure, and the point decides which.
* A closed segment and an open triangle are disjoint iff the line of one edge of the
  triangle, or the segment's own line, separates them weakly (separating axes of two convex
  polygons).
* Unknowns of level l: vertices inside the root box whose whole star in sigma^(l) is kept. A
  dropped simplex therefore has no unknown among its vertices, and the assembly, the nodal
  P_l and the Scott-Zhang transfer need no other change.

Mixed Dirichlet/Neumann auxiliary grids (the remark of Section 3.5; ``Domain(..., dirichlet)``,
``mixed``): T^M_l = {tau in sigma^(l) : tau meets Omega and tau does not meet Gamma_D}, with
natural (Neumann) conditions on the auxiliary boundary except next to Gamma_D. Readings:
* Gamma_D is the union of the mesh's boundary edges whose two vertices are Dirichlet vertices.
* "Meets" is between closed sets. A closed triangle meets Omega iff a boundary edge of the
  mesh meets it, or (no boundary edge meets it, so it lies entirely inside or entirely
  outside) its interior point (2 v0 + v1 + v2) / 4 lies in Omega.
* A closed segment and a closed triangle are disjoint iff the line of one edge of the triangle
  has both segment ends strictly outside, or the segment's line has the three triangle
  vertices strictly on one side.
* Essential (Dirichlet) conditions at the "neighbours of boxes meeting Gamma_D": the vertices
  of every simplex of sigma^(l) that meets Gamma_D. Every other vertex of a kept simplex is an
  unknown, on the root box boundary too (natural conditions there).
* The near-boundary correction of Algorithm 3 is not part of this option.

Pins: the 64 x 64 square keeps every simplex and gives the box hierarchy unchanged; on an
L-shaped domain whose re-entrant corner sits on a dyadic line, the kept simplices are exactly
those of sigma^(l) outside the removed quadrant; kept simplices pass a dense point-sampling
check against the mesh; the union grows with the level and stays inside the domain; the
Galerkin identity still holds.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def boundary_edges(elems):
    """Edges (sorted vertex pairs) that belong to exactly one triangle."""
    e = np.sort(np.concatenate([elems[:, [0, 1]], elems[:, [1, 2]], elems[:, [2, 0]]]), axis=1)
    u, c = np.unique(e, axis=0, return_counts=True)
    return u[c == 1]


def boundary_vertices(elems, n_vertices):
    """Vertices on a boundary edge (the natural Dirichlet set of a general domain)."""
    m = np.zeros(n_vertices, dtype=bool)
    m[boundary_edges(np.asarray(elems)).ravel()] = True
    return m


def _orient(a, b, c):
    """Sign of the signed area of (a, b, c), exact on Fraction coordinates."""
    d = (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])
    return (d > 0) - (d < 0)


class Domain:
    """The closed union of a 2-D mesh's triangles, with exact membership tests."""

    def __init__(self, coords, elems, dirichlet=None):
        coords = np.asarray(coords, dtype=np.float64)
        elems = np.asarray(elems, dtype=np.int64)
        if coords.shape[1] != 2:
            raise ValueError("general domains are 2-D")
        self.coords = coords
        self.F = [(Fraction(float(x)), Fraction(float(y))) for x, y in coords]
        self.bedges = boundary_edges(elems)
        self.tris = elems
        self.ebox = np.stack([coords[self.bedges].min(axis=1), coords[self.bedges].max(axis=1)], axis=1)
        self.tbox = np.stack([coords[elems].min(axis=1), coords[elems].max(axis=1)], axis=1)
        # Gamma_D: boundary edges with both vertices Dirichlet (mixed grids)
        self.gd = np.zeros((0, 2), dtype=np.int64)
        if dirichlet is not None:
            m = np.asarray(dirichlet, dtype=bool)
            self.gd = self.bedges[m[self.bedges[:, 0]] & m[self.bedges[:, 1]]]
        self.gbox = (np.stack([coords[self.gd].min(axis=1), coords[self.gd].max(axis=1)], axis=1)
                     if len(self.gd) else np.zeros((0, 2, 2)))

    def aux_point(self, tree, X):
        """Double coordinates of an integer point of the finest box grid (units 2^-J of L)."""
        s = 2.0 ** (-tree.J)
        return np.array([tree.a[k] + tree.L * (float(X[k]) * s) for k in range(2)])

    def _segment_meets_open(self, p, q, T):
        for i in range(3):
            a, b, c = T[i], T[(i + 1) % 3], T[(i + 2) % 3]
            side = _orient(a, b, c)     # the triangle's interior side of edge (a, b)
            if _orient(a, b, p) * side <= 0 and _orient(a, b, q) * side <= 0:
                return False
        o = [_orient(p, q, v) for v in T]
        if all(x >= 0 for x in o) or all(x <= 0 for x in o):
            return False
        return True

    @staticmethod
    def _segment_meets_closed(p, q, T):
        for i in range(3):
            a, b, c = T[i], T[(i + 1) % 3], T[(i + 2) % 3]
            side = _orient(a, b, c)
            if _orient(a, b, p) * side < 0 and _orient(a, b, q) * side < 0:
                return False
        o = [_orient(p, q, v) for v in T]
        if all(x > 0 for x in o) or all(x < 0 for x in o):
            return False
        return True

    def _edges_meet_closed(self, edges, boxes, T, lo, hi):
        if not len(edges):
            return False
        cand = np.nonzero((boxes[:, 0, 0] <= hi[0]) & (lo[0] <= boxes[:, 1, 0]) &
                          (boxes[:, 0, 1] <= hi[1]) & (lo[1] <= boxes[:, 1, 1]))[0]
        return any(self._segment_meets_closed(self.F[edges[e][0]], self.F[edges[e][1]], T) for e in cand)

    def mixed(self, tree, Xs):
        """(kept, meets Gamma_D) of the auxiliary triangle with integer vertices Xs in the mixed
        grids: kept iff it meets Omega and not Gamma_D (closed sets)."""
        pts = [self.aux_point(tree, X) for X in Xs]
        T = [(Fraction(float(p[0])), Fraction(float(p[1]))) for p in pts]
        lo = np.min(pts, axis=0)
        hi = np.max(pts, axis=0)
        if self._edges_meet_closed(self.gd, self.gbox, T, lo, hi):
            return False, True
        if self._edges_meet_closed(self.bedges, self.ebox, T, lo, hi):
            return True, False
        X = np.asarray(Xs, dtype=np.int64)
        inner = 2 * X[0] + X[1] + X[2]
        s = 2.0 ** (-(tree.J + 2))
        c = np.array([tree.a[k] + tree.L * (float(inner[k]) * s) for k in range(2)])
        return self.contains_point(c), False

    def contains_point(self, x):
        """x (two doubles) in the closed union of the triangles."""
        P = (Fraction(float(x[0])), Fraction(float(x[1])))
        cand = np.nonzero((self.tbox[:, 0, 0] <= x[0]) & (x[0] <= self.tbox[:, 1, 0]) &
                          (self.tbox[:, 0, 1] <= x[1]) & (x[1] <= self.tbox[:, 1, 1]))[0]
        for t in cand:
            a, b, c = (self.F[v] for v in self.tris[t])
            s = _orient(a, b, c)
            if _orient(a, b, P) * s >= 0 and _orient(b, c, P) * s >= 0 and _orient(c, a, P) * s >= 0:
                return True
        return False

    def keeps(self, tree, Xs):
        """Is the auxiliary triangle with integer vertices Xs (3 x 2) inside the domain?"""
        pts = [self.aux_point(tree, X) for X in Xs]
        T = [(Fraction(float(p[0])), Fraction(float(p[1]))) for p in pts]
        lo = np.min(pts, axis=0)
        hi = np.max(pts, axis=0)
        cand = np.nonzero((self.ebox[:, 0, 0] <= hi[0]) & (lo[0] <= self.ebox[:, 1, 0]) &
                          (self.ebox[:, 0, 1] <= hi[1]) & (lo[1] <= self.ebox[:, 1, 1]))[0]
        for e in cand:
            p, q = self.F[self.bedges[e][0]], self.F[self.bedges[e][1]]
            if self._segment_meets_open(p, q, T):
                return False
        X = np.asarray(Xs, dtype=np.int64)
        inner = 2 * X[0] + X[1] + X[2]                     # 4 times an interior point, integer
        s = 2.0 ** (-(tree.J + 2))
        c = np.array([tree.a[k] + tree.L * (float(inner[k]) * s) for k in range(2)])
        return self.contains_point(c)
