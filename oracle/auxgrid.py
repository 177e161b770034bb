"""Conforming nested auxiliary triangulations sigma^(l) of the closed box tree (oracle).

Section 3.3 (construction of a conforming auxiliary grid hierarchy) and
Section 3.4 (Dirichlet auxiliary grids). The hanging-node templates are figures
that are missing from the available text. The reading used is as follows.

Coordinates are integers in units of L * 2^(-J), where J is the deepest leaf
level. A level-k box has side S = 2^(J - k + 1) units.

* Active boxes of sigma^(l): the tree boxes of level l (refined or not),
  together with the leaves of level < l.
* A box of level k < l is a fan box if one of its same-level neighbours that
  touch it (2-D: across an edge; 3-D: across a face or an edge) is refined. Then
  that neighbour's children put a vertex at the shared edge midpoint (and, in
  3-D, at the shared face centre).
* 2-D, non-fan box: the two Kuhn triangles {x >= y} = (LL, LR, UR) and
  {y >= x} = (LL, UL, UR), split along the lower-left to upper-right diagonal.
  Fan box: the centre c, and for each edge in counter-clockwise order starting at
  the bottom, the triangles (v0, m, c), (m, v1, c) if the edge carries the
  midpoint m, else (v0, v1, c). This gives 4 + k triangles, every angle is 45 or
  90 degrees (Section 3.3 states a minimum angle of 45 degrees), and the fan is
  the newest-vertex bisection of the two diagonal triangles, so the levels are
  nested.
* 3-D, non-fan box: six Kuhn tetrahedra {x_p0 >= x_p1 >= x_p2}, with vertices
  0, e_p0, e_p0 + e_p1, (1,1,1), for the permutations p in lexicographic order.
  Fan box: a cone from the cube centre over a triangulation of each face, taking
  faces in the order x-, x+, y-, y+, z-, z+. A face whose centre is a vertex
  (face neighbour refined) is cut into 4 sub-squares, each split into 2 Kuhn
  triangles. Otherwise, a face with a vertex at some edge midpoint gets a fan
  around its centre. Otherwise it is split into 2 Kuhn triangles. The Kuhn
  triangulation is nested under dyadic refinement, and the cone over the 12 Kuhn
  face triangles is the 6 Kuhn tetrahedra bisected at the cube centre.
* Dirichlet auxiliary grid (Section 3.4): for a domain equal to the root box,
  every simplex lies in the closure of Omega. The unknowns are the vertices
  strictly inside the root box.
* Numbering: the vertices of a level are sorted in Morton order of their integer
  coordinates (axis 0 the most significant bit in each group). The unknowns keep
  that order. Simplices are listed by box (Morton order of the box's lower
  corner), then by template position.

Pins (tests/test_oracle_auxgrid.py): total area/volume equals the root box's;
every interior facet is shared by exactly two simplices and no vertex lies inside
a facet (conformity); each level-l simplex lies in exactly one level-(l-1)
simplex (nestedness); 2-D minimum angle is exactly 45 degrees; the jittered
64 x 64 square gives the uniform 64 x 64 Kuhn grid at the finest level.
"""
from __future__ import annotations

import itertools

import numpy as np

from .cluster import children, in_tree, touch_offsets, valid

PERMS = {2: [(0, 1), (1, 0)],
         3: [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]}


def morton_order(X: np.ndarray) -> np.ndarray:
    """argsort of integer points (n, d) in Morton order (axis 0 most significant per bit group)."""
    X = np.asarray(X, dtype=np.int64)
    n, d = X.shape
    if n == 0:
        return np.zeros(0, dtype=np.int64)
    nbits = max(1, int(X.max()).bit_length())
    nw = (nbits * d + 62) // 63
    words = [np.zeros(n, dtype=np.uint64) for _ in range(nw)]  # least significant first
    for b in range(nbits):
        for k in range(d):
            bit = ((X[:, k] >> b) & 1).astype(np.uint64)
            slot = b * d + (d - 1 - k)
            words[slot // 63] |= bit << np.uint64(slot % 63)
    return np.lexsort(tuple(words))


class LevelMesh:
    """sigma^(l): integer vertices, simplices and unknown numbering of one level."""

    def __init__(self, verts, simp, simp_box, simp_tmpl, boxes, box_fan, J, d, kept=None, touch=None):
        self.verts = verts            # (nv, d) int64, Morton order
        self.simp = simp              # (ns, d+1) int64 into verts
        self.simp_box = simp_box      # (ns,) index into boxes
        self.simp_tmpl = simp_tmpl    # (ns,) template index (Kuhn permutation for non-fan boxes)
        self.boxes = boxes            # list of active boxes (Morton order of lower corner)
        self.box_fan = box_fan        # (nb,) bool
        self.J = J
        self.d = d
        top = 1 << J
        self.interior = np.all((verts > 0) & (verts < top), axis=1)
        # general domain (Section 3.4): only the kept simplices form the grid, and an unknown
        # needs its whole star kept
        self.kept = np.ones(len(simp), dtype=bool) if kept is None else np.asarray(kept, dtype=bool)
        if touch is not None:
            # mixed grids: every vertex of a kept simplex, except the vertices of simplices that
            # meet Gamma_D (essential conditions there; natural ones elsewhere, root box included)
            inkept = np.zeros(len(verts), dtype=bool)
            inkept[simp[self.kept].ravel()] = True
            bad = np.zeros(len(verts), dtype=bool)
            bad[simp[np.asarray(touch, dtype=bool)].ravel()] = True
            self.interior = inkept & ~bad
        elif kept is not None:
            bad = np.zeros(len(verts), dtype=bool)
            bad[simp[~self.kept].ravel()] = True
            self.interior &= ~bad
        self.dof_of_vert = np.full(len(verts), -1, dtype=np.int64)
        self.dof_vert = np.nonzero(self.interior)[0]
        self.dof_of_vert[self.dof_vert] = np.arange(len(self.dof_vert))
        self.n = len(self.dof_vert)


class AuxMeshes:
    """All level meshes sigma^(1..J) of a closed box tree."""

    def __init__(self, tree, domain=None, mixed=False):
        self.mixed = mixed            # mixed Dirichlet/Neumann grids (domain must be given)
        self.tree = tree
        self.d = tree.d
        self.J = tree.J
        self.R = tree.R
        self.offs = touch_offsets(self.d)
        self.domain = domain          # oracle.domain.Domain, or None for the root box
        self._cache = {}

    # -- geometry ------------------------------------------------------------
    def side(self, b):
        return 1 << (self.J - b[0] + 1)

    def corner(self, b):
        s = self.side(b)
        return np.array([v * s for v in b[1:]], dtype=np.int64)

    def is_leaf(self, b):
        return b not in self.R

    def is_fan(self, b, level):
        if b[0] >= level:
            return False
        d = self.d
        for o in self.offs:
            nb = (b[0],) + tuple(b[1 + k] + o[k] for k in range(d))
            if valid(nb) and nb in self.R:
                return True
        return False

    def active_boxes(self, level):
        d = self.d
        out = []
        root = (1,) + (0,) * d
        stack = [root]
        while stack:
            b = stack.pop()
            if b[0] == level or b not in self.R:
                out.append(b)
            else:
                stack.extend(children(b))
        corners = np.array([self.corner(b) for b in out], dtype=np.int64).reshape(len(out), d)
        order = morton_order(corners)
        return [out[i] for i in order]

    # -- templates -----------------------------------------------------------
    def kuhn(self, b):
        d = self.d
        c = self.corner(b)
        S = self.side(b)
        e = np.eye(d, dtype=np.int64) * S
        out = []
        for p in PERMS[d]:
            v = [c.copy()]
            cur = c.copy()
            for k in range(d - 1):
                cur = cur + e[p[k]]
                v.append(cur.copy())
            v.append(c + S)
            out.append(np.array(v))
        return out

    def fan2(self, b):
        c0 = self.corner(b)
        S = self.side(b)
        H = S // 2
        LL = c0
        LR = c0 + [S, 0]
        UR = c0 + [S, S]
        UL = c0 + [0, S]
        C = c0 + [H, H]
        edges = [(LL, LR, (0, -1)), (LR, UR, (1, 0)), (UR, UL, (0, 1)), (UL, LL, (-1, 0))]
        out = []
        for v0, v1, o in edges:
            nb = (b[0], b[1] + o[0], b[2] + o[1])
            if valid(nb) and nb in self.R:
                m = (v0 + v1) // 2
                out.append(np.array([v0, m, C]))
                out.append(np.array([m, v1, C]))
            else:
                out.append(np.array([v0, v1, C]))
        return out

    def fan3(self, b):
        c0 = self.corner(b)
        S = self.side(b)
        H = S // 2
        C = c0 + H
        out = []
        bi = np.array(b[1:])
        for ax in range(3):
            u, v = [k for k in range(3) if k != ax]
            for s in (0, 1):
                of = np.zeros(3, np.int64)
                of[ax] = 2 * s - 1
                base = c0.copy()
                base[ax] += s * S

                def P(al2, be2):  # al2, be2 in half-units of the face (0, 1, 2)
                    q = base.copy()
                    q[u] += al2 * H
                    q[v] += be2 * H
                    return q

                def inR(off):
                    nb = (b[0],) + tuple(int(x) for x in bi + off)
                    return valid(nb) and nb in self.R

                eu = np.zeros(3, np.int64)
                eu[u] = 1
                ev = np.zeros(3, np.int64)
                ev[v] = 1
                # edges CCW in (u, v): bottom, right, top, left
                fedges = [((0, 0), (2, 0), -ev), ((2, 0), (2, 2), eu), ((2, 2), (0, 2), ev),
                          ((0, 2), (0, 0), -eu)]
                mids = [inR(of) or inR(ip) or inR(of + ip) for _, _, ip in fedges]
                tris = []
                if inR(of):
                    for be0 in (0, 1):
                        for al0 in (0, 1):
                            p00 = P(al0, be0)
                            p10 = P(al0 + 1, be0)
                            p11 = P(al0 + 1, be0 + 1)
                            p01 = P(al0, be0 + 1)
                            tris.append((p00, p10, p11))
                            tris.append((p00, p01, p11))
                elif any(mids):
                    FC = P(1, 1)
                    for (a0, a1, _), m in zip(fedges, mids):
                        p0 = P(*a0)
                        p1 = P(*a1)
                        if m:
                            pm = (p0 + p1) // 2
                            tris.append((p0, pm, FC))
                            tris.append((pm, p1, FC))
                        else:
                            tris.append((p0, p1, FC))
                else:
                    tris.append((P(0, 0), P(2, 0), P(2, 2)))
                    tris.append((P(0, 0), P(0, 2), P(2, 2)))
                for t in tris:
                    out.append(np.array([t[0], t[1], t[2], C]))
        return out

    # -- level mesh ----------------------------------------------------------
    def level(self, level) -> LevelMesh:
        if level in self._cache:
            return self._cache[level]
        d = self.d
        boxes = self.active_boxes(level)
        simps, sbox, stmpl, fan = [], [], [], []
        for bi, b in enumerate(boxes):
            f = self.is_fan(b, level)
            fan.append(f)
            if f:
                ts = self.fan2(b) if d == 2 else self.fan3(b)
            else:
                ts = self.kuhn(b)
            for t, s in enumerate(ts):
                simps.append(s)
                sbox.append(bi)
                stmpl.append(t)
        P = np.array(simps, dtype=np.int64)             # (ns, d+1, d)
        flat = P.reshape(-1, d)
        uniq, inv = np.unique(flat, axis=0, return_inverse=True)
        order = morton_order(uniq)
        rank = np.empty(len(order), dtype=np.int64)
        rank[order] = np.arange(len(order))
        verts = uniq[order]
        simp = rank[inv.ravel()].reshape(len(simps), d + 1)
        kept = touch = None
        if self.domain is not None and self.mixed:
            kt = np.array([self.domain.mixed(self.tree, verts[t]) for t in simp], dtype=bool).reshape(-1, 2)
            kept, touch = kt[:, 0], kt[:, 1]
        elif self.domain is not None:
            kept = np.array([self.domain.keeps(self.tree, verts[t]) for t in simp], dtype=bool)
        lm = LevelMesh(verts, simp, np.array(sbox), np.array(stmpl), boxes, np.array(fan), self.J, d, kept,
                       touch)
        self._cache[level] = lm
        return lm

    def tree_boxes_at(self, level):
        """All tree boxes of a level (root, or children of refined boxes)."""
        if level == 1:
            return [(1,) + (0,) * self.d]
        return [c for b in self.R if b[0] == level - 1 for c in children(b)]

    def contains_active(self, b, level):
        return in_tree(b, self.R) and (b[0] == level or (b[0] < level and b not in self.R))


def kuhn_child_inside(a, sigma, pi) -> bool:
    """Is Kuhn simplex sigma of child a (a in {0,1}^d) inside Kuhn simplex pi of the parent?"""
    for m in range(len(pi) - 1):
        p, q = pi[m], pi[m + 1]
        if a[p] > a[q]:
            continue
        if a[p] < a[q]:
            return False
        if sigma.index(p) > sigma.index(q):
            return False
    return True


def kuhn_means(tree, leaf_kappa: dict) -> dict:
    """Area-weighted mean coefficient of every Kuhn simplex of every box in the tree.

    Leaves: all simplices carry the leaf value kappa~. Refined boxes: the mean of
    the 2^d child Kuhn simplices inside (each 1/2^d of the parent simplex).
    """
    d = tree.d
    perms = PERMS[d]
    inside = {}
    for t, pi in enumerate(perms):
        lst = []
        for a in itertools.product((0, 1), repeat=d):
            ci = int(sum(a[k] << (d - 1 - k) for k in range(d)))
            for s, sg in enumerate(perms):
                if kuhn_child_inside(a, sg, pi):
                    lst.append((ci, s))
        assert len(lst) == 2 ** d
        inside[t] = lst
    w = {}
    for b, k in leaf_kappa.items():
        w[b] = np.full(len(perms), k)
    for b in sorted(tree.R, key=lambda x: -x[0]):
        ch = children(b)  # order: itertools.product over (0,1)^d, axis 0 most significant
        vals = np.empty(len(perms))
        for t in range(len(perms)):
            s = 0.0
            for ci, sg in inside[t]:
                s += w[ch[ci]][sg]
            vals[t] = s / 2 ** d
        w[b] = vals
    return w
