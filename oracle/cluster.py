"""Barycenters, regular box tree, cluster tree and closure (oracle).

Section 3.1 (clustering and auxiliary box trees) and Section 3.2 (closure of the
auxiliary box tree). Readings taken where the paper is silent or ambiguous:

* barycenter xi_i = ((p_a + p_b) + p_c) / 3 in 2-D and
  (((p_a + p_b) + p_c) + p_d) / 4 in 3-D, evaluated left to right in IEEE
  double precision with no fused multiply-add. This fixes the integer keys.
* The root box B^1 is the smallest square (cube) anchored at the minimum corner
  a of the vertex coordinates, with side L = the largest bounding-box extent.
  Boxes are half-open. An integer key per axis is
  k = min(floor(((xi - a) / L) * 2^D), 2^D - 1), with D = 30 in 2-D and D = 20
  in 3-D. The level-l box (root level 1) of xi is given by the top (l - 1) bits
  of each axis key. A barycenter on a split line therefore goes to the upper
  child.
* A box is refined iff its cluster has more than n_min indices and its level is
  at most D. Section 3.1 fixes n_min = 3 in 2-D (the text's rule; the figure
  caption says "less than three"). n_min = 7 = 3! + 1 is used in 3-D, where the
  paper is silent.
* Closure: the closed refined set R is the least superset of R_0 such that no
  leaf at level l touches a refined box at level l + 1. "Touches" means along a
  segment of positive length in 2-D, and along a face or an edge in 3-D. This
  is the condition "at most one hanging node per edge". It is computed twice:
  once by a worklist, and once by the paper's level-by-level Mark / Retain /
  Close / Refine procedure. The tests assert that both give the same set.

Boxes are tuples (level, i_0, ..., i_{d-1}), with 0 <= i < 2^(level-1).

Pins (tests/test_oracle_cluster.py):
* brute-force recount of every cluster on small point sets;
* leaves hold at most n_min indices, and every refined box holds more (or was
  forced by closure);
* depth bound of the Section 3.1 lemma;
* brute-force balance check, and minimality (every closure box is forced);
* worklist == literal procedure;
* worked examples: the 64 x 64 jittered square gives the uniform level-7 tree,
  and the 3-D Kuhn cube with n_min = 7 gives the uniform tree of matching depth.
"""
from __future__ import annotations

import itertools

import numpy as np

KEY_BITS = {2: 30, 3: 20}


def default_n_min(d: int) -> int:
    return {2: 3, 3: 7}[d]


# ----------------------------------------------------------------------------
# barycenters and keys (Section 3.1)
# ----------------------------------------------------------------------------


def barycenters(coords: np.ndarray, elems: np.ndarray) -> np.ndarray:
    P = coords[np.asarray(elems)]
    s = P[:, 0] + P[:, 1]
    for k in range(2, P.shape[1]):
        s = s + P[:, k]
    return s / float(P.shape[1])


def root_box(coords: np.ndarray):
    a = coords.min(axis=0)
    L = float((coords.max(axis=0) - a).max())
    return a, L


def axis_keys(xi: np.ndarray, a: np.ndarray, L: float, d: int) -> np.ndarray:
    D = KEY_BITS[d]
    t = ((xi - a) / L) * float(2 ** D)
    k = np.floor(t)
    k = np.clip(k, 0, 2 ** D - 1)
    return k.astype(np.int64)


def box_of(keys: np.ndarray, level: int, d: int) -> np.ndarray:
    """Integer box indices (N, d) at ``level`` (root = 1) of each key."""
    return keys >> (KEY_BITS[d] - (level - 1))


# ----------------------------------------------------------------------------
# cluster counts and the unclosed refined set R_0
# ----------------------------------------------------------------------------


def cluster_counts(keys: np.ndarray, level: int, d: int) -> dict:
    idx = box_of(keys, level, d)
    boxes, counts = np.unique(idx, axis=0, return_counts=True)
    return {(level,) + tuple(int(v) for v in b): int(c) for b, c in zip(boxes, counts)}


def refined_by_count(keys: np.ndarray, d: int, n_min: int) -> set:
    """R_0: boxes whose cluster has more than n_min barycenters (level <= D)."""
    D = KEY_BITS[d]
    R0 = set()
    for level in range(1, D + 1):
        cnt = cluster_counts(keys, level, d)
        sel = [b for b, c in cnt.items() if c > n_min]
        if not sel:
            break
        R0.update(sel)
    return R0


# ----------------------------------------------------------------------------
# tree helpers
# ----------------------------------------------------------------------------


def touch_offsets(d: int):
    """Same-level offsets of boxes that share a facet (2-D: an edge; 3-D: a face) or a 3-D edge."""
    offs = []
    for o in itertools.product((-1, 0, 1), repeat=d):
        nz = sum(1 for v in o if v != 0)
        if nz == 1 or (d == 3 and nz == 2):
            offs.append(o)
    return offs


def children(b):
    lev = b[0]
    d = len(b) - 1
    return [(lev + 1,) + tuple(2 * b[1 + k] + a[k] for k in range(d))
            for a in itertools.product((0, 1), repeat=d)]


def parent(b):
    return (b[0] - 1,) + tuple(v >> 1 for v in b[1:])


def valid(b):
    n = 1 << (b[0] - 1)
    return all(0 <= v < n for v in b[1:])


def in_tree(b, R):
    return b[0] == 1 or parent(b) in R


def touching_children(b, o):
    """Children of the neighbour b + o that touch b (facet or edge contact)."""
    d = len(b) - 1
    nb = tuple(b[1 + k] + o[k] for k in range(d))
    choices = []
    for k in range(d):
        if o[k] == 1:
            choices.append((0,))
        elif o[k] == -1:
            choices.append((1,))
        else:
            choices.append((0, 1))
    return [(b[0] + 1,) + tuple(2 * nb[k] + a[k] for k in range(d)) for a in itertools.product(*choices)]


def violates(b, R, offs) -> bool:
    """A leaf b violates the closure rule if it touches a refined box one level finer."""
    d = len(b) - 1
    for o in offs:
        nb = (b[0],) + tuple(b[1 + k] + o[k] for k in range(d))
        if not valid(nb) or nb not in R:
            continue
        for c in touching_children(b, o):
            if c in R:
                return True
    return False


def leaves(R, d):
    root = (1,) + (0,) * d
    if root not in R:
        return [root]
    out = []
    for b in R:
        for c in children(b):
            if c not in R:
                out.append(c)
    return out


# ----------------------------------------------------------------------------
# closure, form 1: least fixed point by a worklist
# ----------------------------------------------------------------------------


def close_worklist(R0: set, d: int) -> set:
    offs = touch_offsets(d)
    R = set(R0)
    stack = leaves(R, d)
    while stack:
        b = stack.pop()
        if b in R or not in_tree(b, R):
            continue
        if violates(b, R, offs):
            R.add(b)
            stack.extend(children(b))
            if b[0] >= 2:
                for o in offs:
                    q = (b[0],) + tuple(b[1 + k] + o[k] for k in range(d))
                    if not valid(q):
                        continue
                    p = parent(q)
                    if p not in R and in_tree(p, R):
                        stack.append(p)
    return R


# ----------------------------------------------------------------------------
# closure, form 2: the paper's level-by-level Mark / Retain / Close / Refine
# ----------------------------------------------------------------------------


def close_literal(keys: np.ndarray, d: int, n_min: int) -> set:
    D = KEY_BITS[d]
    offs = touch_offsets(d)
    R = set()
    frontier = [(1,) + (0,) * d]
    level = 1
    while frontier:
        cnt = cluster_counts(keys, level, d)
        # (Mark) / (Retain)
        marked = {b for b in frontier if cnt.get(b, 0) > n_min and level <= D}
        # (Close): lists L^(j), j = level-1, ..., 1
        newly = set(marked)
        allm = set(marked)
        while newly:
            lst = set()
            for b in newly:
                for o in offs:
                    q = (b[0],) + tuple(b[1 + k] + o[k] for k in range(d))
                    if not valid(q) or q[0] < 2:
                        continue
                    p = parent(q)
                    if p not in R and p not in allm and in_tree(p, R):
                        lst.add(p)
            newly = lst
            allm |= lst
        # (Refine)
        R |= allm
        frontier = [c for b in marked for c in children(b)]
        level += 1
    return R


# ----------------------------------------------------------------------------
# convenience
# ----------------------------------------------------------------------------


class BoxTree:
    """The closed box tree of one mesh."""

    def __init__(self, coords, elems, n_min=None, check_literal=False):
        coords = np.asarray(coords, dtype=np.float64)
        self.d = coords.shape[1]
        self.n_min = default_n_min(self.d) if n_min in (None, 0) else int(n_min)
        self.xi = barycenters(coords, elems)
        self.a, self.L = root_box(coords)
        self.keys = axis_keys(self.xi, self.a, self.L, self.d)
        self.R0 = refined_by_count(self.keys, self.d, self.n_min)
        self.R = close_worklist(self.R0, self.d)
        if check_literal:
            lit = close_literal(self.keys, self.d, self.n_min)
            assert lit == self.R, "closure: worklist and literal procedure disagree"
        self.leaves = sorted(leaves(self.R, self.d))
        self.J = max(b[0] for b in self.leaves)

    def leaf_kappa(self, kappa: np.ndarray) -> dict:
        """kappa~ per leaf: mean of kappa over the leaf's cluster.

        An empty cluster takes the mean of its nearest ancestor with a non-empty
        cluster.
        """
        d = self.d
        mult = 1 << (KEY_BITS[d] + 1)   # box indices < 2^KEY_BITS: packed codes stay below 2^63
        sums = {}
        levels = sorted({b[0] for b in self.leaves})
        needed = set(range(1, self.J + 1))
        for lev in needed:
            idx = box_of(self.keys, lev, d)
            codes = idx[:, 0].copy()
            for k in range(1, d):
                codes = codes * mult + idx[:, k]
            u, inv = np.unique(codes, return_inverse=True)
            s = np.zeros(len(u))
            np.add.at(s, inv, kappa)
            c = np.bincount(inv, minlength=len(u))
            for j in range(len(u)):
                sums[(lev, int(u[j]))] = (float(s[j]), int(c[j]))
        del levels

        def code(b):
            v = b[1]
            for k in range(2, d + 1):
                v = v * mult + b[k]
            return v

        out = {}
        for b in self.leaves:
            q = b
            while True:
                s_c = sums.get((q[0], code(q)))
                if s_c is not None and s_c[1] > 0:
                    out[b] = s_c[0] / s_c[1]
                    break
                q = parent(q)
        return out
