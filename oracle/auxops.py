"""Auxiliary stiffness matrices A_l and prolongations P_l (oracle).

Section 4.1: the auxiliary space V = V_J carries the bilinear form of the model
problem. In Section 2.3, A_l is the restriction of A to V_l. Section 5.1 sets up
the stiffness matrices A^l and the prolongation matrices P^l as one would on a
general grid hierarchy.

Readings:
* Coefficient on the auxiliary grids. Each leaf box b carries kappa~_b, the mean
  of kappa over its cluster. An empty cluster takes the value of the nearest
  ancestor whose cluster is not empty.
* A_J is the P1 stiffness matrix on sigma^(J) with kappa~.
* A_l for l < J is the P1 stiffness matrix on sigma^(l), with each simplex
  carrying the area-weighted mean of kappa~ over the finest simplices inside it.
  Coarse gradients are constant on coarse simplices, so this equals the Galerkin
  product P^T A_(l+1) P. The tests assert that identity.
* Element matrices come from integer coordinates, in units of half the side of
  the simplex's box. The cofactor vectors a_i are integers, and
  K_ij = kappa * h^(d-2) * (a_i . a_j) / (d! |det|).
  A coupling that vanishes geometrically (a right angle in 2-D, a right
  dihedral angle in 3-D) is therefore exactly 0.0. Every auxiliary simplex is
  non-obtuse, so an assembled off-diagonal entry is 0 exactly when every
  contribution is 0. Such entries are dropped, and the sparsity pattern does not
  depend on rounding.
* P_l is nodal P1 interpolation from sigma^(l-1) to sigma^(l). It is computed by
  point location with exact integer barycentric coordinates. Every new vertex is
  an edge midpoint, so the weights are 1 or 1/2.

Pins: Galerkin identity (1e-13); P_l reproduces linear functions exactly; P_l
has the midpoint structure; the uniform hierarchy of the 64 x 64 square gives
the textbook 5-point matrices on (2^(l-1) - 1)^2 grids.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from .auxgrid import kuhn_means


def _adjugate_rows(E):
    """Integer cofactor vectors a_0..a_d (rows) of simplices with edge matrix E (ns, d, d) rows=edges."""
    ns, d, _ = E.shape
    M = np.transpose(E, (0, 2, 1))  # columns = edges
    if d == 2:
        adj = np.empty_like(M)
        adj[:, 0, 0] = M[:, 1, 1]
        adj[:, 0, 1] = -M[:, 0, 1]
        adj[:, 1, 0] = -M[:, 1, 0]
        adj[:, 1, 1] = M[:, 0, 0]
        det = M[:, 0, 0] * M[:, 1, 1] - M[:, 0, 1] * M[:, 1, 0]
    else:
        adj = np.empty_like(M)
        for i in range(3):
            for j in range(3):
                r = [k for k in range(3) if k != j]
                c = [k for k in range(3) if k != i]
                minor = M[:, r[0], c[0]] * M[:, r[1], c[1]] - M[:, r[0], c[1]] * M[:, r[1], c[0]]
                adj[:, i, j] = (-1) ** (i + j) * minor
        det = (M[:, 0, 0] * (M[:, 1, 1] * M[:, 2, 2] - M[:, 1, 2] * M[:, 2, 1])
               - M[:, 0, 1] * (M[:, 1, 0] * M[:, 2, 2] - M[:, 1, 2] * M[:, 2, 0])
               + M[:, 0, 2] * (M[:, 1, 0] * M[:, 2, 1] - M[:, 1, 1] * M[:, 2, 0]))
    a = np.empty((ns, d + 1, d), dtype=np.int64)
    a[:, 1:, :] = adj             # rows of adj(M) = det * grad lambda_{1..d}
    a[:, 0, :] = -adj.sum(axis=1)
    return a, det


def simplex_kappa(meshes, lm, w):
    """Mean coefficient carried by every simplex of level mesh lm."""
    out = np.empty(len(lm.simp))
    for s in range(len(lm.simp)):
        b = lm.boxes[lm.simp_box[s]]
        if lm.box_fan[lm.simp_box[s]]:
            out[s] = w[b][0]      # fan boxes are leaves: constant coefficient
        else:
            out[s] = w[b][lm.simp_tmpl[s]]
    return out


def stiffness(meshes, lm, kappa_s, unit_length):
    """Assemble A_l over the unknowns of level mesh lm (exact zeros dropped)."""
    d = lm.d
    sel = lm.kept                                           # the grid's simplices (all, or kept)
    simp = lm.simp[sel]
    kappa_s = np.asarray(kappa_s)[sel]
    V = lm.verts[simp]                                      # (ns, d+1, d)
    box_level = np.array([lm.boxes[i][0] for i in lm.simp_box[sel]], dtype=np.int64)
    half = (1 << (lm.J - box_level)).astype(np.int64)       # half side in units
    E = (V[:, 1:, :] - V[:, :1, :])
    assert np.all(E % half[:, None, None] == 0)
    E = E // half[:, None, None]
    a, det = _adjugate_rows(E)
    denom = (math.factorial(d) * np.abs(det)).astype(np.float64)
    dots = np.einsum("sid,sjd->sij", a, a).astype(np.float64)
    K = dots / denom[:, None, None]
    if d == 3:
        K = K * (half * unit_length)[:, None, None]
    K = K * kappa_s[:, None, None]
    nv = len(lm.verts)
    k = d + 1
    rows = np.repeat(simp, k, axis=1).ravel()
    cols = np.tile(simp, (1, k)).ravel()
    A = sp.coo_matrix((K.ravel(), (rows, cols)), shape=(nv, nv)).tocsr()
    A.sum_duplicates()
    A = A[lm.dof_vert][:, lm.dof_vert].tocsr()
    A.eliminate_zeros()
    A.sort_indices()
    return A


def locate(meshes, lm_coarse, X):
    """Index of a simplex of lm_coarse containing integer point X, with exact barycentrics."""
    J = meshes.J
    d = meshes.d
    for k in range(1, lm_coarse_level(lm_coarse) + 1):
        sh = J - k + 1
        idx = tuple(min(int(x) >> sh, (1 << (k - 1)) - 1) for x in X)
        b = (k,) + idx
        bi = lm_coarse._box_index.get(b)
        if bi is None:
            continue
        for s in lm_coarse._box_simps[bi]:
            V = lm_coarse.verts[lm_coarse.simp[s]]
            lam = _bary_int(V, X)
            if lam is not None:
                return s, lam
    raise RuntimeError("point location failed")


def lm_coarse_level(lm):
    return lm._level


def _bary_int(V, X):
    d = V.shape[1]
    M = (V[1:] - V[0]).T.astype(object)
    rhs = (np.asarray(X) - V[0]).astype(object)

    def det(m):
        if d == 2:
            return m[0][0] * m[1][1] - m[0][1] * m[1][0]
        return (m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1])
                - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0])
                + m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]))
    D = det(M.tolist())
    lam = []
    for j in range(d):
        Mj = M.tolist()
        for r in range(d):
            Mj[r][j] = rhs[r]
        lam.append(det(Mj))
    l0 = D - sum(lam)
    num = [l0] + lam
    if D < 0:
        num = [-x for x in num]
        D = -D
    if any(x < 0 for x in num):
        return None
    return [x / D for x in num]


def prolongation(meshes, lm_fine, lm_coarse):
    """P (n_fine x n_coarse): nodal interpolation of coarse P1 functions at fine unknowns."""
    if not hasattr(lm_coarse, "_box_index"):
        lm_coarse._box_index = {b: i for i, b in enumerate(lm_coarse.boxes)}
        bs = {}
        for s, bi in enumerate(lm_coarse.simp_box):
            bs.setdefault(int(bi), []).append(s)
        lm_coarse._box_simps = bs
    rows, cols, vals = [], [], []
    for i, v in enumerate(lm_fine.dof_vert):
        X = lm_fine.verts[v]
        s, lam = locate(meshes, lm_coarse, X)
        for m, l in enumerate(lam):
            if l == 0:
                continue
            cv = lm_coarse.simp[s][m]
            j = lm_coarse.dof_of_vert[cv]
            if j < 0:
                continue
            rows.append(i)
            cols.append(j)
            vals.append(float(l))
    P = sp.csr_matrix((vals, (rows, cols)), shape=(lm_fine.n, lm_coarse.n))
    P.sum_duplicates()
    P.sort_indices()
    return P


def local_set(P):
    """Index set of the local decomposition of V_J (Section 4.3, the decomposition into
    V_{l,k}, k in N~_l), as a boolean mask over the unknowns of level l.

    k is in N~_l if it is new on level l (not an unknown of level l-1) or its nodal basis
    function changed, phi_{k,l} != phi_{k,l-1}. In the level-l basis,
    phi_{k,l-1} = sum_i P[i, k] phi_{i,l}, so the function is unchanged exactly when column k
    of P_l holds nothing but the entry 1 on the row of k itself. The row of an unknown that
    already existed on level l-1 is that single entry 1 (nodal interpolation reproduces its
    value); a new unknown's row holds its edge's two parents with weight 1/2 (or one, next to
    the boundary).
    """
    P = P.tocsr()
    n = P.shape[0]
    rl = np.diff(P.indptr)
    one = np.zeros(n, dtype=bool)
    has = rl == 1
    one[has] = P.data[P.indptr[:-1][has]] == 1.0
    old = has & one
    colcount = np.diff(P.tocsc().indptr)
    out = ~old
    parent = P.indices[P.indptr[:-1][old]]
    out[np.nonzero(old)[0]] = colcount[parent] > 1
    return out


class AuxOperators:
    """A_l (l = lc..J), P_l (l = lc+1..J) and the coarse Cholesky factor."""

    def __init__(self, tree, meshes, kappa, coarse_max_dofs=1024):
        self.tree = tree
        self.meshes = meshes
        J = tree.J
        leaf_k = tree.leaf_kappa(np.asarray(kappa, dtype=np.float64))
        self.leaf_kappa = leaf_k
        self.w = kuhn_means(tree, leaf_k)
        unit = tree.L * 2.0 ** (-J)
        self.levels = {}
        sizes = {}
        for l in range(J, 0, -1):
            lm = meshes.level(l)
            lm._level = l
            sizes[l] = lm.n
            if lm.n <= coarse_max_dofs:
                break
        self.sizes = sizes
        self.J = J
        self.lc = min(sizes)      # coarsest level visited: the first with n <= N_c (or level 1)
        self.A = {}
        self.P = {}
        for l in range(J, self.lc - 1, -1):
            lm = meshes.level(l)
            ks = simplex_kappa(meshes, lm, self.w)
            self.A[l] = stiffness(meshes, lm, ks, unit)
        for l in range(J, self.lc, -1):
            self.P[l] = prolongation(meshes, meshes.level(l), meshes.level(l - 1))
        # B_0 = A_0^{-1} by Cholesky; on a pure Neumann problem A_0 is singular, and each component
        # with zero row sums is solved with its rank-one regularisation (nearbnd.regularised)
        from .nearbnd import ExactSolve
        self.coarse = ExactSolve(self.A[self.lc])

    def coarse_solve(self, g):
        """B_0 = A_0^{-1} (Algorithm 2): two triangular solves with the Cholesky factor."""
        return self.coarse(g)
