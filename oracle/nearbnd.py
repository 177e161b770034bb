"""Near-boundary correction of the auxiliary V-cycle (Section 3.5, Algorithm 3; oracle) and the
exact solves of singular subsystems that pure Neumann problems bring.

Section 3.5 adds to the coarse-grid correction of level l an exact solve on the unknowns near
the boundary Gamma_l of the level's grid:
    r = f - A_l u,   u|_J += (A_l|_{J x J})^{-1} r|_J,   J = J_{l,j}.
T_(l,0) are the simplices of the level's grid at distance 0 from Gamma_l, T_(l,i) those at
distance 0 from T_(l,i-1) (i = 1..j), and J_{l,j} the unknowns that are vertices of a simplex of
T_(l,j).

Readings:
* The level's grid is the set of kept simplices of sigma^(l) (all of them on the root box), and
  Gamma_l is the boundary of their union: the facets (edges in 2-D, triangles in 3-D) that
  belong to exactly one kept simplex.
* The grids are conforming, so a closed simplex is at distance 0 from a set of simplices (or
  from Gamma_l) exactly when it shares a vertex with it. Hence V_0 = the vertices on Gamma_l,
  T_(l,i) = the kept simplices with a vertex in V_i, V_(i+1) = the vertices of T_(l,i), and
  J_{l,j} = the unknowns among V_(j+1).
* Algorithm 3 corrects once, after the coarse-grid correction. CG needs a symmetric
  preconditioner, so the V-cycle also corrects before the coarse-grid correction (the symmetric
  product of the two subspace corrections, as symmetric Gauss-Seidel is of its two sweeps).
* The paper solves the subsystem with an H-matrix solver; here the solve is exact.
* Singular subsystems (a pure Neumann problem: the coarsest level, or a near-boundary set
  that covers a whole connected component of the level's unknowns): a connected component c of
  the subsystem's graph whose rows sum to zero (A 1_c = 0 up to rounding) is solved with
  A_cc + gamma_c 1_c 1_c^T, gamma_c = mean(diag A_cc) / |c|, which is SPD, acts as the
  pseudo-inverse on vectors with zero sum over c, and keeps the V-cycle symmetric.

Pins (tests): Gamma_l and the layers by a brute-force geometric construction on small grids;
after the correction the residual vanishes on J; the regularised solve returns the
minimum-norm solution on zero-sum right-hand sides; B_co with the correction is symmetric and
positive definite; on a Neumann problem the correction takes fewer iterations than without.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csgraph


def grid_boundary_vertices(lm):
    """Vertices (indices into lm.verts) on Gamma_l, the boundary of the union of kept simplices."""
    simp = lm.simp[lm.kept]
    k = lm.d + 1
    facets = np.concatenate([np.sort(simp[:, [a for a in range(k) if a != skip]], axis=1) for skip in range(k)])
    u, c = np.unique(facets, axis=0, return_counts=True)
    on = np.zeros(len(lm.verts), dtype=bool)
    on[u[c == 1].ravel()] = True
    return on


def near_boundary_set(lm, j):
    """J_{l,j}: sorted unknown indices of level mesh lm within j layers of Gamma_l."""
    simp = lm.simp[lm.kept]
    V = grid_boundary_vertices(lm)
    for _ in range(j + 1):
        T = np.any(V[simp], axis=1)               # simplices with a vertex in V
        Vn = np.zeros_like(V)
        Vn[simp[T].ravel()] = True
        V = Vn
    return np.sort(lm.dof_of_vert[np.nonzero(V & (lm.dof_of_vert >= 0))[0]])


def regularised(A):
    """Dense SPD matrix of the subsystem A (sparse, symmetric): A plus gamma_c 1_c 1_c^T on every
    connected component c whose rows sum to zero."""
    A = sp.csr_matrix(A)
    M = A.toarray()
    n = A.shape[0]
    if n == 0:
        return M
    ncomp, lab = csgraph.connected_components(abs(A) > 0, directed=False)
    d = A.diagonal()
    rs = np.asarray(A.sum(axis=1)).ravel()
    for c in range(ncomp):
        idx = np.nonzero(lab == c)[0]
        scale = np.abs(d[idx]).max()
        if np.abs(rs[idx]).max() <= 1e-10 * scale:
            gamma = d[idx].mean() / len(idx)
            M[np.ix_(idx, idx)] += gamma
    return M


class ExactSolve:
    """x = M^{-1} b with M = regularised(A): a Cholesky factor, applied by two triangular solves."""

    def __init__(self, A, dtype=np.float64):
        M = regularised(A)
        self.n = M.shape[0]
        self.dtype = dtype
        if dtype == np.float64:
            self.L = np.linalg.cholesky(M) if self.n else np.zeros((0, 0))
            self.inv = None
        else:   # the mixed-precision V-cycle applies the rounded inverse, as the GPU does
            self.inv = (np.linalg.inv(M) if self.n else np.zeros((0, 0))).astype(dtype)

    def __call__(self, b):
        if self.n == 0:
            return np.asarray(b).copy()
        if self.inv is not None:
            return self.inv @ np.asarray(b, dtype=self.dtype)
        import scipy.linalg as sla
        y = sla.solve_triangular(self.L, b, lower=True)
        return sla.solve_triangular(self.L.T, y, lower=False)


class NearBoundary:
    """The correction u|_J += (A|_{JxJ})^{-1} (f - A u)|_J of one level."""

    def __init__(self, A, J, dtype=np.float64):
        self.J = np.asarray(J, dtype=np.int64)
        A = sp.csr_matrix(A)
        self.AJ = A[self.J].astype(dtype).tocsr()               # rows J, all columns
        self.solve = ExactSolve(A[self.J][:, self.J], dtype)

    def correct(self, e, g):
        """e += E_J (A_JJ)^{-1} E_J^T (g - A e), in place; returns e."""
        if len(self.J) == 0:
            return e
        r = g[self.J] - self.AJ @ e
        e[self.J] += np.asarray(self.solve(r), dtype=e.dtype)
        return e


def brute_force_layers(lm, j):
    """J_{l,j} by the definition, with plain loops over simplices (for tests on small grids)."""
    kept = [tuple(s) for s, k in zip(lm.simp.tolist(), lm.kept) if k]
    facets = {}
    for s in kept:
        for f in itertools.combinations(sorted(s), len(s) - 1):
            facets[f] = facets.get(f, 0) + 1
    gamma = {v for f, c in facets.items() if c == 1 for v in f}
    T = [s for s in kept if gamma & set(s)]
    for _ in range(j):
        Vt = {v for s in T for v in s}
        T = [s for s in kept if Vt & set(s)]
    verts = {v for s in T for v in s}
    return sorted(int(lm.dof_of_vert[v]) for v in verts if lm.dof_of_vert[v] >= 0)
