"""Gauss-Seidel smoother, auxiliary V-cycle and the multiplicative ASMG preconditioner (oracle).

* Smoother (Section 4.1): Gauss-Seidel S = (D - L)^(-1), applied in the
  colour-major ordering of ``colour``. A forward sweep visits colours
  0..C-1 and updates every unknown i of the colour with
  x_i <- x_i + (b_i - (A x)_i) / a_ii. The backward sweep (S^T) visits the
  colours in reverse order.
* V-cycle (Algorithm 2) on the auxiliary hierarchy. Readings: the residual
  equation uses f (the paper writes g); the post-smoothing runs nu backward
  sweeps, so the cycle uses symmetric Gauss-Seidel (Section 5.1, nu = 2); the
  bottom level l_c is the finest level with at most N_c unknowns, and it is
  solved exactly with the Cholesky factor (B_0 = A_0^(-1)).
* ASMG preconditioner B_co (Algorithm 1, eq. (fasp2)), with the update signs read
  as + (the algorithm prints -; Algorithm 2 uses +):
      u1 = S r                              (nu_fine forward sweeps from 0)
      u2 = u1 + Pi Vcycle_J(Pi^T (r - A u1))
      z  = u2 + S^T (r - A u2)              (nu_fine backward sweeps from u2)
  This makes I - B_co A = (I - S^T A)(I - Pi B~ Pi^T A)(I - S A). Because
  S^(-1) + S^(-T) - A = D, B_co = S^T D S + (I - S^T A) Pi B~ Pi^T (I - A S)
  is symmetric positive definite whenever B~ is.

* Local smoothing (option ``smoothing="local"``): the V-cycle smooths level l
  only on the unknowns of N~_l (``auxops.local_set``), the index set of the
  decomposition V_J = sum_l sum_{k in N~_l} V_{l,k} under which Section 4.3
  proves the multigrid bound. The sweeps visit the same colours in the same
  order, restricted to those rows; residuals and transfers stay whole.

* Near-boundary correction (option ``nb_layers`` = j > 0; Section 3.5, Algorithm 3): on every
  level above the bottom, an exact solve on the unknowns J_{l,j} within j layers of the level
  grid's boundary, before and after the coarse-grid correction (``nearbnd``).

* Nested iteration (Section 5.2 starts CG from a nested iteration over the levels of the
  hierarchy, coarsest to finest). Reading: the levels are the auxiliary levels l_c..J and
  then the original grid. The load vector is carried down by the transposed transfers,
  g_J = Pi^T f and g_(l-1) = P_l^T g_l (for nested P1 spaces P_l^T g_l is exactly level
  l-1's load vector); e_(l_c) = A_(l_c)^(-1) g_(l_c); on each finer level
  e_l = P_l e_(l-1) followed by ``cycles`` iterations e_l <- e_l + B_l (g_l - A_l e_l) with
  the V-cycle B_l of Algorithm 2; the initial guess of CG is u_0 = Pi e_J.

Pins: on small meshes B_co, formed densely, is symmetric (1e-13) and positive
definite, and matches the closed form above; a V-cycle on the uniform hierarchy
of the square is the textbook geometric multigrid of Section 5.1; with local
smoothing, B_co stays symmetric positive definite, N~_l agrees with a geometric
count of bisected edges, and on the uniform hierarchy (N~_l = N_l) it is the
full-smoothing B_co.
"""
from __future__ import annotations

import numpy as np


class Smoother:
    """Multicolour Gauss-Seidel for one matrix (rows of each colour pre-sliced). With ``mask``,
    only the rows where it is true are smoothed (the other unknowns keep their values)."""

    def __init__(self, A, colour, dtype=np.float64, mask=None):
        A = A.tocsr().astype(dtype)
        self.A = A
        self.dtype = dtype
        self.diag = A.diagonal().astype(dtype)
        C = int(colour.max()) + 1 if len(colour) else 0
        sel = np.ones(len(colour), dtype=bool) if mask is None else np.asarray(mask, dtype=bool)
        self.rows = [np.nonzero((colour == c) & sel)[0] for c in range(C)]
        self.blocks = [A[r] for r in self.rows]
        self.dblk = [self.diag[r] for r in self.rows]

    def _pass(self, c, x, b):
        r = self.rows[c]
        x[r] = x[r] + (b[r] - self.blocks[c] @ x) / self.dblk[c]

    def forward(self, x, b):
        for c in range(len(self.rows)):
            self._pass(c, x, b)

    def backward(self, x, b):
        for c in range(len(self.rows) - 1, -1, -1):
            self._pass(c, x, b)


class ASMGPreconditioner:
    """B_co of Algorithm 1 with the V-cycle of Algorithm 2 on the auxiliary levels."""

    def __init__(self, hier, dtype=np.float64, nu_aux=2, nu_fine=1, smoothing="full", nb_layers=0):
        from .auxops import local_set
        from .nearbnd import ExactSolve, NearBoundary, near_boundary_set
        self.h = hier
        self.dtype = dtype
        self.nu_aux = nu_aux
        self.nu_fine = nu_fine
        ops = hier.aux
        self.lc = ops.lc
        self.J = ops.J
        self.fine = Smoother(hier.A, hier.colour_fine, dtype)
        if smoothing not in ("full", "local"):
            raise ValueError(smoothing)
        self.masks = {l: (local_set(ops.P[l]) if smoothing == "local" else None)
                      for l in range(self.lc + 1, self.J + 1)}
        self.aux = {l: Smoother(ops.A[l], hier.colour_aux[l], dtype, self.masks[l])
                    for l in range(self.lc + 1, self.J + 1)}
        self.Aaux = {l: ops.A[l].astype(dtype) for l in ops.A}
        self.P = {l: ops.P[l].astype(dtype) for l in ops.P}
        self.PT = {l: ops.P[l].T.tocsr().astype(dtype) for l in ops.P}
        self.Pi = hier.Pi.astype(dtype)
        self.PiT = hier.Pi.T.tocsr().astype(dtype)
        if dtype == np.float64:
            self._coarse = ops.coarse_solve
        else:
            self._coarse = ExactSolve(ops.A[self.lc], dtype)
        # near-boundary correction (Section 3.5, Algorithm 3) on the levels above the bottom
        self.nb = {}
        if nb_layers > 0:
            for l in range(self.lc + 1, self.J + 1):
                J = near_boundary_set(hier.meshes.level(l), nb_layers)
                if len(J):
                    self.nb[l] = NearBoundary(ops.A[l], J, dtype)

    def vcycle(self, level, g):
        """Algorithm 2 (B_l applied to g)."""
        if level == self.lc:
            return self._coarse(g).astype(self.dtype)
        S = self.aux[level]
        A = self.Aaux[level]
        e = np.zeros_like(g)
        nb = self.nb.get(level)
        for _ in range(self.nu_aux):
            S.forward(e, g)
        if nb is not None:     # before the coarse-grid correction too: B_l stays symmetric
            nb.correct(e, g)
        r = g - A @ e
        e = e + self.P[level] @ self.vcycle(level - 1, self.PT[level] @ r)
        if nb is not None:     # Algorithm 3: after the coarse-grid correction
            nb.correct(e, g)
        for _ in range(self.nu_aux):
            S.backward(e, g)
        return e

    def apply(self, r):
        """z = B_co r (Algorithm 1 from u = 0)."""
        dt = self.dtype
        r = np.asarray(r).astype(dt)
        A = self.fine.A
        u = np.zeros_like(r)
        for _ in range(self.nu_fine):
            self.fine.forward(u, r)
        r1 = r - A @ u
        u = u + self.Pi @ self.vcycle(self.J, self.PiT @ r1)
        for _ in range(self.nu_fine):
            self.fine.backward(u, r)
        return u

    __call__ = apply

    def nested_guess(self, f, cycles=1, levels=False):
        """Initial guess u_0 = Pi e_J of the nested iteration over the auxiliary levels (in the
        preconditioner's dtype). With ``levels``, also returns the dicts g and e per level."""
        dt = self.dtype
        f = np.asarray(f).astype(dt)
        g = {self.J: self.PiT @ f}
        for l in range(self.J, self.lc, -1):
            g[l - 1] = self.PT[l] @ g[l]
        e = {self.lc: np.asarray(self._coarse(g[self.lc])).astype(dt)}
        for l in range(self.lc + 1, self.J + 1):
            el = self.P[l] @ e[l - 1]
            for _ in range(cycles):
                el = el + self.vcycle(l, g[l] - self.Aaux[l] @ el)
            e[l] = el
        u0 = self.Pi @ e[self.J]
        return (u0, g, e) if levels else u0
