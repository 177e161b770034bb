"""P1 finite-element stiffness matrix of the model problem (oracle).

Section 2, eq. (2): a(u, v) = <A u, v>, with a_ij the integral of
kappa * grad(phi_i) . grad(phi_j) over Omega (the paper writes kappa = 1; the
coefficient is piecewise constant per element here). The basis functions are
continuous and piecewise affine on the simplices of a conforming triangulation.
Dirichlet vertices (Section 2.1, the set J_D) are eliminated. The unknowns are
the remaining vertices in ascending vertex id.

Pins (tests/test_oracle_fem.py):
* element matrix against the closed-form cotangent formula (2-D) and against
  the Kuhn stencil (3-D);
* row sums of the unreduced matrix are zero (constants are in the kernel);
* an unjittered mesh whose diagonals all run lower-left to upper-right gives the
  5-point stencil [4, -1, -1, -1, -1], and the diagonal couplings are exactly 0;
* P1 reproduction: with kappa = 1 and boundary data g = a + b.x, the system
  A u = -A_IB g_B is solved by u = g.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


def element_gradients(coords: np.ndarray, elems: np.ndarray):
    """Barycentric gradients and volumes of every simplex.

    Returns (G, vol): G[e, i, :] is grad(lambda_i) on element e, and vol[e] is
    |tau_e|. With M = [p_1 - p_0, ..., p_d - p_0] (the edge vectors as columns),
    lambda_{1..d} = M^{-1} (x - p_0). So the gradients of lambda_1..lambda_d are
    the rows of M^{-1}, and grad(lambda_0) = -sum of the others.
    """
    d = coords.shape[1]
    P = coords[elems]                                   # (N, d+1, d)
    M = np.transpose(P[:, 1:, :] - P[:, :1, :], (0, 2, 1))  # columns = edges
    det = np.linalg.det(M)
    if np.any(det == 0.0):
        raise ValueError("degenerate element (zero volume)")
    Minv = np.linalg.inv(M)                             # rows = grad lambda_1..d
    G = np.empty((len(elems), d + 1, d))
    G[:, 1:, :] = Minv
    G[:, 0, :] = -Minv.sum(axis=1)
    vol = np.abs(det) / math.factorial(d)
    return G, vol


def element_matrices(coords, elems, kappa):
    """K_e = kappa_e |tau_e| G_e G_e^T (local (d+1) x (d+1) stiffness)."""
    G, vol = element_gradients(coords, elems)
    K = np.einsum("eid,ejd->eij", G, G) * (kappa * vol)[:, None, None]
    return K


def assemble_full(coords, elems, kappa) -> sp.csr_matrix:
    """Unreduced stiffness matrix over all vertices; pattern = the mesh edge graph.

    Entries that happen to be 0 (right angles) stay stored, so the pattern does
    not depend on the values.
    """
    n = len(coords)
    K = element_matrices(coords, elems, kappa)
    k = elems.shape[1]
    rows = np.repeat(elems, k, axis=1).ravel()
    cols = np.tile(elems, (1, k)).ravel()
    A = sp.coo_matrix((K.ravel(), (rows, cols)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A


def default_dirichlet(coords: np.ndarray) -> np.ndarray:
    """Dirichlet vertex set J_D: vertices on the boundary of the bounding box."""
    lo = coords.min(axis=0)
    hi = coords.max(axis=0)
    return np.any((coords == lo) | (coords == hi), axis=1)


def dof_vertices(dirichlet: np.ndarray) -> np.ndarray:
    """Unknowns: the non-Dirichlet vertices in ascending vertex id."""
    return np.nonzero(~np.asarray(dirichlet, dtype=bool))[0]


def assemble(coords, elems, kappa, dirichlet=None):
    """Reduced stiffness matrix A (rows/cols = unknowns) and the unknown->vertex map."""
    coords = np.asarray(coords, dtype=np.float64)
    elems = np.asarray(elems, dtype=np.int64)
    kappa = np.asarray(kappa, dtype=np.float64)
    if np.any(~np.isfinite(kappa)) or np.any(kappa <= 0):
        raise ValueError("kappa must be finite and positive")
    if dirichlet is None:
        dirichlet = default_dirichlet(coords)
    dofs = dof_vertices(dirichlet)
    A = assemble_full(coords, elems, kappa)
    Ar = A[dofs][:, dofs].tocsr()
    Ar.sort_indices()
    return Ar, dofs


def element_gradient_of_energy(coords, elems, kappa, u_vertex, lam_vertex):
    """g_e = d/dm_e of lam^T A(exp(m)) u = kappa_e lam_e^T K1_e u_e (K1 = element matrix at kappa 1)."""
    K1 = element_matrices(coords, elems, np.ones(len(elems)))
    ue = u_vertex[elems]
    le = lam_vertex[elems]
    return kappa * np.einsum("ei,eij,ej->e", le, K1, ue)
