"""Adjoint gradient of a least-squares loss w.r.t. per-element log-coefficients (oracle).

The model problem's coefficient enters A linearly: A(kappa) = sum_e kappa_e K1_e,
where K1_e is the element matrix at kappa = 1 (Section 2, eq. (2)). With
kappa = exp(m), the loss J(m) = 1/2 ||u(m) - u_obs||^2 and A(m) u = f give the
following. A is symmetric, so the adjoint solve reuses the same matrix:

    A lam = u - u_obs,    dJ/dm_e = -kappa_e lam_e^T K1_e u_e,

with Dirichlet entries of u and lam taken as 0.

The reference gradient solves with scipy.sparse.linalg.spsolve. The PCG
variant reuses the oracle's preconditioned CG. Pins: directional finite
differences of J, with forward solves to 1e-12.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as sla

from . import fem


def loss_and_gradient(coords, elems, m, f, u_obs, dirichlet=None, solver=None):
    """Returns (J, dJ/dm (n_elems,), u). ``solver(A, b)`` defaults to a sparse direct solve."""
    kappa = np.exp(m)
    A, dofs = fem.assemble(coords, elems, kappa, dirichlet)
    if solver is None:
        def solver(A_, b):
            return sla.spsolve(A_.tocsc(), b)
    u = solver(A, f)
    res = u - u_obs
    J = 0.5 * float(res @ res)
    lam = solver(A, res)
    nv = len(coords)
    uv = np.zeros(nv)
    lv = np.zeros(nv)
    uv[dofs] = u
    lv[dofs] = lam
    g = -fem.element_gradient_of_energy(coords, elems, kappa, uv, lv)
    return J, g, u
