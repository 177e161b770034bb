"""Preconditioned conjugate gradients with the ASMG preconditioner (oracle).

Section 5.2: CG preconditioned by ASMG. Readings: start from u_0 = 0 (or from the nested
iteration's guess, ``ASMGPreconditioner.nested_guess``); stop at the
first k with ||r_k||_2 <= tol ||f||_2 (the paper iterates to the discretisation
error with nested iteration, which needs a family of meshes). The iteration
count is the number of products A p. f = 0 gives u = 0 after 0 iterations. The
mixed-precision variant applies the same B_co in float32 (matrices and vectors
rounded to nearest). Everything else stays in float64: the products with A, the
dot products, alpha, beta and the updates of u, r and p. At exit the true
residual f - A u is recomputed in float64. If it is above tol, CG restarts from
the true residual.

Pins: on tiny meshes the result agrees with a dense solve; with constant kappa
and lifted linear boundary data the discrete solution is that linear function
(P1 reproduction); the iteration count grows like a + b log N over the square
family (Theorem: kappa(BA) <~ log N).
"""
from __future__ import annotations

import numpy as np


def pcg(A, f, B, tol=1e-8, max_iter=1000, record=False, u0=None):
    """Returns (u, iterations, info) with info = dict(true_rel_residual, history, status).
    ``u0``: initial guess (default 0); the stopping rule stays relative to ||f||."""
    f = np.asarray(f, dtype=np.float64)
    n = len(f)
    u = np.zeros(n)
    nf = float(np.linalg.norm(f))
    hist = []
    if nf == 0.0:
        return u, 0, dict(true_rel_residual=0.0, history=hist, status="ok", restarts=0)
    total = 0
    restarts = 0
    if u0 is None:
        r = f.copy()
    else:
        u[:] = np.asarray(u0, dtype=np.float64)
        r = f - A @ u
        if float(np.linalg.norm(r)) <= tol * nf:   # the guess already meets the rule
            return u, 0, dict(true_rel_residual=float(np.linalg.norm(r)) / nf, history=hist, status="ok",
                              restarts=0)
    while True:
        z = np.asarray(B(r), dtype=np.float64)
        p = z.copy()
        rho = float(r @ z)
        conv = False
        while total < max_iter:
            q = A @ p
            pq = float(p @ q)
            if not pq > 0:
                return u, total, dict(true_rel_residual=np.nan, history=hist, status="notspd", restarts=restarts)
            alpha = rho / pq
            u += alpha * p
            r -= alpha * q
            total += 1
            rn = float(np.linalg.norm(r))
            if record:
                hist.append(rn / nf)
            if rn <= tol * nf:
                conv = True
                break
            z = np.asarray(B(r), dtype=np.float64)
            rho_new = float(r @ z)
            beta = rho_new / rho
            rho = rho_new
            p = z + beta * p
        true = float(np.linalg.norm(f - A @ u)) / nf
        if not conv:
            return u, total, dict(true_rel_residual=true, history=hist, status="noconv", restarts=restarts)
        if true <= tol or restarts >= 3:
            return u, total, dict(true_rel_residual=true, history=hist, status="ok", restarts=restarts)
        restarts += 1
        r = f - A @ u
