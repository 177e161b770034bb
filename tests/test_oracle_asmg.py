"""Pins of the V-cycle and the ASMG preconditioner (oracle.asmg; Algorithms 1 and 2)."""
import numpy as np
import pytest

import workloads as W
from oracle import asmg
from oracle.hierarchy import Hierarchy


def _dense(op, n):
    return np.column_stack([op(e) for e in np.eye(n)])


def _gs_dense(A, col):
    """Dense S = (D - L_pi)^{-1} in the original numbering (colour-major order pi)."""
    n = A.shape[0]
    order = np.lexsort((np.arange(n), col))
    Ad = A.toarray()
    Ap = Ad[np.ix_(order, order)]
    M = np.tril(Ap)                       # D - L in the permuted numbering
    Sp = np.linalg.inv(M)
    S = np.zeros_like(Sp)
    S[np.ix_(order, order)] = Sp
    return S


@pytest.fixture(scope="module")
def tiny():
    c = W.make_config(1, scale=0.0004)      # a few hundred unknowns, graded
    H = Hierarchy(c["coords"], c["elems"], c["kappa"], coarse_max_dofs=30)
    assert H.n <= 600
    return c, H


def test_preconditioner_symmetric_positive_definite(tiny):
    _, H = tiny
    B = H.preconditioner()
    Bd = _dense(B, H.n)
    assert np.abs(Bd - Bd.T).max() <= 1e-13 * np.abs(Bd).max()
    assert np.linalg.eigvalsh(0.5 * (Bd + Bd.T)).min() > 0


def test_preconditioner_closed_form(tiny):
    # B_co = S^T D S + (I - S^T A) Pi B~ Pi^T (I - A S)
    _, H = tiny
    B = H.preconditioner()
    n = H.n
    A = H.A.toarray()
    S = _gs_dense(H.A, H.colour_fine)
    D = np.diag(np.diag(A))
    nJ = H.Pi.shape[1]
    Bt = _dense(lambda g: B.vcycle(H.aux.J, g), nJ)
    Pi = H.Pi.toarray()
    I = np.eye(n)
    closed = S.T @ D @ S + (I - S.T @ A) @ Pi @ Bt @ Pi.T @ (I - A @ S)
    Bd = _dense(B, n)
    np.testing.assert_allclose(Bd, closed, rtol=1e-11, atol=1e-11 * np.abs(closed).max())


def test_vcycle_two_grid_identity(tiny):
    # one level above the bottom: I - B_l A_l = (I - S^T A)^nu (I - P A_c^{-1} P^T A) (I - S A)^nu
    _, H = tiny
    B = H.preconditioner()
    l = H.aux.lc + 1
    A = H.aux.A[l].toarray()
    n = A.shape[0]
    S = _gs_dense(H.aux.A[l], H.colour_aux[l])
    P = H.aux.P[l].toarray()
    Ac = H.aux.A[l - 1].toarray()
    I = np.eye(n)
    E = (np.linalg.matrix_power(I - S.T @ A, 2) @ (I - P @ np.linalg.solve(Ac, P.T @ A))
         @ np.linalg.matrix_power(I - S @ A, 2))
    Bl = _dense(lambda g: B.vcycle(l, g), n)
    np.testing.assert_allclose(I - Bl @ A, E, atol=1e-11)


def test_vcycle_rate_uniform_hierarchy(cfg0_hier):
    # Section 5.1: on the uniform hierarchy the aux V-cycle is geometric multigrid with textbook rates
    _, H = cfg0_hier
    B = H.preconditioner()
    J = H.aux.J
    A = H.aux.A[J]
    rng = np.random.default_rng(0)
    e = rng.standard_normal(A.shape[0])
    norms = []
    for _ in range(8):
        e = e - B.vcycle(J, A @ e)
        norms.append(np.sqrt(e @ (A @ e)))
    rate = (norms[-1] / norms[2]) ** (1 / 5)
    assert rate < 0.2


def test_stationary_asmg_rate(graded_small):
    # Figures 8-9: level-independent residual reduction of roughly 0.4-0.5; require < 0.6
    _, H = graded_small
    B = H.preconditioner()
    A = H.A
    f = np.random.default_rng(2).standard_normal(H.n)
    u = np.zeros(H.n)
    res = [np.linalg.norm(f)]
    for _ in range(12):
        u = u + B(f - A @ u)
        res.append(np.linalg.norm(f - A @ u))
    rate = (res[-1] / res[4]) ** (1 / 8)
    assert rate < 0.6
