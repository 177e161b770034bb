"""Pins of the multicolour ordering and the Gauss-Seidel smoother (oracle.colour, oracle.asmg)."""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as sla
import pytest

from oracle import asmg, colour


def test_fmix32_reference_values():
    # MurmurHash3 fmix32 of 0 is 0; values below computed by hand from the published finaliser
    assert int(colour.fmix32(np.array([0]))[0]) == 0
    h = 1
    h ^= h >> 16
    h = (h * 0x85EBCA6B) & 0xFFFFFFFF
    h ^= h >> 13
    h = (h * 0xC2B2AE35) & 0xFFFFFFFF
    h ^= h >> 16
    assert int(colour.fmix32(np.array([1]))[0]) == h == 0x514E28B7


def test_colouring_proper_and_deterministic(cfg0_hier):
    _, H = cfg0_hier
    for A, col in [(H.A, H.colour_fine)] + [(H.aux.A[l], H.colour_aux[l]) for l in H.colour_aux]:
        A = A.tocoo()
        off = A.row != A.col
        assert np.all(col[A.row[off]] != col[A.col[off]])
        assert np.array_equal(col, colour.greedy_colouring(A, 0))
        hc = colour.greedy_colouring(A, 7, "hash")
        assert np.all(hc[A.row[off]] != hc[A.col[off]])


def _perm_parts(A, col):
    order = np.lexsort((np.arange(len(col)), col))
    Ap = A.tocsr()[order][:, order]
    D = sp.diags(Ap.diagonal())
    Lo = -sp.tril(Ap, -1)
    return order, Ap, D, Lo


def test_natural_order_checkerboard_on_five_point():
    import scipy.sparse as sp
    n = 9
    T = sp.diags([-1, 2, -1], [-1, 0, 1], shape=(n, n))
    A = sp.kron(T, sp.eye(n)) + sp.kron(sp.eye(n), T)
    col = colour.greedy_colouring(A)
    i, j = np.divmod(np.arange(n * n), n)
    assert np.array_equal(col, (i + j) % 2)


def test_multicolour_sweep_is_gauss_seidel_in_colour_order(cfg0_hier):
    _, H = cfg0_hier
    A, col = H.A, H.colour_fine
    order, Ap, D, Lo = _perm_parts(A, col)
    b = np.random.default_rng(0).standard_normal(A.shape[0])
    S = asmg.Smoother(A, col)
    x = np.zeros_like(b)
    S.forward(x, b)
    ref = sla.spsolve_triangular((D - Lo).tocsr(), b[order], lower=True)
    np.testing.assert_allclose(x[order], ref, rtol=1e-13, atol=1e-13)
    # backward sweep = S^T
    y = np.zeros_like(b)
    S.backward(y, b)
    refT = sla.spsolve_triangular((D - Lo).T.tocsr(), b[order], lower=False)
    np.testing.assert_allclose(y[order], refT, rtol=1e-13, atol=1e-13)


def test_jacobi_and_gauss_seidel_continuity(cfg0_hier):
    # Section 4.3: ||v||_A^2 <= K <Dv,v>, K = max nnz per row; (1/K)<(D-L)x,x> <= <Dx,x> <= 2<(D-L)x,x>
    _, H = cfg0_hier
    A, col = H.A, H.colour_fine
    order, Ap, D, Lo = _perm_parts(A, col)
    K = int(np.diff(Ap.indptr).max())
    rng = np.random.default_rng(1)
    for _ in range(20):
        x = rng.standard_normal(A.shape[0])
        dx = x @ (D @ x)
        gs = x @ ((D - Lo) @ x)
        assert x @ (Ap @ x) <= K * dx * (1 + 1e-12)
        assert gs / K <= dx * (1 + 1e-12)
        assert dx <= 2 * gs * (1 + 1e-12)
