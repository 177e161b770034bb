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
        assert np.array_equal(col, colour.greedy_colouring(A, 0, "smallest_last"))
        nc = colour.greedy_colouring(A, 0)
        assert np.all(nc[A.row[off]] != nc[A.col[off]])
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


def _graph(n, edges):
    r = [i for i, j in edges] + [j for i, j in edges] + list(range(n))
    c = [j for i, j in edges] + [i for i, j in edges] + list(range(n))
    return sp.csr_matrix((np.ones(len(r)), (r, c)), shape=(n, n))


def test_smallest_last_path_by_hand():
    # path 0-1-2-3, degrees (1,2,2,1): removals by smallest (degree, index) are 0 (deg 1),
    # then 1 (deg 1 once 0 is gone), then 2, then 3; colouring order 3,2,1,0 gives
    # colours 0,1,0,1 in that order, i.e. [1,0,1,0] by index
    A = _graph(4, [(0, 1), (1, 2), (2, 3)])
    assert list(colour.smallest_last_order(A)) == [3, 2, 1, 0]
    assert list(colour.greedy_colouring(A, 0, "smallest_last")) == [1, 0, 1, 0]
    # star, centre 0 and leaves 1..4: leaves 1, 2, 3 go first (deg 1); then centre and leaf 4
    # both have degree 1 and the centre (index 0) goes; leaf 4 last. Colouring order 4,0,3,2,1
    A = _graph(5, [(0, k) for k in range(1, 5)])
    assert list(colour.smallest_last_order(A)) == [4, 0, 3, 2, 1]
    assert list(colour.greedy_colouring(A, 0, "smallest_last")) == [1, 0, 0, 0, 0]


def _degeneracy_brute(A):
    # max over all vertex subsets S of the minimum degree of the induced subgraph (exhaustive)
    A = A.tocsr()
    n = A.shape[0]
    adj = [set(int(j) for j in A.indices[A.indptr[i]:A.indptr[i + 1]] if j != i) for i in range(n)]
    best = 0
    for mask in range(1, 1 << n):
        S = [i for i in range(n) if mask >> i & 1]
        m = min(sum(1 for j in adj[i] if mask >> j & 1) for i in S)
        best = max(best, m)
    return best


def test_smallest_last_within_degeneracy_bound():
    # Matula-Beck: greedy colouring in smallest-last order uses at most degeneracy + 1 colours
    rng = np.random.default_rng(5)
    for trial in range(25):
        n = int(rng.integers(3, 11))
        p = rng.uniform(0.15, 0.8)
        edges = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]
        A = _graph(n, edges)
        col = colour.greedy_colouring(A, 0, "smallest_last")
        Ac = A.tocoo()
        off = Ac.row != Ac.col
        assert np.all(col[Ac.row[off]] != col[Ac.col[off]])
        assert col.max() + 1 <= _degeneracy_brute(A) + 1
    # complete graph: n colours; random tree: 2 colours
    assert colour.greedy_colouring(_graph(6, [(i, j) for i in range(6) for j in range(i + 1, 6)]), 0,
                                   "smallest_last").max() == 5
    parent = [int(rng.integers(0, k)) for k in range(1, 40)]
    tree = _graph(40, [(k + 1, parent[k]) for k in range(39)])
    assert colour.greedy_colouring(tree, 0, "smallest_last").max() == 1


def test_smallest_last_on_mesh_graphs(cfg0_hier):
    # planar mesh graphs have degeneracy <= 5, so at most 6 colours; proper on every level
    _, H = cfg0_hier
    for A in [H.A] + [H.aux.A[l] for l in H.colour_aux]:
        col = colour.greedy_colouring(A, 0, "smallest_last")
        Ac = A.tocoo()
        off = Ac.row != Ac.col
        assert np.all(col[Ac.row[off]] != col[Ac.col[off]])
        assert col.max() + 1 <= 6
