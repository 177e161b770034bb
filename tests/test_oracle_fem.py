"""Pins of the fine P1 assembly (oracle.fem) against closed forms (Section 2, eq. (2))."""
import numpy as np
import pytest

import workloads as W
from oracle import fem


def test_reference_triangle_closed_form():
    # unit right triangle: K = 1/2 [[2,-1,-1],[-1,1,0],[-1,0,1]]
    c = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    K = fem.element_matrices(c, np.array([[0, 1, 2]]), np.array([1.0]))[0]
    np.testing.assert_allclose(K, 0.5 * np.array([[2, -1, -1], [-1, 1, 0], [-1, 0, 1]]), atol=1e-15)


def test_random_triangle_cotangent_formula():
    rng = np.random.default_rng(7)
    for _ in range(20):
        p = rng.uniform(-1, 1, (3, 2))
        kap = rng.uniform(0.5, 3.0)
        K = fem.element_matrices(p, np.array([[0, 1, 2]]), np.array([kap]))[0]
        for i in range(3):
            for j in range(3):
                if i == j:
                    continue
                k = 3 - i - j
                u = p[i] - p[k]
                v = p[j] - p[k]
                cot = (u @ v) / abs(u[0] * v[1] - u[1] * v[0])
                assert K[i, j] == pytest.approx(-0.5 * kap * cot, rel=1e-12, abs=1e-14)


def test_reference_tetrahedron_closed_form():
    c = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]])
    K = fem.element_matrices(c, np.array([[0, 1, 2, 3]]), np.array([2.0]))[0]
    ref = np.array([[3, -1, -1, -1], [-1, 1, 0, 0], [-1, 0, 1, 0], [-1, 0, 0, 1]]) / 6.0 * 2.0
    np.testing.assert_allclose(K, ref, atol=1e-15)


@pytest.mark.parametrize("dim", [2, 3])
def test_linear_functions_in_kernel(dim):
    if dim == 2:
        coords, elems, _ = W.square_mesh(12, 0.3, cfg=0, item=5)
    else:
        coords, elems, _ = W.kuhn_cube_mesh(5, 0.2, cfg=2, item=5)
    kappa = np.random.default_rng(1).uniform(0.1, 10, len(elems))
    A = fem.assemble_full(coords, elems, kappa)
    np.testing.assert_allclose(A @ np.ones(len(coords)), 0, atol=1e-12)
    g = 0.3 + coords @ np.arange(1, dim + 1)
    bnd = fem.default_dirichlet(coords)
    # rows of interior vertices annihilate linear functions only where kappa is constant on the patch:
    A1 = fem.assemble_full(coords, elems, np.ones(len(elems)))
    np.testing.assert_allclose((A1 @ g)[~bnd], 0, atol=1e-12)


def test_five_point_stencil():
    coords, elems, _ = W.square_mesh(8, 0.0, diagonals="ur")
    A, dofs = fem.assemble(coords, elems, np.ones(len(elems)))
    D = A.toarray()
    n = 7
    for a, va in enumerate(dofs):
        ia, ja = va % 9, va // 9
        for b, vb in enumerate(dofs):
            ib, jb = vb % 9, vb // 9
            if a == b:
                assert D[a, b] == pytest.approx(4.0, rel=1e-14)
            elif abs(ia - ib) + abs(ja - jb) == 1:
                assert D[a, b] == pytest.approx(-1.0, rel=1e-14)
            else:
                assert abs(D[a, b]) < 1e-15
    assert A.shape == (n * n, n * n)


def test_kuhn_seven_point_stencil():
    n = 6
    coords, elems, _ = W.kuhn_cube_mesh(n, 0.0)
    A, dofs = fem.assemble(coords, elems, np.ones(len(elems)))
    h = 1.0 / n
    D = A.toarray()
    m = n + 1
    ijk = np.stack([dofs % m, (dofs // m) % m, dofs // (m * m)], 1)
    dist = np.abs(ijk[:, None, :] - ijk[None, :, :]).sum(-1)
    np.testing.assert_allclose(np.diag(D), 6 * h, rtol=1e-14)
    np.testing.assert_allclose(D[dist == 1], -h, rtol=1e-13)
    off = (dist > 1)
    assert np.all(np.abs(D[off]) < 1e-16)


def test_p1_reproduction_solve():
    import scipy.sparse.linalg as sl
    coords, elems, _ = W.square_mesh(16, 0.3, cfg=0, item=3)
    A_full = fem.assemble_full(coords, elems, np.ones(len(elems)))
    bnd = fem.default_dirichlet(coords)
    g = 1.5 - 2.0 * coords[:, 0] + 0.7 * coords[:, 1]
    I = np.nonzero(~bnd)[0]
    B = np.nonzero(bnd)[0]
    f = -(A_full[I][:, B] @ g[B])
    A, dofs = fem.assemble(coords, elems, np.ones(len(elems)))
    u = sl.spsolve(A.tocsc(), f)
    np.testing.assert_allclose(u, g[I], atol=1e-12)


def test_rejects_bad_input():
    coords, elems, _ = W.square_mesh(4, 0.0)
    with pytest.raises(ValueError):
        fem.assemble(coords, elems, -np.ones(len(elems)))
    bad = elems.copy()
    bad[0] = [0, 0, 1]
    with pytest.raises(ValueError):
        fem.assemble(coords, bad, np.ones(len(elems)))
