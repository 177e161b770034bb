"""The C++ host setup (through the C ABI, host-only handle) against the oracle.

Bit-exact: box keys, refined set, J, bottom level, level vertices/simplices/
unknown numbering, sparsity patterns of A, A_l, P_l, colourings. Values: A,
A_l, P_l, Pi to 1e-13 relative (P_l exactly).
"""
import numpy as np
import pytest

import workloads as W
from oracle.hierarchy import Hierarchy

A = pytest.importorskip("paper_1410_2153_amd")


def _graded_cube():
    coords, elems, _ = W.kuhn_cube_mesh(8, 0.1, cfg=2, item=3)
    return dict(coords=coords ** 2, elems=elems, kappa=np.random.default_rng(0).uniform(0.5, 2, len(elems))), 3


def _general(gen):
    coords, elems, _ = gen()
    k = np.exp(np.random.default_rng(2).normal(0, 0.5, len(elems)))
    return dict(coords=coords, elems=elems, kappa=k), 0, 1


def _mixed(gen, side):
    # mixed Dirichlet/Neumann problem: Dirichlet on the boundary vertices that `side` selects
    from oracle.domain import boundary_vertices
    coords, elems, _ = gen()
    k = np.exp(np.random.default_rng(2).normal(0, 0.5, len(elems)))
    mask = boundary_vertices(elems, len(coords)) & side(coords)
    return dict(coords=coords, elems=elems, kappa=k, dirichlet=mask), 0, 2


CASES = {
    "square64": lambda: (W.make_config(0), 0, 0),
    "graded": lambda: (W.make_config(1, scale=0.004), 0, 0),
    "cube8": lambda: (W.make_config(2, scale=1 / 16), 0, 0),
    "graded_cube": lambda: _graded_cube() + (0,),
    "square64_meshdomain": lambda: (W.make_config(0), 0, 1),
    "lshape": lambda: _general(lambda: W.lshape_mesh(24, 0.3)),
    "annulus": lambda: _general(lambda: W.annulus_mesh(64)),
    "square32_mixed": lambda: _mixed(lambda: W.square_mesh(32, 0.0), lambda X: X[:, 0] == 0.0),
    "lshape_mixed": lambda: _mixed(lambda: W.lshape_mesh(24, 0.3), lambda X: (X[:, 0] == 0.0) | (X[:, 1] == 0.0)),
    "annulus_mixed": lambda: _mixed(lambda: W.annulus_mesh(64),
                                    lambda X: np.hypot(X[:, 0] - 0.5, X[:, 1] - 0.5) > 0.35),
    # pure Neumann problems: no Dirichlet vertex, the Neumann grids (mixed grids with empty Gamma_D)
    "square32_neumann": lambda: _mixed(lambda: W.square_mesh(32, 0.3, cfg=0, item=1), lambda X: X[:, 0] > 2.0),
    "annulus_neumann": lambda: _mixed(lambda: W.annulus_mesh(64), lambda X: X[:, 0] > 2.0),
}


@pytest.fixture(scope="module", params=list(CASES))
def pair(request):
    c, n_min, dom = CASES[request.param]()
    S = A.Solver(c["coords"], c["elems"], c["kappa"], device=-1, n_min=n_min, domain=dom,
                 dirichlet=c.get("dirichlet"))
    H = Hierarchy(c["coords"], c["elems"], c["kappa"], n_min=n_min, domain=["box", "mesh", "mixed"][dom],
                  dirichlet=c.get("dirichlet"))
    return c, S, H


def test_tree(pair):
    c, S, H = pair
    d = c["coords"].shape[1]
    info = S.info()
    assert np.array_equal(S.export("keys").reshape(-1, d), H.tree.keys)
    assert set(map(tuple, S.export("refined").reshape(-1, d + 1).tolist())) == H.tree.R
    assert sorted(map(tuple, S.export("leaves").reshape(-1, d + 1).tolist())) == sorted(H.tree.leaves)
    assert info["J"] == H.tree.J and info["lc"] == H.aux.lc


def test_level_meshes(pair):
    c, S, H = pair
    d = c["coords"].shape[1]
    for l in range(H.aux.lc, H.tree.J + 1):
        lm = H.meshes.level(l)
        assert np.array_equal(S.export("level_verts", l).reshape(-1, d), lm.verts)
        assert np.array_equal(S.export("level_simp", l).reshape(-1, d + 1), lm.simp)
        assert np.array_equal(S.export("level_dofs", l), lm.dof_vert)
        assert np.array_equal(S.export("level_kept", l).astype(bool), lm.kept)


def _same_pattern(X, Y):
    return np.array_equal(X.indptr, Y.indptr) and np.array_equal(X.indices, Y.indices)


def test_operators(pair):
    c, S, H = pair
    Af = S.export_csr("A", shape=H.A.shape)
    assert _same_pattern(Af, H.A)
    assert abs(Af - H.A).max() <= 1e-13 * abs(H.A).max()
    for l in range(H.aux.lc, H.tree.J + 1):
        Al = S.export_csr("Al", l, shape=H.aux.A[l].shape)
        assert _same_pattern(Al, H.aux.A[l])
        assert abs(Al - H.aux.A[l]).max() <= 1e-13 * abs(H.aux.A[l]).max()
    for l in range(H.aux.lc + 1, H.tree.J + 1):
        P = S.export_csr("P", l, shape=H.aux.P[l].shape)
        assert _same_pattern(P, H.aux.P[l])
        assert abs(P - H.aux.P[l]).max() == 0.0
    Pi = S.export_csr("Pi", shape=H.Pi.shape)
    assert abs(Pi - H.Pi).max() <= 1e-13


def test_colourings(pair):
    c, S, H = pair
    assert np.array_equal(S.export("colour_fine"), H.colour_fine)
    for l, col in H.colour_aux.items():
        assert np.array_equal(S.export("colour_aux", l), col)


def test_level_sizes(pair):
    c, S, H = pair
    n = S.export("level_n")
    assert list(n) == [H.meshes.level(l).n for l in range(1, H.tree.J + 1)]


def test_hash_colouring_mode_matches():
    c = W.make_config(1, scale=0.003)
    S = A.Solver(c["coords"], c["elems"], c["kappa"], device=-1, colouring=1, colour_seed=12345)
    H = Hierarchy(c["coords"], c["elems"], c["kappa"], colour_seed=12345, colouring="hash")
    assert np.array_equal(S.export("colour_fine"), H.colour_fine)
    for l, col in H.colour_aux.items():
        assert np.array_equal(S.export("colour_aux", l), col)


@pytest.mark.parametrize("cfg,scale,mode", [(1, 0.003, 2), (2, 0.0625, 2), (1, 0.003, 0), (2, 0.0625, 0)])
def test_colouring_modes_match(cfg, scale, mode):
    c = W.make_config(cfg, scale=scale)
    S = A.Solver(c["coords"], c["elems"], c["kappa"], device=-1, colouring=mode)
    H = Hierarchy(c["coords"], c["elems"], c["kappa"], colouring={0: "natural", 2: "smallest_last"}[mode])
    assert np.array_equal(S.export("colour_fine"), H.colour_fine)
    for l, col in H.colour_aux.items():
        assert np.array_equal(S.export("colour_aux", l), col)


@pytest.mark.parametrize("cfg,scale", [(1, 0.003), (2, 0.0625)])
def test_local_sets_match(cfg, scale):
    from oracle import auxops
    c = W.make_config(cfg, scale=scale)
    S = A.Solver(c["coords"], c["elems"], c["kappa"], device=-1, smoothing=1)
    H = Hierarchy(c["coords"], c["elems"], c["kappa"])
    for l in range(H.aux.lc + 1, H.aux.J + 1):
        assert np.array_equal(S.export("local_set", l).astype(bool), auxops.local_set(H.aux.P[l])), l


@pytest.mark.parametrize("name", ["square32_neumann", "annulus_neumann", "lshape_mixed", "square64"])
def test_near_boundary_sets_and_regularised_bottom(name):
    # J_{l,j} of every level above the bottom (Section 3.5) equals the oracle's, and the bottom
    # inverse (regularised on singular components) equals the oracle's factorisation's inverse
    from oracle import nearbnd
    c, n_min, dom = CASES[name]()
    S = A.Solver(c["coords"], c["elems"], c["kappa"], device=-1, n_min=n_min, domain=dom,
                 dirichlet=c.get("dirichlet"), nb_layers=2)
    H = Hierarchy(c["coords"], c["elems"], c["kappa"], n_min=n_min, domain=["box", "mesh", "mixed"][dom],
                  dirichlet=c.get("dirichlet"))
    for l in range(H.aux.lc + 1, H.tree.J + 1):
        J = nearbnd.near_boundary_set(H.meshes.level(l), 2)
        assert np.array_equal(S.export("nb_set", l), J), l
        info = S.export("nb_info", l)
        assert info[0] == len(J)
    nc = H.aux.A[H.aux.lc].shape[0]
    inv = S.export("coarse_inv").reshape(nc, nc)
    ref = np.linalg.inv(nearbnd.regularised(H.aux.A[H.aux.lc]))
    assert np.abs(inv - ref).max() <= 1e-10 * np.abs(ref).max()
