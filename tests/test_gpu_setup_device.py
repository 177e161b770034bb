"""The setup steps built on the device (option setup_device: the fine matrix, Section 2, the
cluster tree, Sections 3.1-3.2, the level meshes, Section 3.3, the level matrices A_l, the
prolongations P_l and the Scott-Zhang transfer Pi, Section 4.1, and with the hash order the
colourings) against the host setup and the oracle.

Bar: bit-exact. The unknown numbering, the fine matrix (pattern and values), element keys, the
refined set, the leaves (with their order), J and kappa~ per leaf equal the host build's; the
refined set and the leaves equal the oracle's, and the fine matrix equals the oracle's within
1e-13; and the solve that follows is the same (identical iteration count and bit-identical u).
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import cluster, fem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
A = pytest.importorskip("paper_1410_2153_amd")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _kuhn_graded():
    coords, elems, _ = W.kuhn_cube_mesh(8, 0.1, cfg=2, item=3)
    return dict(coords=coords ** 2, elems=elems, kappa=np.random.default_rng(0).uniform(0.5, 2, len(elems)))


def _lshape():
    coords, elems, _ = W.lshape_mesh(96, 0.3)
    return dict(coords=coords, elems=elems, kappa=np.exp(np.random.default_rng(2).normal(0, 0.5, len(elems))))


def _tiny():
    # 2 triangles: nothing is refined, the root is the only leaf
    coords = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0], [1.0, 1.0]])
    elems = np.array([[0, 1, 2], [1, 3, 2]], dtype=np.int32)
    return dict(coords=coords, elems=elems, kappa=np.array([1.0, 3.0]))


CASES = {
    "square64": lambda: W.make_config(0),
    "graded20k": lambda: W.make_config(1, scale=0.01),
    "graded200k": lambda: W.make_config(1, scale=0.1),
    "cube16": lambda: W.make_config(2, scale=1 / 8),
    "graded_cube": _kuhn_graded,
    "lshape": _lshape,
    "two_triangles": _tiny,
}


@pytest.mark.parametrize("name", list(CASES))
def test_device_tree_matches_host_and_oracle(name):
    _say(f"[gpu tree] case {name}")
    c = CASES[name]()
    kw = dict(device=0)
    Sh = A.Solver(c["coords"], c["elems"], c["kappa"], **kw)
    Sd = A.Solver(c["coords"], c["elems"], c["kappa"], setup_device=1, **kw)
    for ex in ("keys", "refined", "leaves", "leaf_kappa", "A_rowptr", "A_col", "A_val"):
        a, b = Sh.export(ex), Sd.export(ex)
        assert a.dtype == b.dtype and np.array_equal(a, b), ex
    assert np.array_equal(Sh.dof_vertex(), Sd.dof_vertex())
    assert Sh.info() == Sd.info()
    # the level meshes, A_l of every level, P_l and Pi (built on the device), bit for bit
    assert int(Sh.export("device_stages")[0]) == 0
    assert int(Sd.export("device_stages")[0]) == 1 | 2 | 4 | 8 | 16 | 32
    info = Sh.info()
    assert np.array_equal(Sh.export("level_n"), Sd.export("level_n"))
    for ex in ("Pi_rowptr", "Pi_col", "Pi_val"):
        a, b = Sh.export(ex), Sd.export(ex)
        assert a.dtype == b.dtype and np.array_equal(a, b), ex
    for l in range(info["lc"], info["J"] + 1):
        for ex in ("level_verts", "level_simp", "level_dofs", "level_kept", "Al_rowptr", "Al_col", "Al_val") + (
                ("P_rowptr", "P_col", "P_val") if l > info["lc"] else ()):
            a, b = Sh.export(ex, l), Sd.export(ex, l)
            assert a.dtype == b.dtype and np.array_equal(a, b), (ex, l)
    d = c["coords"].shape[1]
    T = cluster.BoxTree(c["coords"], c["elems"])
    ref = Sd.export("refined").reshape(-1, d + 1)
    assert set(map(tuple, ref.tolist())) == set(T.R)
    lv = Sd.export("leaves").reshape(-1, d + 1)
    assert set(map(tuple, lv.tolist())) == set(cluster.leaves(T.R, d))
    Ao, dofs = fem.assemble(c["coords"], c["elems"], c["kappa"], None)
    assert np.array_equal(Sd.dof_vertex(), dofs)
    if Sd.n:
        Ad = Sd.export_csr("A", shape=Ao.shape)
        assert abs(Ad - Ao).max() <= 1e-13 * abs(Ao).max()
    if len(c["elems"]) > 2:
        f = np.random.default_rng(5).uniform(-1, 1, Sh.n)
        uh, ih, _ = Sh.solve(f, 1e-8)
        ud, idv, _ = Sd.solve(f, 1e-8)
        assert ih == idv and np.array_equal(uh, ud)
    th, td = Sh.setup_seconds(), Sd.setup_seconds()
    _say(name, "fine + tree s: host", round(th["fine"] + th["tree"], 4), "device", round(td["fine"] + td["tree"], 4),
         "levels s: host", round(th["levels"], 4), "device", round(td["levels"], 4))


def test_device_assembly_rejects_degenerate_elements():
    c = _tiny()
    elems = c["elems"].copy()
    elems[1] = [1, 1, 2]   # zero area
    with pytest.raises(A.AsmgError) as e:
        A.Solver(c["coords"], elems, c["kappa"], device=0, setup_device=1)
    assert e.value.code == A.EINVAL and "degenerate element 1" in str(e.value)



@pytest.mark.parametrize("name,seed", [("square64", 0), ("graded200k", 12345), ("cube16", 7), ("graded_cube", 0),
                                       ("lshape", 3)])
def test_device_colouring_matches_host(name, seed):
    # Jones-Plassmann rounds on the device give the host's greedy colouring in the hash order,
    # on the original grid and every smoothed auxiliary level; the solves are bit-identical
    _say(f"[gpu colouring] case {name}, seed {seed}")
    c = CASES[name]()
    kw = dict(device=0, colouring=1, colour_seed=seed)
    Sh = A.Solver(c["coords"], c["elems"], c["kappa"], **kw)
    Sd = A.Solver(c["coords"], c["elems"], c["kappa"], setup_device=1, **kw)
    assert int(Sd.export("device_stages")[0]) & 64
    assert np.array_equal(Sh.export("colour_fine"), Sd.export("colour_fine"))
    info = Sh.info()
    for l in range(info["lc"] + 1, info["J"] + 1):
        assert np.array_equal(Sh.export("colour_aux", l), Sd.export("colour_aux", l)), l
    f = np.random.default_rng(6).uniform(-1, 1, Sh.n)
    uh, ih, _ = Sh.solve(f, 1e-8)
    ud, idv, _ = Sd.solve(f, 1e-8)
    assert ih == idv and np.array_equal(uh, ud)
    th, td = Sh.setup_seconds(), Sd.setup_seconds()
    _say(name, "colourings s: host", round(th["colourings"], 4), "device", round(td["colourings"], 4))


@pytest.mark.parametrize("name,domain", [("lshape", 1), ("annulus_mixed", 2)])
def test_device_level_matrices_on_general_domains(name, domain):
    # the level grids keep only part of sigma^(l) (a general domain, or the mixed grids): the
    # device assembly skips the dropped simplices as the host does
    _say(f"[gpu levels] case {name}, domain {domain}")
    dm = None
    if name == "lshape":
        c = _lshape()
    else:
        from oracle.domain import boundary_vertices
        X, T, _ = W.annulus_mesh(200)
        c = dict(coords=X, elems=T, kappa=np.exp(np.random.default_rng(2).normal(0, 0.5, len(T))))
        dm = boundary_vertices(T, len(X)) & (np.hypot(X[:, 0] - 0.5, X[:, 1] - 0.5) > 0.35)
    Sh = A.Solver(c["coords"], c["elems"], c["kappa"], dm, device=0, domain=domain)
    Sd = A.Solver(c["coords"], c["elems"], c["kappa"], dm, device=0, domain=domain, setup_device=1)
    # general domains: the level meshes stay on the host, the rest runs on the device
    assert int(Sd.export("device_stages")[0]) == 1 | 2 | 8 | 16 | 32
    info = Sh.info()
    assert info == Sd.info()
    assert not np.all(Sh.export("level_kept", info["J"]).astype(bool))   # some simplices dropped
    for ex in ("Pi_rowptr", "Pi_col", "Pi_val"):
        a, b = Sh.export(ex), Sd.export(ex)
        assert a.dtype == b.dtype and np.array_equal(a, b), ex
    for l in range(info["lc"], info["J"] + 1):
        for ex in ("Al_rowptr", "Al_col", "Al_val") + (("P_rowptr", "P_col", "P_val") if l > info["lc"] else ()):
            a, b = Sh.export(ex, l), Sd.export(ex, l)
            assert a.dtype == b.dtype and np.array_equal(a, b), (ex, l)
    f = np.random.default_rng(8).uniform(-1, 1, Sh.n)
    uh, ih, _ = Sh.solve(f, 1e-8)
    ud, idv, _ = Sd.solve(f, 1e-8)
    assert ih == idv and np.array_equal(uh, ud)


@pytest.mark.parametrize("setup_device", [0, 1])
def test_mesh_without_unknowns(setup_device):
    # every vertex Dirichlet (n = 0): the solve, B_co, the product and the gradient return at once
    c = _tiny()
    S = A.Solver(c["coords"], c["elems"], c["kappa"], device=0, setup_device=setup_device)
    assert S.n == 0
    u, it, tr = S.solve(np.zeros(0), 1e-8)
    assert u.shape == (0,) and it == 0
    e = torch.zeros(0, dtype=torch.float64, device="cuda")
    ud, itd, _ = S.solve_device(e, 1e-8)
    assert ud.numel() == 0 and itd == 0
    assert S.apply_preconditioner(e).numel() == 0
    assert S.matvec(e).numel() == 0
    g = S.element_gradient(e, e).cpu().numpy()
    assert g.shape == (len(c["elems"]),) and np.all(g == 0)
