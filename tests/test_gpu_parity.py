"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Bar (stated per test): same PCG iteration count and ||u_gpu - u_oracle|| <=
1e-10 ||u_oracle|| in FP64 (same algorithm, same ordering; only the summation
order inside a row or a dot product differs); mixed precision within 1e-6 of
the oracle solved to 1e-12.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle.hierarchy import Hierarchy

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
A = pytest.importorskip("paper_1410_2153_amd")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _graded_cube():
    coords, elems, _ = W.kuhn_cube_mesh(8, 0.1, cfg=2, item=3)
    c = dict(coords=coords ** 2, elems=elems, kappa=np.random.default_rng(0).uniform(0.5, 2, len(elems)))
    c["f_vertex"] = W.rhs_per_vertex(len(coords), 2, 3)
    return c, 3, 0, 0


def _general(gen):
    coords, elems, _ = gen()
    c = dict(coords=coords, elems=elems, kappa=np.exp(np.random.default_rng(2).normal(0, 0.5, len(elems))))
    c["f_vertex"] = W.rhs_per_vertex(len(coords), 5, 1)
    return c, 0, 2, 0, 1


def _mixed(gen, side):
    # mixed problem: Dirichlet on the boundary vertices `side` selects, Neumann elsewhere
    from oracle.domain import boundary_vertices
    coords, elems, _ = gen()
    c = dict(coords=coords, elems=elems, kappa=np.exp(np.random.default_rng(2).normal(0, 0.5, len(elems))))
    c["f_vertex"] = W.rhs_per_vertex(len(coords), 5, 1)
    c["dirichlet"] = boundary_vertices(elems, len(coords)) & side(coords)
    return c, 0, 2, 0, 2


# name -> (workload, n_min (0 = default), colouring: 0 natural order, 2 smallest-last,
#          smoothing: 0 whole auxiliary levels, 1 local on N~_l[, domain: 0 root box, 1 mesh domain,
#          2 mixed Dirichlet/Neumann grids (workload carries the Dirichlet mask)])
CASES = {
    "square64": lambda: (W.make_config(0), 0, 0, 0),
    "graded20k": lambda: (W.make_config(1, scale=0.01), 0, 0, 0),
    "cube16": lambda: (W.make_config(2, scale=1 / 8), 0, 0, 0),
    "graded_cube": _graded_cube,
    "graded20k_smallest_last": lambda: (W.make_config(1, scale=0.01), 0, 2, 0),
    "cube16_smallest_last": lambda: (W.make_config(2, scale=1 / 8), 0, 2, 0),
    "graded20k_local": lambda: (W.make_config(1, scale=0.01), 0, 2, 1),
    "graded_cube_local": lambda: _graded_cube()[:2] + (2, 1),
    "lshape_domain": lambda: _general(lambda: W.lshape_mesh(96, 0.3)),
    "annulus_domain": lambda: _general(lambda: W.annulus_mesh(400)),
    "annulus_mixed": lambda: _mixed(lambda: W.annulus_mesh(300),
                                    lambda X: np.hypot(X[:, 0] - 0.5, X[:, 1] - 0.5) > 0.35),
    "lshape_mixed": lambda: _mixed(lambda: W.lshape_mesh(96, 0.3), lambda X: (X[:, 0] == 0.0) | (X[:, 1] == 0.0)),
    "annulus_mixed_local": lambda: _mixed(lambda: W.annulus_mesh(200),
                                          lambda X: np.hypot(X[:, 0] - 0.5, X[:, 1] - 0.5) > 0.35)[:3] + (1, 2),
}
ORACLE_COLOURING = {0: "natural", 2: "smallest_last"}
ORACLE_SMOOTHING = {0: "full", 1: "local"}


class _Oracle:
    """The oracle hierarchy with the case's smoothing as the default of preconditioner() and solve()."""

    def __init__(self, H, smoothing):
        self._H, self._sm = H, smoothing

    def __getattr__(self, k):
        return getattr(self._H, k)

    def preconditioner(self, *a, **kw):
        kw.setdefault("smoothing", self._sm)
        return self._H.preconditioner(*a, **kw)

    def solve(self, *a, **kw):
        kw.setdefault("smoothing", self._sm)
        return self._H.solve(*a, **kw)


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    _say(f"[gpu parity] case {request.param}")
    c, n_min, col, sm, *rest = CASES[request.param]()
    dom = rest[0] if rest else 0
    dm = c.get("dirichlet")
    H = _Oracle(Hierarchy(c["coords"], c["elems"], c["kappa"], dirichlet=dm, n_min=n_min,
                          colouring=ORACLE_COLOURING[col], domain=["box", "mesh", "mixed"][dom]), ORACLE_SMOOTHING[sm])
    S64 = A.Solver(c["coords"], c["elems"], c["kappa"], dm, n_min=n_min, colouring=col, smoothing=sm, domain=dom)
    S64.kwargs = dict(n_min=n_min, colouring=col, smoothing=sm, domain=dom, dirichlet=dm)
    S32 = A.Solver(c["coords"], c["elems"], c["kappa"], dm, n_min=n_min, precision=A.PREC_MIXED, colouring=col,
                   smoothing=sm, domain=dom)
    f = c["f_vertex"][H.dofs]
    return request.param, c, H, S64, S32, f


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _rel_inf(a, b):
    """element-wise bar: max_i |a_i - b_i| / max_i |b_i|"""
    return float(np.abs(a - b).max() / np.abs(b).max())


def test_matvec(case):
    name, c, H, S64, S32, f = case
    x = np.random.default_rng(1).standard_normal(H.n)
    y = S64.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    assert _rel(y, H.A @ x) <= 1e-14


def test_preconditioner_fp64(case):
    name, c, H, S64, S32, f = case
    r = np.random.default_rng(2).standard_normal(H.n)
    z = S64.apply_preconditioner(torch.from_numpy(r).cuda()).cpu().numpy()
    zo = H.preconditioner()(r)
    _say(name, "B_co fp64 rel diff", _rel(z, zo), "element-wise", _rel_inf(z, zo))
    assert _rel(z, zo) <= 1e-12
    assert _rel_inf(z, zo) <= 1e-12


def test_preconditioner_mixed(case):
    name, c, H, S64, S32, f = case
    r = np.random.default_rng(3).standard_normal(H.n)
    z = S32.apply_preconditioner(torch.from_numpy(r).cuda()).cpu().numpy()
    zo = H.preconditioner()(r)
    _say(name, "B_co fp32 vs fp64 oracle rel diff", _rel(z, zo))
    assert _rel(z, zo) <= 1e-5


def test_preconditioner_symmetric(case):
    name, c, H, S64, S32, f = case
    g = np.random.default_rng(4)
    x, y = g.standard_normal(H.n), g.standard_normal(H.n)
    Bx = S64.apply_preconditioner(torch.from_numpy(x).cuda()).cpu().numpy()
    By = S64.apply_preconditioner(torch.from_numpy(y).cuda()).cpu().numpy()
    assert abs(Bx @ y - x @ By) <= 1e-12 * abs(Bx @ y)
    assert Bx @ x > 0


def test_solve_fp64(case):
    name, c, H, S64, S32, f = case
    uo, ito, info = H.solve(f, 1e-8, record=True)
    u, it, tr = S64.solve(f, 1e-8)
    _say(name, "iters gpu", it, "oracle", ito, "rel diff", _rel(u, uo), "true res", tr)
    hist = info["history"]
    near = any(abs(h - 1e-8) < 1e-3 * 1e-8 for h in hist[-2:])
    assert it == ito or near
    assert tr <= 1e-8 * (1 + 1e-6)
    assert _rel(u, uo) <= 1e-10
    assert _rel_inf(u, uo) <= 1e-10


# reduction grids capped at a few blocks: every grid-stride loop of the PCG kernels (initial
# residual, q = A p with p.q, the updates with ||r||^2, r.z, the true residual) runs many rounds
@pytest.mark.parametrize("blocks", [3, 11])
def test_solve_fp64_grid_stride_loops(case, blocks):
    name, c, H, S64, S32, f = case
    if name not in ("graded20k", "cube16", "annulus_mixed"):
        pytest.skip("three cases cover the loops")
    uo, ito, info = H.solve(f, 1e-8, record=True)
    S = A.Solver(c["coords"], c["elems"], c["kappa"], red_blocks=blocks, **S64.kwargs)
    u, it, tr = S.solve(f, 1e-8)
    near = any(abs(h - 1e-8) < 1e-3 * 1e-8 for h in info["history"][-2:])
    _say(name, f"red_blocks={blocks}: iters gpu {it} oracle {ito}, element-wise {_rel_inf(u, uo):.2e}")
    assert it == ito or near
    assert tr <= 1e-8 * (1 + 1e-6)
    assert _rel_inf(u, uo) <= 1e-10
    S.set_precision(A.PREC_MIXED)
    um, itm, trm = S.solve(f, 1e-8)
    ref, _, _ = H.solve(f, 1e-12)
    assert trm <= 1e-8 and _rel_inf(um, ref) <= 1e-6


def test_solve_device_matches_host_and_is_deterministic(case):
    name, c, H, S64, S32, f = case
    u1, it1, _ = S64.solve(f, 1e-8)
    fd = torch.from_numpy(f).cuda()
    u2, it2, _ = S64.solve_device(fd, 1e-8)
    u3, it3, _ = S64.solve_device(fd, 1e-8)
    assert it1 == it2 == it3
    assert np.array_equal(u1, u2.cpu().numpy())
    assert torch.equal(u2, u3)


def test_solve_mixed(case):
    name, c, H, S64, S32, f = case
    ref, _, _ = H.solve(f, 1e-12)
    u, it, tr = S32.solve(f, 1e-8)
    u64, it64, _ = S64.solve(f, 1e-8)
    err = _rel(u, ref)
    _say(name, "mixed iters", it, "fp64 iters", it64, "err vs 1e-12 oracle", err, "fp64 err", _rel(u64, ref),
         "element-wise", _rel_inf(u, ref))
    assert tr <= 1e-8
    assert err <= 1e-6
    assert _rel_inf(u, ref) <= 1e-6


def test_zero_rhs_and_max_iter(case):
    name, c, H, S64, S32, f = case
    u, it, tr = S64.solve(np.zeros(H.n), 1e-8)
    assert it == 0 and np.all(u == 0)
    S1 = A.Solver(c["coords"], c["elems"], c["kappa"], max_iter=2, **S64.kwargs)
    with pytest.raises(A.AsmgError) as e:
        S1.solve(f, 1e-14)
    assert e.value.code == A.ENOCONV
    u, it, tr = S1.solve(f, 1e-14, allow_noconv=True)
    assert it == 2


def test_autotuned_shapes_do_not_change_b_co(case):
    # B_co before any solve (default launch shapes) and after the first solve (autotuned shapes)
    # is bitwise identical: the tuned kernels have no reductions
    name, c, H, S64, S32, f = case
    S = A.Solver(c["coords"], c["elems"], c["kappa"], **S64.kwargs)
    r = torch.from_numpy(np.random.default_rng(9).standard_normal(S.n)).cuda()
    assert len(S.tuned_shapes()) == 0
    z0 = S.apply_preconditioner(r).cpu().numpy()
    S.solve_device(torch.from_numpy(f).cuda(), 1e-8)
    shapes = S.tuned_shapes()
    assert len(shapes) > 0 and set(shapes[:, 0].tolist()) <= {128, 256, 512}
    assert set(shapes[:, 2].tolist()) <= {0, 1}
    assert S.tune_times().shape == (len(shapes), A.N_SHAPES)
    z1 = S.apply_preconditioner(r).cpu().numpy()
    assert np.array_equal(z0, z1)


def test_kernel_timing_leaves_the_solver_intact():
    # asmg_time_kernel: SpMV, B_co as graph replays (both precisions), colour passes with
    # kernel-stamped events; all positive, and a solve afterwards is unchanged
    c = W.make_config(1, scale=0.01)
    S = A.Solver(c["coords"], c["elems"], c["kappa"])
    f = c["f_vertex"][S.dof_vertex()]
    u0, it0, _ = S.solve(f, 1e-8)
    # mode 7 (the LDS-staged product) first checks its result against the solve's product
    for which, prec in ((0, A.PREC_FP64), (6, A.PREC_FP64), (7, A.PREC_FP64), (2, A.PREC_FP64), (2, A.PREC_MIXED),
                        (4, A.PREC_FP64)):
        ms, by = S.time_kernel(which, reps=20, precision=prec)
        _say("time_kernel", which, prec, f"{ms * 1e3:.1f} us, {by / 1e6:.2f} MB")
        assert 0 < ms < 1e3 and by > 0
    u1, it1, _ = S.solve(f, 1e-8)
    assert it1 == it0 and np.array_equal(u1, u0)
