"""GPU parity of the nested-iteration start (asmg_options.nested) against the oracle.

Bar: the same PCG iteration count as the oracle started from its own nested guess, and
||u_gpu - u_oracle|| <= 1e-10 ||u_oracle|| in FP64; mixed precision within 1e-6 of the oracle
solved to 1e-12 with its true residual at the tolerance.
"""
import sys

import numpy as np
import pytest
import scipy.sparse.linalg as sla

import workloads as W
from oracle.hierarchy import Hierarchy

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
A = pytest.importorskip("paper_1410_2153_amd")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _lshape():
    coords, elems, _ = W.lshape_mesh(96, 0.3)
    c = dict(coords=coords, elems=elems, kappa=np.exp(np.random.default_rng(2).normal(0, 0.5, len(elems))))
    c["f_vertex"] = W.rhs_per_vertex(len(coords), 5, 1)
    return c, 1


def _annulus_mixed():
    from oracle.domain import boundary_vertices
    coords, elems, _ = W.annulus_mesh(200)
    c = dict(coords=coords, elems=elems, kappa=np.exp(np.random.default_rng(3).normal(0, 0.5, len(elems))))
    c["f_vertex"] = W.rhs_per_vertex(len(coords), 6, 1)
    c["dirichlet"] = boundary_vertices(elems, len(coords)) & (np.hypot(coords[:, 0] - 0.5, coords[:, 1] - 0.5) > 0.35)
    return c, 2


# name -> (workload, domain: 0 root box, 1 mesh domain, 2 mixed Dirichlet/Neumann grids)
CASES = {
    "square64": lambda: (W.make_config(0), 0),
    "graded20k": lambda: (W.make_config(1, scale=0.01), 0),
    "cube16": lambda: (W.make_config(2, scale=1 / 8), 0),
    "lshape_domain": _lshape,
    "annulus_mixed": _annulus_mixed,
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    _say(f"[gpu nested] case {request.param}")
    c, dom = CASES[request.param]()
    H = Hierarchy(c["coords"], c["elems"], c["kappa"], dirichlet=c.get("dirichlet"), domain=["box", "mesh", "mixed"][dom])
    f = c["f_vertex"][H.dofs]
    return request.param, c, H, dom, f


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("cycles", [1, 2])
def test_nested_fp64(case, cycles):
    name, c, H, dom, f = case
    S = A.Solver(c["coords"], c["elems"], c["kappa"], c.get("dirichlet"), domain=dom, nested=cycles)
    uo, ito, info = H.solve(f, 1e-8, nested=cycles)
    u, it, tr = S.solve(f, 1e-8)
    u0, it0, _ = H.solve(f, 1e-8)
    _say(name, f"nested={cycles}: iterations gpu {it} oracle {ito} (from 0: {it0}), rel diff {_rel(u, uo):.2e}")
    assert it == ito
    assert _rel(u, uo) <= 1e-10
    assert np.abs(u - uo).max() <= 1e-10 * np.abs(uo).max()
    assert tr <= 1e-8
    # the start's residual kernel (k_cg_guess) with its grid-stride loop over a capped grid
    Sg = A.Solver(c["coords"], c["elems"], c["kappa"], c.get("dirichlet"), domain=dom, nested=cycles, red_blocks=5)
    ug, itg, _ = Sg.solve(f, 1e-8)
    assert itg == ito and np.abs(ug - uo).max() <= 1e-10 * np.abs(uo).max()
    # a second solve on the same handle: zero right-hand side, then the first one again
    z, itz, trz = S.solve(np.zeros_like(f), 1e-8)
    assert itz == 0 and not np.any(z)
    u2, it2, _ = S.solve(f, 1e-8)
    assert it2 == it and _rel(u2, uo) <= 1e-10


def test_nested_mixed(case):
    name, c, H, dom, f = case
    S = A.Solver(c["coords"], c["elems"], c["kappa"], c.get("dirichlet"), domain=dom, nested=1,
                 precision=A.PREC_MIXED)
    u, it, tr = S.solve(f, 1e-8)
    uo, _, _ = H.solve(f, 1e-12)
    _say(name, f"nested mixed: iterations {it}, true rel residual {tr:.2e}, rel diff {_rel(u, uo):.2e}")
    assert tr <= 1e-8
    assert _rel(u, uo) <= 1e-6


def test_guess_that_meets_the_rule():
    # uniform 32^2: the bottom is the finest auxiliary grid, the guess is the discrete solution
    X, T, _ = W.square_mesh(32, jitter=0.0)
    H = Hierarchy(X, T, np.ones(len(T)))
    assert H.aux.J == H.aux.lc
    f = W.rhs_per_vertex(len(X), 0, 7)[H.dofs]
    uh = sla.spsolve(H.A.tocsc(), f)
    for prec in (A.PREC_FP64, A.PREC_MIXED):
        S = A.Solver(X, T, np.ones(len(T)), nested=1, precision=prec)
        S.solve(np.random.default_rng(1).standard_normal(S.n), 1e-8)   # leaves an iteration history
        u, it, tr = S.solve(f, 1e-8 if prec == A.PREC_FP64 else 1e-3)   # FP32 guess: ~1e-6 accurate
        _say(f"[gpu nested] 32^2 precision {prec}: iterations {it}, rel diff {_rel(u, uh):.2e}")
        assert it == 0
        assert _rel(u, uh) <= (1e-12 if prec == A.PREC_FP64 else 1e-5)
