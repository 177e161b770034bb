"""The restart of PCG from the true residual (Section 5.2 solve; the rule of the oracle's pcg),
driven on both sides at a tolerance below the FP64 floor of the true residual.

At tol = 1e-15 the recursively updated residual meets the rule while f - A u stays at about
1.5e-15 relative: both sides restart 3 times and return with the true residual above tol.
Bar: the same number of restarts; the same iteration count, except where the oracle's updated
residual lies within 1e-3 relative of tol at the crossing (the summation order may move the
crossing by one iteration); u within 1e-10 relative. With the iteration budget spent at the
crossing both sides end unconverged (ENOCONV).
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


def _near(hist, tol):
    return any(abs(h - tol) < 1e-3 * tol for h in hist)


@pytest.mark.parametrize("cfg,scale", [(0, 1.0), (1, 0.01)])
@pytest.mark.parametrize("prec", [0, 1])
def test_restarts_match_the_oracle(cfg, scale, prec):
    _say(f"[gpu restart] config {cfg} scale {scale} precision {prec}")
    c = W.make_config(cfg, scale=scale)
    H = Hierarchy(c["coords"], c["elems"], c["kappa"])
    f = c["f_vertex"][H.dofs]
    uo, ito, info = H.solve(f, 1e-15, mixed=bool(prec), record=True)
    S = A.Solver(c["coords"], c["elems"], c["kappa"], precision=prec)
    u, it, tr = S.solve(f, 1e-15)
    it2, rs = S.solve_stats()
    err = np.linalg.norm(u - uo) / np.linalg.norm(uo)
    _say(f"  oracle {ito} iterations {info['restarts']} restarts, gpu {it} iterations {rs} restarts, "
         f"true residual {tr:.2e}, rel diff {err:.2e}")
    assert it2 == it
    assert rs == info["restarts"] == 3
    assert it == ito or _near(info["history"], 1e-15)
    assert tr > 1e-15
    assert err <= 1e-10


@pytest.mark.parametrize("prec", [0, 1])
def test_restart_with_spent_budget_is_noconv(prec):
    c = W.make_config(0)
    H = Hierarchy(c["coords"], c["elems"], c["kappa"])
    f = c["f_vertex"][H.dofs]
    _, _, info = H.solve(f, 1e-15, mixed=bool(prec), record=True)
    first = next(k for k, h in enumerate(info["history"]) if h <= 1e-15) + 1
    if _near(info["history"][first - 2:first], 1e-15):
        pytest.skip("crossing within rounding of tol")
    _, it_o, info_o = H.solve(f, 1e-15, mixed=bool(prec), max_iter=first)
    assert info_o["status"] == "noconv"
    S = A.Solver(c["coords"], c["elems"], c["kappa"], precision=prec, max_iter=first)
    with pytest.raises(A.AsmgError) as e:
        S.solve(f, 1e-15)
    assert e.value.code == A.ENOCONV
    u, it, tr = S.solve(f, 1e-15, allow_noconv=True)
    assert it == it_o == first and tr > 1e-15
