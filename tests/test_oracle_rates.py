"""Pins of the preconditioner's quality against the paper's reported behaviour (Section 5.2):
the stationary iteration u <- u + B_co (f - A u) contracts at a rate of about 0.4 (Dirichlet
problem), independent of the level, and the auxiliary hierarchy costs a few times the storage of
A (Tables 2-3 report 2-6x in bytes). The multicolour Gauss-Seidel and symmetric V-cycle used here
contract somewhat faster than the paper's sequential smoother; a wrong sign, a dropped transfer
or a broken smoother gives rates near 1 or divergence."""
import numpy as np
import pytest

import workloads as W
from oracle.hierarchy import Hierarchy


def _rate(H, its=12):
    # asymptotic contraction of the error iteration e <- (I - B_co A) e in the A-norm
    B, A = H.preconditioner(), H.A
    e = np.random.default_rng(0).standard_normal(H.n)
    norm = lambda v: float(np.sqrt(v @ (A @ v)))
    ns = [norm(e)]
    for _ in range(its):
        e = e - B(A @ e)
        ns.append(norm(e))
    return (ns[-1] / ns[4]) ** (1.0 / (its - 4))


def _aux_nnz_ratio(H):
    aux = sum(H.aux.A[l].nnz for l in H.aux.A) + sum(H.aux.P[l].nnz for l in H.aux.P) + H.Pi.nnz
    return aux / H.A.nnz


@pytest.mark.parametrize("family", ["square", "graded"])
def test_stationary_rate_is_small_and_level_independent(family):
    if family == "square":
        hs = []
        for n in (64, 128):
            X, T, _ = W.square_mesh(n, jitter=0.3)
            hs.append(Hierarchy(X, T, np.ones(len(T))))
    else:
        hs = [Hierarchy(c["coords"], c["elems"], c["kappa"])
              for c in (W.make_config(1, scale=s) for s in (0.004, 0.01))]
    rates = [_rate(H) for H in hs]
    assert all(r < 0.45 for r in rates), rates
    assert rates[1] <= rates[0] + 0.1, rates      # no growth with the number of levels
    ratios = [_aux_nnz_ratio(H) for H in hs]
    assert all(1.0 <= q <= 8.0 for q in ratios), ratios
