"""asmg_solve_device_noalloc (through the C ABI) against asmg_solve_device.

The entry point keeps the PCG control block and the reduction partials in the library's static
per-GPU scratch and allocates nothing. Bar: the same iteration count and u bit for bit (the same
kernels with the same grids run; only the address of the control block and partials differs).
Two calls in a row on two handles, the second with the smaller system, in both precisions; a
nested-start handle; a host-only handle is refused.
"""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
A = pytest.importorskip("paper_1410_2153_amd")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _handle(cfg, scale, **kw):
    c = W.make_config(cfg, scale=scale)
    S = A.Solver(c["coords"], c["elems"], c["kappa"], **kw)
    f = torch.from_numpy(np.ascontiguousarray(c["f_vertex"][S.dof_vertex()])).cuda()
    return S, f


@pytest.mark.parametrize("prec", [A.PREC_FP64, A.PREC_MIXED])
def test_noalloc_matches_solve_device(prec):
    _say(f"[no-alloc] precision {prec}: graded 10k then square 64^2")
    big, fb = _handle(1, 0.01, precision=prec)
    small, fs = _handle(0, 1.0, precision=prec)
    assert small.n < big.n
    # the entry point first (fresh handles: default launch shapes, no graph yet), twice in a row
    ub = torch.empty_like(fb)
    us = torch.empty_like(fs)
    _, itb, trb = big.solve_device_noalloc(fb, ub, 1e-8)
    _, its, trs = small.solve_device_noalloc(fs, us, 1e-8)
    # the allocating entry point (graph, autotuned shapes), then the scratch entry point again
    rb, itb2, trb2 = big.solve_device(fb, 1e-8)
    rs, its2, trs2 = small.solve_device(fs, 1e-8)
    _say(f"  noalloc iterations {itb}/{its}, solve_device {itb2}/{its2}")
    assert (itb, its) == (itb2, its2)
    assert torch.equal(ub, rb) and torch.equal(us, rs)
    assert trb == trb2 and trs == trs2 and trb <= 1e-8 and trs <= 1e-8
    ub2 = torch.empty_like(fb)
    us2 = torch.empty_like(fs)
    _, itb3, _ = big.solve_device_noalloc(fb, ub2, 1e-8)
    _, its3, _ = small.solve_device_noalloc(fs, us2, 1e-8)
    assert (itb3, its3) == (itb, its)
    assert torch.equal(ub2, rb) and torch.equal(us2, rs)
    # the handle's own solve is untouched by the scratch calls in between
    rb2, itb4, _ = big.solve_device(fb, 1e-8)
    assert itb4 == itb and torch.equal(rb2, rb)


def test_noalloc_nested_start_and_zero_rhs():
    S, f = _handle(1, 0.01, nested=1)
    u, it, _ = S.solve_device(f, 1e-8)
    v = torch.empty_like(f)
    _, it2, _ = S.solve_device_noalloc(f, v, 1e-8)
    assert it2 == it and torch.equal(u, v)
    z = torch.zeros_like(f)
    _, itz, trz = S.solve_device_noalloc(z, v, 1e-8)
    assert itz == 0 and not bool(v.any())


def test_noalloc_refuses_host_only_handles():
    c = W.make_config(0)
    S = A.Solver(c["coords"], c["elems"], c["kappa"], device=-1)
    f = torch.zeros(S.n, dtype=torch.float64, device="cuda")
    with pytest.raises(A.AsmgError) as e:
        S.solve_device_noalloc(f, torch.empty_like(f), 1e-8)
    assert e.value.code == A.EDEVICE
