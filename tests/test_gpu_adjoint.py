"""Adjoint gradient on the GPU (element kernel + second PCG solve) against the oracle and finite differences."""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint, fem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
A = pytest.importorskip("paper_1410_2153_amd")


def test_element_gradient_kernel_matches_oracle():
    coords, elems, _ = W.square_mesh(24, 0.3, cfg=4, item=1)
    rng = np.random.default_rng(0)
    kappa = np.exp(rng.normal(0, 0.3, len(elems)))
    S = A.Solver(coords, elems, kappa)
    u = rng.standard_normal(S.n)
    lam = rng.standard_normal(S.n)
    g = S.element_gradient(torch.from_numpy(u).cuda(), torch.from_numpy(lam).cuda()).cpu().numpy()
    uv = np.zeros(len(coords))
    lv = np.zeros(len(coords))
    dofs = S.dof_vertex()
    uv[dofs] = u
    lv[dofs] = lam
    ref = fem.element_gradient_of_energy(coords, elems, kappa, uv, lv)
    assert np.abs(g - ref).max() <= 1e-12 * np.abs(ref).max()


def test_autograd_gradient_vs_oracle_and_fd():
    c = W.make_config(4, scale=24 / 724)
    coords, elems = c["coords"], c["elems"]
    m = torch.tensor(c["m"], dtype=torch.float64, device="cuda", requires_grad=True)
    S = A.Solver(coords, elems, np.exp(c["m"]))
    dofs = S.dof_vertex()
    f = torch.tensor(c["f_vertex"][dofs], device="cuda")
    # observations: solve at the second coefficient plus noise (oracle direct solve)
    Aobs, _ = fem.assemble(coords, elems, np.exp(c["m_obs"]))
    import scipy.sparse.linalg as sla
    u_obs = sla.spsolve(Aobs.tocsc(), c["f_vertex"][dofs]) + c["noise_vertex"][dofs]
    uo = torch.tensor(u_obs, device="cuda")
    Fn = A.LogCoefficientSolve.function()
    u = Fn.apply(m, f, S, 1e-12)
    J = 0.5 * ((u - uo) ** 2).sum()
    J.backward()
    g = m.grad.cpu().numpy()
    J0, gref, _ = adjoint.loss_and_gradient(coords, elems, c["m"], c["f_vertex"][dofs], u_obs)
    assert abs(J.item() - J0) <= 1e-9 * abs(J0)
    assert np.abs(g - gref).max() <= 1e-8 * np.abs(gref).max()
    for d in c["directions"][:5]:
        eps = 1e-6
        Jp = adjoint.loss_and_gradient(coords, elems, c["m"] + eps * d, c["f_vertex"][dofs], u_obs)[0]
        Jm = adjoint.loss_and_gradient(coords, elems, c["m"] - eps * d, c["f_vertex"][dofs], u_obs)[0]
        assert (Jp - Jm) / (2 * eps) == pytest.approx(g @ d, rel=1e-5)


def test_set_coefficient_device_refreshes_operator():
    import scipy.sparse.linalg as sla
    c = W.make_config(1, scale=0.01)
    coords, elems = c["coords"], c["elems"]
    S = A.Solver(coords, elems, c["kappa"])
    k2 = np.exp(np.random.default_rng(9).normal(0, 0.7, len(elems)))
    S.set_coefficient_device(torch.from_numpy(k2).cuda())
    A2, dofs = fem.assemble(coords, elems, k2)
    x = np.random.default_rng(1).standard_normal(S.n)
    y = S.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    assert np.linalg.norm(y - A2 @ x) <= 1e-14 * np.linalg.norm(A2 @ x)
    f = c["f_vertex"][dofs]
    for prec in (A.PREC_FP64, A.PREC_MIXED):
        S.set_precision(prec)
        u, it, tr = S.solve(f, 1e-10)
        assert np.linalg.norm(f - A2 @ u) <= 1e-10 * (1 + 1e-6) * np.linalg.norm(f)
        ref = sla.spsolve(A2.tocsc(), f)
        assert np.linalg.norm(u - ref) <= 1e-7 * np.linalg.norm(ref)
    lam = np.random.default_rng(2).standard_normal(S.n)
    g = S.element_gradient(torch.from_numpy(u).cuda(), torch.from_numpy(lam).cuda()).cpu().numpy()
    uv = np.zeros(len(coords))
    lv = np.zeros(len(coords))
    uv[dofs] = u
    lv[dofs] = lam
    assert np.abs(g - fem.element_gradient_of_energy(coords, elems, k2, uv, lv)).max() <= 1e-12 * np.abs(g).max()


def test_set_coefficient_device_twice_after_a_solve():
    # the refresh maps are built at the first refresh (here after a solve) and reused
    c = W.make_config(1, scale=0.01)
    coords, elems = c["coords"], c["elems"]
    S = A.Solver(coords, elems, c["kappa"])
    f = c["f_vertex"][S.dof_vertex()]
    S.solve(f, 1e-8)
    for seed in (10, 11):
        k = np.exp(np.random.default_rng(seed).normal(0, 0.7, len(elems)))
        S.set_coefficient_device(torch.from_numpy(k).cuda())
        Ak, dofs = fem.assemble(coords, elems, k)
        x = np.random.default_rng(seed).standard_normal(S.n)
        y = S.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
        assert np.linalg.norm(y - Ak @ x) <= 1e-14 * np.linalg.norm(Ak @ x)
        u, it, tr = S.solve(f, 1e-10)
        assert np.linalg.norm(f - Ak @ u) <= 1e-10 * (1 + 1e-6) * np.linalg.norm(f)


def test_log_coefficient_entry_points():
    # kappa = exp(m) and the adjoint sign are computed in the library
    c = W.make_config(4, scale=24 / 724)
    coords, elems = c["coords"], c["elems"]
    S = A.Solver(coords, elems, np.ones(len(elems)))
    m = torch.tensor(c["m"], device="cuda")
    S.set_log_coefficient_device(m)
    Am, dofs = fem.assemble(coords, elems, np.exp(c["m"]))
    x = np.random.default_rng(3).standard_normal(S.n)
    y = S.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    assert np.linalg.norm(y - Am @ x) <= 1e-14 * np.linalg.norm(Am @ x)
    u = torch.from_numpy(np.random.default_rng(4).standard_normal(S.n)).cuda()
    lam = torch.from_numpy(np.random.default_rng(5).standard_normal(S.n)).cuda()
    g = S.adjoint_gradient(u, lam)
    assert torch.equal(g, -S.element_gradient(u, lam))


def test_backward_after_a_second_forward_on_the_same_solver():
    # two forwards at m1 and m2 on one solver, then backward of J(u(m1)) alone: the gradient is
    # the oracle's at m1 (backward restores A(exp(m1)) before its adjoint solve)
    c = W.make_config(4, scale=24 / 724)
    coords, elems = c["coords"], c["elems"]
    S = A.Solver(coords, elems, np.exp(c["m"]))
    dofs = S.dof_vertex()
    f = torch.tensor(c["f_vertex"][dofs], device="cuda")
    Aobs, _ = fem.assemble(coords, elems, np.exp(c["m_obs"]))
    import scipy.sparse.linalg as sla
    u_obs = sla.spsolve(Aobs.tocsc(), c["f_vertex"][dofs]) + c["noise_vertex"][dofs]
    uo = torch.tensor(u_obs, device="cuda")
    Fn = A.LogCoefficientSolve.function()
    m1 = torch.tensor(c["m"], device="cuda", requires_grad=True)
    m2 = torch.tensor(c["m_obs"], device="cuda", requires_grad=True)
    u1 = Fn.apply(m1, f, S, 1e-12)
    u2 = Fn.apply(m2, f, S, 1e-12)
    J1 = 0.5 * ((u1 - uo) ** 2).sum()
    J1.backward()
    _, gref, _ = adjoint.loss_and_gradient(coords, elems, c["m"], c["f_vertex"][dofs], u_obs)
    g = m1.grad.cpu().numpy()
    assert np.abs(g - gref).max() <= 1e-8 * np.abs(gref).max()
    assert m2.grad is None
    # the later backward of J(u(m2)) is right too
    J2 = 0.5 * ((u2 - uo) ** 2).sum()
    J2.backward()
    _, gref2, _ = adjoint.loss_and_gradient(coords, elems, c["m_obs"], c["f_vertex"][dofs], u_obs)
    assert np.abs(m2.grad.cpu().numpy() - gref2).max() <= 1e-8 * np.abs(gref2).max()
