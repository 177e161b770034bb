"""Benchmark: DOF-solves/s of the ASMG-preconditioned CG solve on one MI355X.

Headline workload: 256 independent jittered square meshes of the unit square, sides drawn
uniformly from 32..512 (22.3 M unknowns in all), 4 right-hand sides each, f ~ U[-1, 1],
kappa = 1, homogeneous Dirichlet data, solved together by the batched engine. A step is one
batched solve of all 1024 systems, from F resident in HBM to U resident in HBM, every system
stopping at ||r|| <= 1e-8 ||f||. `value` is the FP64 solve; `mixed` the FP32-preconditioner
solve inside FP64 CG.

Beside it: the graded unstructured 2-D mesh (1.0 M unknowns), the 3-D Kuhn cube (2.0 M
unknowns), the adjoint gradient (0.52 M unknowns) and a general-domain annulus, each with its
own figures; `roofline` is for the dominant kernel of the headline solve (the batched
Gauss-Seidel colour pass), timed per launch with HIP events inside the library on torch's
stream; the graded and cube workloads carry their own roofline entries. `cpu_baseline` times
the FP64 oracle on a bounded sample of the headline's meshes on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def load_workload(scale: float):
    import workloads as W
    cache = os.path.join(os.environ.get("TMPDIR", "/tmp"), f"asmg_cfg1_{scale:g}.npz")
    if os.path.exists(cache):
        z = np.load(cache)
        return {k: z[k] for k in z.files}
    c = W.make_config(1, scale=scale)
    out = dict(coords=c["coords"], elems=c["elems"], kappa=c["kappa"], f_vertex=c["f_vertex"])
    try:
        np.savez(cache, **out)
    except OSError:
        pass
    return out


def counter_record(workload: str):
    """The committed hardware-counter record of a workload (HBM bytes per launch of its dominant
    kernel and per B_co application), if that kernel's code has not changed since the counters
    were taken (else {})."""
    from paper_1410_2153_amd.counters import WORKLOADS, _srcs, source_key
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return {}
    return rec if rec.get("kernel_code_key") == source_key(_srcs(*WORKLOADS[workload]["sources"])) else {}


def cpu_baseline(budget_s: float = 20.0, n_meshes: int = 256):
    """Oracle solve phase on a bounded sample of the headline workload: the smallest meshes of the
    256-mesh batch (their 4 right-hand sides each), FP64 PCG to 1e-8, one thread (BLAS thread
    pools limited to 1 for the timed region), repeated until about `budget_s` seconds."""
    from threadpoolctl import threadpool_limits

    import workloads as W
    from oracle.hierarchy import Hierarchy
    sides = W.rng(3, W.S_SIDES, 0).integers(32, 512 + 1, n_meshes)
    order = np.argsort(sides, kind="stable")[:4]
    ms = W.batched_config(n_meshes=n_meshes)
    sample = [ms[int(m)] for m in order]
    hs = [Hierarchy(m["coords"], m["elems"], m["kappa"]) for m in sample]
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    dofs = 0
    with threadpool_limits(limits=1):
        for H, m in zip(hs, sample):
            H.solve(m["f_vertex"][0, H.dofs], 1e-8)  # warm-up (builds the per-colour slices)
        t0 = time.perf_counter()
        reps = 0
        while True:
            for H, m in zip(hs, sample):
                for r in range(4):
                    H.solve(m["f_vertex"][r, H.dofs], 1e-8)
                    dofs += H.n
            reps += 1
            if time.perf_counter() - t0 > budget_s:
                break
        dt = time.perf_counter() - t0
    return dict(value=dofs / dt, unit="DOF-solves/s", cores=1, kind="oracle", cpu_model=model,
                sample=f"the {len(hs)} smallest meshes of the 256-mesh batch (sides "
                       f"{[int(sides[m]) for m in order]}, {sum(H.n for H in hs)} unknowns) x 4 right-hand sides, "
                       f"FP64 oracle PCG to 1e-8, {reps} rounds in {dt:.1f} s, 1 thread of "
                       f"{len(os.sched_getaffinity(0))}")


def batched(n_meshes: int, steps: int, warmup: int, kernel_timing: bool = True, autotune: int = 1):
    """The batched workload: n_meshes jittered squares, sides ~ U{32..512}, 4 right-hand sides each,
    all (mesh, rhs) systems solved together. A step is one batched solve, F resident in HBM to U
    resident in HBM, every system to ||r|| <= 1e-8 ||f||."""
    import torch

    import paper_1410_2153_amd as A
    import workloads as W
    t0 = time.perf_counter()
    ms = W.batched_config(n_meshes=n_meshes)
    log(f"batched: generated {n_meshes} meshes in {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    B = A.BatchSolver([(m["coords"], m["elems"], m["kappa"]) for m in ms], precision=A.PREC_FP64,
                      autotune=autotune)
    t_setup = time.perf_counter() - t0
    log(f"batched: setup {t_setup:.1f} s, {B.n_total} unknowns")
    # right-hand sides per unknown, [mesh][rhs][unknown]
    F = []
    for m, mesh in enumerate(ms):
        bnd = W.boundary_vertices(mesh["coords"])
        F.append(mesh["f_vertex"][:, ~bnd].ravel())
    F = torch.from_numpy(np.concatenate(F)).cuda()
    sides = [int(m["n"]) for m in ms]
    res = {"workload": f"{n_meshes} jittered square meshes, side ~ U{{32..512}}, 4 right-hand sides each, "
                       f"{B.n_total} unknowns, kappa=1, f~U[-1,1], every system PCG to 1e-8 from u0=0",
           "meshes": n_meshes, "rhs": 4, "unknowns": B.n_total, "sides_min_max": [min(sides), max(sides)],
           "setup_s": t_setup}
    U = torch.empty_like(F)
    for name, prec in (("fp64", A.PREC_FP64), ("mixed", A.PREC_MIXED)):
        B.set_precision(prec)
        for _ in range(max(warmup, 1)):
            U, its, tr = B.solve(F, 4, 1e-8, out=U)
        torch.cuda.synchronize()
        per = []
        t = time.perf_counter()
        for _ in range(steps):
            t1 = time.perf_counter()
            U, its, tr = B.solve(F, 4, 1e-8, out=U)   # returns once U is in device memory
            per.append((time.perf_counter() - t1) * 1e3)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / steps
        res[name] = {"value": B.n_total * 4 / dt, "ms_per_step": dt * 1e3, "ms_per_step_median": float(np.median(per)),
                     "max_iterations": int(its.max()), "max_true_rel_residual": float(tr.max())}
        log(f"batched {name}: {dt * 1e3:.1f} ms per batch ({B.n_total * 4 / dt:.3e} DOF-solves/s), "
            f"iterations <= {its.max()}")
    B.set_precision(A.PREC_FP64)
    if kernel_timing:
        vc = {}
        for key, prec in (("fp64", A.PREC_FP64), ("fp32", A.PREC_MIXED)):
            m_b, b_b = B.time_kernel(0, 4, reps=20, precision=prec)
            vc[key] = {"ms": m_b, "model_bytes": b_b, "GBs": b_b / m_b / 1e6, "frac_of_peak": b_b / m_b / 1e6 / HBM_PEAK_GBS}
        res["vcycle_4rhs"] = vc
        ms_gs, by_gs = B.time_kernel(1, 4, reps=3, precision=A.PREC_FP64)
        res["gs_pass"] = {"ms_per_launch": ms_gs, "bytes_per_launch": by_gs}
    shapes = B.tuned_shapes(4, A.PREC_FP64)
    res["tuned_launch_shapes_fp64_4rhs"] = {
        f"{t}x{'xcd' if x else 'rr'}/var{o}": int(((shapes[:, 0] == t) & (shapes[:, 1] == x) & (shapes[:, 2] == o)).sum())
        for t, x, o in sorted(set(map(tuple, shapes.tolist())))}
    tt = B.tune_times(4, A.PREC_FP64)
    if len(tt):
        # per candidate: the sum over launch sites of its best time, against the default's
        res["tune_sum_ms_fp64_4rhs"] = {f"{t}x{'xcd' if x else 'rr'}/var{o}": float(tt[:, k][tt[:, k] > 0].sum())
                                        for k, (t, x, o) in enumerate(A.SHAPES)}
    del B
    # the same systems solved one at a time with the single-mesh engine, on a sample of meshes
    sample = list(range(0, n_meshes, max(1, n_meshes // 16)))
    tot_dofs, tot_t = 0, 0.0
    for m in sample:
        mesh = ms[m]
        S = A.Solver(mesh["coords"], mesh["elems"], mesh["kappa"])
        dofs = S.dof_vertex()
        for r in range(4):
            f = torch.from_numpy(np.ascontiguousarray(mesh["f_vertex"][r, dofs])).cuda()
            S.solve_device(f, 1e-8)
            torch.cuda.synchronize()
            t = time.perf_counter()
            S.solve_device(f, 1e-8)
            torch.cuda.synchronize()
            tot_t += time.perf_counter() - t
            tot_dofs += S.n
        del S
    res["single_solves_fp64_sample"] = {"value": tot_dofs / tot_t, "meshes": len(sample), "rhs": 4}
    log(f"single-mesh solves (sample of {len(sample)} meshes x 4 rhs): {tot_dofs / tot_t:.3e} DOF-solves/s")
    return res


def cube3d(steps: int, colouring: int = 2, kernel_timing: bool = True, autotune: int = 1):
    """3-D workload: 128^3 cubes x 6 Kuhn tetrahedra, jittered, kappa in {1, 10} on an 8^3 checkerboard."""
    import torch

    import paper_1410_2153_amd as A
    import workloads as W
    c = W.make_config(2)
    t0 = time.perf_counter()
    S = A.Solver(c["coords"], c["elems"], c["kappa"], colouring=colouring, autotune=autotune)
    t_setup = time.perf_counter() - t0
    dofs = S.dof_vertex()
    f = torch.from_numpy(np.ascontiguousarray(c["f_vertex"][dofs])).cuda()
    res = {"workload": c["name"], "unknowns": S.n, "setup_s": t_setup, "J": S.info()["J"]}
    for name, prec in (("fp64", A.PREC_FP64), ("mixed", A.PREC_MIXED)):
        S.set_precision(prec)
        u, it, tr = S.solve_device(f, 1e-8)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            u, it, tr = S.solve_device(f, 1e-8, out=u)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / steps
        res[name] = {"value": S.n / dt, "ms_per_step": dt * 1e3, "iterations": it, "true_rel_residual": tr}
        log(f"cube3d {name}: {dt * 1e3:.2f} ms/solve, {it} iterations ({S.n / dt:.3e} DOF-solves/s)")
    if kernel_timing:
        ms_b, by_b = S.time_kernel(2, reps=20, precision=A.PREC_FP64)
        res["preconditioner_fp64"] = {"ms": ms_b, "model_bytes": by_b, "GBs": by_b / ms_b / 1e6,
                                      "frac_of_peak": by_b / ms_b / 1e6 / HBM_PEAK_GBS}
        ms_b, by_b = S.time_kernel(2, reps=20, precision=A.PREC_MIXED)
        res["preconditioner_fp32"] = {"ms": ms_b, "model_bytes": by_b, "GBs": by_b / ms_b / 1e6,
                                      "frac_of_peak": by_b / ms_b / 1e6 / HBM_PEAK_GBS}
        for key, mode in (("fine_spmv_fp64", 6), ("fine_spmv_lds_staged_fp64", 7)):
            ms_k, by_k = S.time_kernel(mode, reps=50)
            res[key] = {"ms": ms_k, "model_bytes": by_k, "GBs": by_k / ms_k / 1e6}
        ms_gs, by_gs = S.time_kernel(4, reps=10, precision=A.PREC_FP64)
        rec = counter_record("cube2M")
        res["roofline"] = {"bound": "hbm", "kernel": "asmg::k_sell<0, double, VAR> (Gauss-Seidel colour pass, sliced ELL; VAR = the variant tuned per launch site; traffic from a run with the default, VAR 0)",
                           "achieved": by_gs / ms_gs / 1e6, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": by_gs / ms_gs / 1e6 / HBM_PEAK_GBS, "traffic": rec.get("traffic_bytes_per_launch"),
                           "bytes_per_launch": by_gs, "ms_per_launch": ms_gs}
    return res


def annulus(steps: int, colouring: int = 2):
    """General-domain workload (Section 3.4 Dirichlet grids on the mesh's own domain): an annulus
    (radii 0.2 and 0.5) of about 0.87 M vertices, kappa = exp(N(0, 0.5^2)), f ~ U[-1, 1]."""
    import torch

    import paper_1410_2153_amd as A
    import workloads as W
    t0 = time.perf_counter()
    coords, elems, dirichlet = W.annulus_mesh(3600)
    kappa = np.exp(W.rng(6, W.S_COEF, 0).normal(0.0, 0.5, len(elems)))
    f_vertex = W.rhs_per_vertex(len(coords), 6, 0)
    log(f"annulus: mesh {len(coords)} vertices in {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    S = A.Solver(coords, elems, kappa, dirichlet, colouring=colouring, domain=1)
    t_setup = time.perf_counter() - t0
    dofs = S.dof_vertex()
    f = torch.from_numpy(np.ascontiguousarray(f_vertex[dofs])).cuda()
    res = {"workload": f"annulus r in [0.2, 0.5], {len(coords)} vertices, {len(elems)} triangles, "
                       "kappa=exp(N(0,0.5^2)), Dirichlet grids on the mesh domain",
           "unknowns": S.n, "setup_s": t_setup, "J": S.info()["J"]}
    for name, prec in (("fp64", A.PREC_FP64), ("mixed", A.PREC_MIXED)):
        S.set_precision(prec)
        u, it, tr = S.solve_device(f, 1e-8)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            u, it, tr = S.solve_device(f, 1e-8, out=u)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / steps
        res[name] = {"value": S.n / dt, "ms_per_step": dt * 1e3, "iterations": it, "true_rel_residual": tr}
        log(f"annulus {name}: {dt * 1e3:.2f} ms/solve, {it} iterations ({S.n / dt:.3e} DOF-solves/s)")
    del S
    # mixed problem on the same mesh: Dirichlet on the outer circle, Neumann on the hole; the
    # Dirichlet grids on the mesh domain against the mixed Dirichlet/Neumann grids (FP64)
    outer = dirichlet & (np.hypot(coords[:, 0] - 0.5, coords[:, 1] - 0.5) > 0.35)
    mres = {"problem": "Dirichlet on the outer circle, Neumann on the hole"}
    for key, dom in (("dirichlet_grids", 1), ("mixed_grids", 2)):
        t0 = time.perf_counter()
        S = A.Solver(coords, elems, kappa, outer, colouring=colouring, domain=dom)
        t_setup = time.perf_counter() - t0
        f = torch.from_numpy(np.ascontiguousarray(f_vertex[S.dof_vertex()])).cuda()
        u, it, tr = S.solve_device(f, 1e-8)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            u, it, tr = S.solve_device(f, 1e-8, out=u)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / steps
        mres[key] = {"value": S.n / dt, "ms_per_step": dt * 1e3, "iterations": it, "true_rel_residual": tr,
                     "unknowns": S.n, "setup_s": t_setup}
        log(f"annulus, Neumann hole, {key.replace('_', ' ')}: {dt * 1e3:.2f} ms/solve, {it} iterations")
        del S
    res["neumann_hole"] = mres
    # pure Neumann problem on the same mesh (no Dirichlet vertex: mixed grids with an empty
    # Dirichlet part, f projected onto the range of A, u mean-free), without and with the
    # near-boundary correction of Section 3.5 (j = 2 layers), FP64
    nres = {"problem": "pure Neumann (every vertex an unknown), mixed grids"}
    for key, nb in (("no_correction", 0), ("near_boundary_j2", 2)):
        t0 = time.perf_counter()
        S = A.Solver(coords, elems, kappa, np.zeros(len(coords), dtype=bool), colouring=colouring, domain=2,
                     nb_layers=nb)
        t_setup = time.perf_counter() - t0
        f = torch.from_numpy(np.ascontiguousarray(f_vertex[S.dof_vertex()])).cuda()
        u, it, tr = S.solve_device(f, 1e-8)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            u, it, tr = S.solve_device(f, 1e-8, out=u)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / steps
        nres[key] = {"value": S.n / dt, "ms_per_step": dt * 1e3, "iterations": it, "true_rel_residual": tr,
                     "unknowns": S.n, "setup_s": t_setup}
        log(f"annulus, pure Neumann, j = {nb}: {dt * 1e3:.2f} ms/solve, {it} iterations, setup {t_setup:.1f} s")
        del S
    res["pure_neumann"] = nres
    return res


def adjoint(steps: int, colouring: int = 2):
    """Adjoint gradient workload: 724^2 jittered square, m ~ N(0, 0.3^2) per element; one step is
    coefficient update + forward solve + adjoint solve + element gradient."""
    import torch

    import paper_1410_2153_amd as A
    import workloads as W
    c = W.make_config(4)
    S = A.Solver(c["coords"], c["elems"], np.exp(c["m"]), colouring=colouring)
    dofs = S.dof_vertex()
    f = torch.tensor(c["f_vertex"][dofs], device="cuda")
    S.update_coefficient(np.exp(c["m_obs"]))
    u_obs = S.solve_device(f, 1e-8)[0] + torch.tensor(c["noise_vertex"][dofs], device="cuda")
    Fn = A.LogCoefficientSolve.function()
    m = torch.tensor(c["m"], device="cuda", requires_grad=True)

    def step():
        m.grad = None
        u = Fn.apply(m, f, S, 1e-8)
        J = 0.5 * ((u - u_obs) ** 2).sum()
        J.backward()
        return J

    step()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / steps
    # the device part alone: two solves + element kernel
    u, _, _ = S.solve_device(f, 1e-8)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        u, _, _ = S.solve_device(f, 1e-8, out=u)
        lam, _, _ = S.solve_device((u - u_obs).contiguous(), 1e-8)
        g = S.element_gradient(u, lam)
    torch.cuda.synchronize()
    dt_dev = (time.perf_counter() - t) / steps
    log(f"adjoint: {dt * 1e3:.1f} ms per gradient incl. coefficient update, {dt_dev * 1e3:.2f} ms device part")
    return {"workload": c["name"], "unknowns": S.n, "elements": len(c["elems"]),
            "ms_per_gradient": dt * 1e3, "ms_per_gradient_device_part": dt_dev * 1e3,
            "note": "device refresh of A from kappa=exp(m) (auxiliary hierarchy kept) + forward PCG + adjoint PCG "
                    "+ element kernel, through the torch.autograd.Function"}


def graded(args):
    """The graded unstructured 2-D mesh (1.0 M unknowns): FP64 and mixed solves, B_co and kernel
    timings with its own roofline entry, local smoothing, the nested start and the device setup."""
    import torch

    import paper_1410_2153_amd as A
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    c = load_workload(args.scale)
    log(f"workload: {len(c['coords'])} vertices, {len(c['elems'])} triangles ({time.perf_counter() - t0:.1f} s)")
    t0 = time.perf_counter()
    S64 = A.Solver(c["coords"], c["elems"], c["kappa"], device=0, precision=A.PREC_FP64, colouring=args.colouring,
                   autotune=args.autotune)
    t_setup = time.perf_counter() - t0
    info = S64.info()
    setup_phases = S64.setup_seconds()
    host_tree = {(k, 0): S64.export(k) for k in ("keys", "refined", "leaves", "leaf_kappa", "A_col", "A_val",
                                                   "Pi_col", "Pi_val")}
    for lv in sorted({lv for lv in (info["J"], info["lc"] + 1) if info["lc"] < lv <= info["J"]}):  # smoothed levels
        host_tree.update({(k, lv): S64.export(k, lv) for k in ("Al_col", "Al_val", "P_col", "P_val")})
    log(f"setup {t_setup:.1f} s: {info}")
    dofs = S64.dof_vertex()
    f = torch.from_numpy(np.ascontiguousarray(c["f_vertex"][dofs])).to(dev)
    n = S64.n

    step_ms = {}

    def run(S, steps, warmup, key=None):
        u = torch.empty_like(f)
        for _ in range(warmup):
            S.solve_device(f, 1e-8, out=u)
        torch.cuda.synchronize()
        t = time.perf_counter()
        its, per = [], []
        for _ in range(steps):
            t1 = time.perf_counter()
            _, it, tr = S.solve_device(f, 1e-8, out=u)   # returns once u is in device memory
            per.append((time.perf_counter() - t1) * 1e3)
            its.append(it)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        if key:
            step_ms[key] = float(np.median(per))
        return dt, its, tr, u

    dt64, its64, tr64, u64 = run(S64, args.steps, args.warmup, "fp64")
    log(f"fp64: {dt64 / args.steps * 1e3:.2f} ms/solve, iters {its64}, true rel res {tr64:.2e}")
    S64.set_precision(A.PREC_MIXED)
    dt32, its32, tr32, u32 = run(S64, args.steps, args.warmup, "mixed")
    S64.set_precision(A.PREC_FP64)
    log(f"mixed: {dt32 / args.steps * 1e3:.2f} ms/solve, iters {its32}, true rel res {tr32:.2e}")
    diff = float(torch.linalg.norm(u32 - u64) / torch.linalg.norm(u64))

    # dominant kernel: the Gauss-Seidel colour pass (sliced ELL, FP64); every pass inside full B_co
    # applications is timed by HIP events stamped with that launch's start and end, on torch's stream
    if args.no_kernel_timing:
        ms_gs = by_gs = ms_spmv = by_spmv = ms_lds = by_lds = ms_mv = by_mv = ms_b64 = by_b64 = ms_b32 = by_b32 = float("nan")
    else:
        ms_gs, by_gs = S64.time_kernel(4, reps=10, precision=A.PREC_FP64)
        ms_spmv, by_spmv = S64.time_kernel(6, reps=50)
        ms_lds, by_lds = S64.time_kernel(7, reps=50)
        ms_mv, by_mv = S64.time_kernel(0, reps=50)
        ms_b64, by_b64 = S64.time_kernel(2, reps=20, precision=A.PREC_FP64)
        ms_b32, by_b32 = S64.time_kernel(2, reps=20, precision=A.PREC_MIXED)
    crec = counter_record("graded1M")
    roof = {"bound": "hbm", "kernel": "asmg::k_sell<0, double, VAR> (Gauss-Seidel colour pass, sliced ELL; VAR = the variant tuned per launch site; traffic from a run with the default, VAR 0)",
            "achieved": by_gs / ms_gs / 1e6, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": by_gs / ms_gs / 1e6 / HBM_PEAK_GBS, "traffic": crec.get("traffic_bytes_per_launch"),
            "bytes_per_launch": by_gs, "ms_per_launch": ms_gs}
    bco = crec.get("bco_per_application", {})
    vcyc = {"fp64": {"ms": ms_b64, "model_bytes": by_b64, "GBs": by_b64 / ms_b64 / 1e6,
                     "frac_of_peak": by_b64 / ms_b64 / 1e6 / HBM_PEAK_GBS,
                     "counted_hbm_bytes": bco.get("fp64", {}).get("traffic_bytes")},
            "fp32": {"ms": ms_b32, "model_bytes": by_b32, "GBs": by_b32 / ms_b32 / 1e6,
                     "frac_of_peak": by_b32 / ms_b32 / 1e6 / HBM_PEAK_GBS,
                     "counted_hbm_bytes": bco.get("fp32", {}).get("traffic_bytes")},
            "fine_spmv_fp64": {"kernel": "asmg::k_cg_spmv (PCG product q = A p with p.q partials, sliced ELL)",
                               "ms": ms_spmv, "model_bytes": by_spmv, "GBs": by_spmv / ms_spmv / 1e6},
            "fine_spmv_lds_staged_fp64": {"kernel": "asmg::k_cg_spmv_lds (same product, p gathers staged in LDS "
                                                    "per 4-slice tile; measured alternative, not used by the solve)",
                                          "ms": ms_lds, "model_bytes": by_lds, "GBs": by_lds / ms_lds / 1e6},
            "abi_matvec_csr_fp64": {"kernel": "asmg::k_matvec (CSR, asmg_matvec_device only)",
                                    "ms": ms_mv, "model_bytes": by_mv, "GBs": by_mv / ms_mv / 1e6}}
    out = {
        "workload": f"graded 2-D Delaunay mesh, {len(c['coords'])} vertices, {len(c['elems'])} "
                    f"triangles, kappa=exp(N(0,0.5^2)), f~U[-1,1], PCG to 1e-8 from u0=0",
        "unknowns": n, "setup_s": t_setup, "J": info["J"], "lc": info["lc"],
        "colouring": ["natural", "hash", "smallest-last"][args.colouring], "colours_fine": info["n_colours_fine"],
        "fp64": {"value": n * args.steps / dt64, "ms_per_step": dt64 / args.steps * 1e3,
                 "ms_per_step_median": step_ms["fp64"], "iterations": its64[-1], "true_rel_residual": tr64},
        "mixed": {"value": n * args.steps / dt32, "ms_per_step": dt32 / args.steps * 1e3,
                  "ms_per_step_median": step_ms["mixed"],
                  "iterations": its32[-1], "true_rel_residual": tr32, "rel_diff_vs_fp64": diff},
        "vcycle": vcyc,
        "roofline": roof,
    }
    del S64
    torch.cuda.synchronize()
    if not args.no_extra:
        # the same workload with local smoothing on N~_l (the decomposition of Section 4.3)
        t0 = time.perf_counter()
        SL = A.Solver(c["coords"], c["elems"], c["kappa"], device=0, precision=A.PREC_FP64,
                      colouring=args.colouring, smoothing=1, autotune=args.autotune)
        t_setup_l = time.perf_counter() - t0
        loc = {"setup_s": t_setup_l}
        for name, prec in (("fp64", A.PREC_FP64), ("mixed", A.PREC_MIXED)):
            SL.set_precision(prec)
            dtl, itl, trl, ul = run(SL, args.steps, args.warmup)
            loc[name] = {"value": n * args.steps / dtl, "ms_per_step": dtl / args.steps * 1e3, "iterations": itl[-1],
                         "true_rel_residual": trl}
            log(f"local smoothing {name}: {dtl / args.steps * 1e3:.2f} ms/solve, iters {itl}, true rel res {trl:.2e}")
        loc["rel_diff_vs_full_fp64"] = float(torch.linalg.norm(ul - u64) / torch.linalg.norm(u64))
        SL.set_precision(A.PREC_FP64)
        ms_bl, by_bl = SL.time_kernel(2, reps=20, precision=A.PREC_FP64)
        loc["vcycle_fp64"] = {"ms": ms_bl, "model_bytes": by_bl, "GBs": by_bl / ms_bl / 1e6}
        out["local_smoothing"] = loc
        del SL
        torch.cuda.synchronize()
        # the same workload started from the nested iteration's guess (one V-cycle per level)
        SN = A.Solver(c["coords"], c["elems"], c["kappa"], device=0, precision=A.PREC_FP64,
                      colouring=args.colouring, nested=1, autotune=args.autotune)
        nst = {}
        for name, prec in (("fp64", A.PREC_FP64), ("mixed", A.PREC_MIXED)):
            SN.set_precision(prec)
            dtn, itn, trn, un = run(SN, args.steps, args.warmup)
            nst[name] = {"value": n * args.steps / dtn, "ms_per_step": dtn / args.steps * 1e3, "iterations": itn[-1],
                         "true_rel_residual": trn}
            log(f"nested start {name}: {dtn / args.steps * 1e3:.2f} ms/solve, iters {itn}, true rel res {trn:.2e}")
        nst["rel_diff_vs_fp64"] = float(torch.linalg.norm(un - u64) / torch.linalg.norm(u64))
        out["nested_start"] = nst
        del SN
        torch.cuda.synchronize()
        # the same setup with the fine matrix and the cluster tree built on the device
        t0 = time.perf_counter()
        SD = A.Solver(c["coords"], c["elems"], c["kappa"], device=0, precision=A.PREC_FP64,
                      colouring=args.colouring, setup_device=1, autotune=args.autotune)
        t_setup_d = time.perf_counter() - t0
        same = SD.info() == info and all(np.array_equal(SD.export(k, lv), host_tree[(k, lv)]) for k, lv in host_tree)
        dph = SD.setup_seconds()
        out["setup"] = {"host_phases_s": setup_phases, "device_setup_phases_s": dph,
                        "total_s_host": t_setup, "total_s_device_setup": t_setup_d,
                        "device_setup_identical": bool(same)}
        log(f"setup: fine matrix + tree on the host {setup_phases['fine'] + setup_phases['tree']:.3f} s, on the "
            f"device {dph['fine'] + dph['tree']:.3f} s (identical: {same}); levels (meshes, A_l, P_l on the "
            f"device) {setup_phases['levels']:.3f} -> {dph['levels']:.3f} s; Pi {setup_phases['transfer']:.3f} -> "
            f"{dph['transfer']:.3f} s; total {t_setup:.1f} -> "
            f"{t_setup_d:.1f} s")
        del SD
        # colourings in the hash order (Jones-Plassmann rounds on the device with setup_device = 1)
        hc = {}
        for key, sd in (("host", 0), ("device", 1)):
            t0 = time.perf_counter()
            SC = A.Solver(c["coords"], c["elems"], c["kappa"], device=0, precision=A.PREC_FP64, colouring=1,
                          setup_device=sd, autotune=args.autotune)
            hc[key] = {"total_s": time.perf_counter() - t0, "phases_s": SC.setup_seconds(),
                       "colours": SC.export("colour_fine")}
            del SC
        col_same = bool(np.array_equal(hc["host"].pop("colours"), hc["device"].pop("colours")))
        out["setup"]["hash_colouring"] = {**hc, "identical_fine_colouring": col_same}
        log(f"setup, hash colouring: colourings on the host {hc['host']['phases_s']['colourings']:.3f} s, on the "
            f"device {hc['device']['phases_s']['colourings']:.3f} s (identical: {col_same}); total "
            f"{hc['host']['total_s']:.1f} -> {hc['device']['total_s']:.1f} s")
        torch.cuda.synchronize()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=float, default=1.0, help="size of the graded mesh (1.0 = 1.0 M vertices)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--batch-meshes", type=int, default=256, help="meshes of the headline batched workload")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the headline: skip the graded, 3-D, adjoint and annulus workloads")
    ap.add_argument("--only", choices=["batched", "graded", "cube3d", "adjoint", "annulus"], default=None,
                    help="run only this workload and print its record (for profiling it alone)")
    ap.add_argument("--no-kernel-timing", action="store_true",
                    help="skip the per-kernel HIP-event measurements (for hardware-counter runs)")
    ap.add_argument("--autotune", type=int, default=1, choices=[0, 1],
                    help="0: fixed default launch shapes (hardware-counter runs, which would otherwise "
                         "also count the autotuner's trial launches)")
    ap.add_argument("--colouring", type=int, default=2,
                    help="Gauss-Seidel colour order of the single-mesh solves: 0 natural, 1 hash, 2 smallest-last")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 512 MiB device copy (reference dispatch for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch

    import paper_1410_2153_amd as A  # noqa: F401  (fails loudly if the library is not built)
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        x = torch.empty(64 * 2 ** 20, dtype=torch.float64, device=dev).fill_(1.0)
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    kt = not args.no_kernel_timing
    if args.only == "batched":
        print(json.dumps({"batched": batched(args.batch_meshes, args.steps, args.warmup, kt, args.autotune)}))
        return
    if args.only == "graded":
        print(json.dumps({"graded": graded(args)}))
        return
    if args.only == "cube3d":
        print(json.dumps({"cube3d": cube3d(args.steps, args.colouring, kt, args.autotune)}))
        return
    if args.only == "adjoint":
        print(json.dumps({"adjoint": adjoint(args.steps, args.colouring)}))
        return
    if args.only == "annulus":
        print(json.dumps({"annulus": annulus(args.steps, args.colouring)}))
        return

    # headline: the batched workload, all 256 x 4 systems per step
    b = batched(args.batch_meshes, args.steps, args.warmup, kt, args.autotune)
    crec = counter_record("batched256x4")
    bco = crec.get("bco_per_application", {})
    gs = b.get("gs_pass", {"ms_per_launch": float("nan"), "bytes_per_launch": float("nan")})
    vc = b.get("vcycle_4rhs", {})
    for key in ("fp64", "fp32"):
        if key in vc:
            vc[key]["counted_hbm_bytes"] = bco.get(key, {}).get("traffic_bytes")
    ach = gs["bytes_per_launch"] / gs["ms_per_launch"] / 1e6
    out = {
        "metric": "DOF-solves/sec to 1e-8 rel. residual + V-cycle HBM GB/s, FP64 vs mixed",
        "value": b["fp64"]["value"], "unit": "DOF-solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": b["fp64"]["ms_per_step"],
        "ms_per_step_median": b["fp64"]["ms_per_step_median"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": b["workload"], "meshes": b["meshes"], "rhs": b["rhs"], "unknowns": b["unknowns"],
                   "sides_min_max": b["sides_min_max"], "max_iterations_fp64": b["fp64"]["max_iterations"],
                   "max_true_rel_residual_fp64": b["fp64"]["max_true_rel_residual"], "setup_s": b["setup_s"]},
        "mixed": b["mixed"],
        "vcycle": vc,
        "roofline": {"bound": "hbm", "kernel": "asmg::kb_sell<MODE, 4, double, VAR> (batched Gauss-Seidel colour "
                                               "pass, sliced ELL, 4 interleaved right-hand sides; MODE 3 in sweeps "
                                               "from zero, 0 otherwise; VAR = the variant tuned per launch site; "
                                               "traffic from a run with the default, VAR 0)",
                     "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                     "traffic": crec.get("traffic_bytes_per_launch"), "bytes_per_launch": gs["bytes_per_launch"],
                     "ms_per_launch": gs["ms_per_launch"]},
        "single_solves_fp64_sample": b["single_solves_fp64_sample"],
        "tuned_launch_shapes_fp64_4rhs": b["tuned_launch_shapes_fp64_4rhs"],
    }
    torch.cuda.synchronize()
    if not args.no_extra:
        out["graded"] = graded(args)
        out["cube3d"] = cube3d(args.steps, args.colouring, kt, args.autotune)
        out["adjoint"] = adjoint(args.steps, args.colouring)
        out["annulus"] = annulus(args.steps, args.colouring)
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(n_meshes=args.batch_meshes)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
