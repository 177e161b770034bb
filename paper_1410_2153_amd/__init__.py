"""Python binding of libasmg (include/asmg.h): argument marshalling only.

Every step of the setup and the solve runs in the C++/HIP library. PyTorch is
used for device memory and streams: device entry points take CUDA/HIP tensors
and run on torch's current stream. The library must have been built
(``python -m paper_1410_2153_amd.build`` or ``__graft_entry__.build()``); if it
is missing, importing this module raises, so a missing extension cannot fall
back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

# torch first: its bundled HIP runtime then provides the `libamdhip64.so.7` this library
# needs, so the process holds one HIP runtime (loading the library first would bring in a
# second runtime from /opt/rocm, and torch would then see no device)
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libasmg.so")

OK, EINVAL, ENOCONV, ENOTSPD, ENAN, EDEVICE, ENOMEM = 0, -1, -2, -3, -4, -5, -6
PREC_FP64, PREC_MIXED = 0, 1
# candidate launch shapes of the autotuner: (threads per block, XCD order, kernel variant)
SHAPES = [(256, 1, 0), (128, 1, 0), (512, 1, 0), (256, 0, 0), (128, 0, 0), (512, 0, 0),
          (256, 1, 1), (512, 1, 1), (256, 0, 1), (512, 0, 1)]
N_SHAPES = len(SHAPES)

EXPORTED = [
    "asmg_default_options", "asmg_setup", "asmg_update_coefficient", "asmg_set_precision",
    "asmg_set_coefficient_device", "asmg_num_dofs", "asmg_dof_vertex",
    "asmg_solve", "asmg_solve_device", "asmg_apply_preconditioner_device", "asmg_matvec_device",
    "asmg_element_gradient_device", "asmg_time_kernel", "asmg_export", "asmg_destroy", "asmg_last_error",
    "asmg_setup_batch", "asmg_solve_batch_device", "asmg_time_batch",
    "asmg_set_log_coefficient_device", "asmg_adjoint_gradient_device", "asmg_solve_device_noalloc",
    "asmg_time_batch_kernel",
]


class AsmgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"asmg error {code}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("n_min", ctypes.c_int), ("nu_aux", ctypes.c_int), ("nu_fine", ctypes.c_int),
                ("coarse_max_dofs", ctypes.c_int), ("max_iter", ctypes.c_int), ("precision", ctypes.c_int),
                ("colour_seed", ctypes.c_uint32), ("device", ctypes.c_int), ("check_every", ctypes.c_int),
                ("colouring", ctypes.c_int), ("smoothing", ctypes.c_int), ("domain", ctypes.c_int),
                ("autotune", ctypes.c_int), ("nested", ctypes.c_int),
                ("setup_device", ctypes.c_int), ("red_blocks", ctypes.c_int), ("nb_layers", ctypes.c_int)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libasmg.so not built ({LIB_PATH}); run paper_1410_2153_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    lib.asmg_last_error.restype = ctypes.c_char_p
    lib.asmg_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.asmg_setup.argtypes = [ctypes.c_int, I64, P, I64, P, P, P, ctypes.POINTER(Options), ctypes.POINTER(P)]
    lib.asmg_update_coefficient.argtypes = [P, P]
    lib.asmg_set_precision.argtypes = [P, ctypes.c_int]
    lib.asmg_set_coefficient_device.argtypes = [P, P, P]
    lib.asmg_set_log_coefficient_device.argtypes = [P, P, P]
    lib.asmg_adjoint_gradient_device.argtypes = [P, P, P, P, P]
    lib.asmg_num_dofs.argtypes = [P, ctypes.POINTER(I64)]
    lib.asmg_dof_vertex.argtypes = [P, P]
    lib.asmg_solve.argtypes = [P, P, ctypes.c_double, P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]
    lib.asmg_solve_device.argtypes = [P, P, ctypes.c_double, P, ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(ctypes.c_double), P]
    lib.asmg_solve_device_noalloc.argtypes = [P, P, ctypes.c_double, P, ctypes.POINTER(ctypes.c_int),
                                              ctypes.POINTER(ctypes.c_double), P]
    lib.asmg_apply_preconditioner_device.argtypes = [P, P, P, ctypes.c_int, P]
    lib.asmg_matvec_device.argtypes = [P, P, P, P]
    lib.asmg_element_gradient_device.argtypes = [P, P, P, P, P]
    lib.asmg_time_kernel.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]
    lib.asmg_export.argtypes = [P, ctypes.c_char_p, ctypes.c_int, P, ctypes.POINTER(I64)]
    lib.asmg_setup_batch.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, P, ctypes.POINTER(Options),
                                     ctypes.POINTER(P)]
    lib.asmg_solve_batch_device.argtypes = [P, ctypes.c_int, P, ctypes.c_double, P, P, P, P]
    lib.asmg_time_batch.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]
    lib.asmg_time_batch_kernel.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, P,
                                           ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    lib.asmg_destroy.argtypes = [P]
    lib.asmg_destroy.restype = None
    return lib


lib = _load()


def _check(rc, allow=()):
    if rc != OK and rc not in allow:
        raise AsmgError(rc, lib.asmg_last_error().decode())
    return rc


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _tptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _need_host(a, n, what):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim != 1 or a.shape[0] != n:
        raise ValueError(f"{what} must be a 1-D array of {n} values, got shape {a.shape}")
    return a


def _need_device(t, n, what):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
            and t.numel() == n):
        raise ValueError(f"{what} must be a contiguous float64 device tensor of {n} values")
    return t


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Solver:
    """One mesh: ``asmg_setup`` on construction, ``asmg_destroy`` on close/garbage collection."""

    def __init__(self, coords, elems, kappa, dirichlet=None, *, device=0, precision=PREC_FP64, n_min=0,
                 nu_aux=2, nu_fine=1, coarse_max_dofs=1024, max_iter=1000, colour_seed=0, check_every=0,
                 colouring=2, smoothing=0, domain=0, autotune=1, nested=0, setup_device=0, red_blocks=0,
                 nb_layers=0):
        coords = np.ascontiguousarray(coords, dtype=np.float64)
        elems = np.ascontiguousarray(elems, dtype=np.int32)
        if coords.ndim != 2 or elems.ndim != 2 or elems.shape[1] != coords.shape[1] + 1:
            raise ValueError("coords must be (n_vertices, d) and elems (n_elements, d + 1)")
        kappa = _need_host(kappa, elems.shape[0], "kappa")
        self.dim = coords.shape[1]
        self.n_vertices = coords.shape[0]
        self.n_elements = elems.shape[0]
        opt = Options()
        lib.asmg_default_options(ctypes.byref(opt))
        opt.n_min, opt.nu_aux, opt.nu_fine = n_min, nu_aux, nu_fine
        opt.coarse_max_dofs, opt.max_iter, opt.precision = coarse_max_dofs, max_iter, precision
        opt.colour_seed, opt.device, opt.check_every = colour_seed, device, check_every
        opt.colouring = colouring
        opt.smoothing = smoothing
        opt.domain = domain
        opt.autotune = autotune
        opt.nested = nested
        opt.setup_device = setup_device
        opt.red_blocks = red_blocks
        opt.nb_layers = nb_layers
        self.precision = precision
        self.coef_version = 0   # bumped by every coefficient change (host or device)
        self.device = device
        dptr = None
        if dirichlet is not None:
            self._dir = np.ascontiguousarray(dirichlet, dtype=np.uint8)
            if self._dir.shape != (coords.shape[0],):
                raise ValueError("dirichlet must hold one flag per vertex")
            dptr = _ptr(self._dir)
        h = ctypes.c_void_p()
        _check(lib.asmg_setup(self.dim, self.n_vertices, _ptr(coords), self.n_elements, _ptr(elems), _ptr(kappa),
                              dptr, ctypes.byref(opt), ctypes.byref(h)))
        self.h = h
        n = ctypes.c_int64()
        _check(lib.asmg_num_dofs(self.h, ctypes.byref(n)))
        self.n = n.value

    def close(self):
        if getattr(self, "h", None) and lib is not None:
            lib.asmg_destroy(self.h)
            self.h = None

    __del__ = close

    # -- host vectors -------------------------------------------------------
    def dof_vertex(self) -> np.ndarray:
        out = np.empty(self.n, dtype=np.int32)
        _check(lib.asmg_dof_vertex(self.h, _ptr(out)))
        return out

    def solve(self, f, tol=1e-8, allow_noconv=False):
        """Host arrays: returns (u, iterations, true relative residual)."""
        f = _need_host(f, self.n, "f")
        u = np.empty(self.n)
        it = ctypes.c_int()
        tr = ctypes.c_double()
        _check(lib.asmg_solve(self.h, _ptr(f), tol, _ptr(u), ctypes.byref(it), ctypes.byref(tr)),
               (ENOCONV,) if allow_noconv else ())
        return u, it.value, tr.value

    def set_precision(self, precision):
        _check(lib.asmg_set_precision(self.h, precision))
        self.precision = precision

    def set_coefficient_device(self, kappa):
        """Operator A from a device coefficient tensor; the auxiliary hierarchy is kept."""
        _need_device(kappa, self.n_elements, "kappa")
        _check(lib.asmg_set_coefficient_device(self.h, _tptr(kappa), _stream()))
        self.coef_version += 1

    def set_log_coefficient_device(self, m):
        """Operator A from per-element log-coefficients (kappa = exp(m) computed in the library)."""
        _need_device(m, self.n_elements, "m")
        _check(lib.asmg_set_log_coefficient_device(self.h, _tptr(m), _stream()))
        self.coef_version += 1

    def update_coefficient(self, kappa):
        kappa = _need_host(kappa, self.n_elements, "kappa")
        _check(lib.asmg_update_coefficient(self.h, _ptr(kappa)))
        self.coef_version += 1

    # -- device tensors (torch) ---------------------------------------------
    def solve_device(self, f, tol=1e-8, out=None, allow_noconv=False):
        import torch
        _need_device(f, self.n, "f")
        u = torch.empty_like(f) if out is None else _need_device(out, self.n, "out")
        it = ctypes.c_int()
        tr = ctypes.c_double()
        _check(lib.asmg_solve_device(self.h, _tptr(f), tol, _tptr(u), ctypes.byref(it), ctypes.byref(tr), _stream()),
               (ENOCONV,) if allow_noconv else ())
        return u, it.value, tr.value

    def solve_device_noalloc(self, f, out, tol=1e-8, allow_noconv=False):
        """asmg_solve_device_noalloc: as solve_device into the caller's `out`; the library
        allocates nothing (control block and partials in its static per-GPU scratch)."""
        _need_device(f, self.n, "f")
        _need_device(out, self.n, "out")
        it = ctypes.c_int()
        tr = ctypes.c_double()
        _check(lib.asmg_solve_device_noalloc(self.h, _tptr(f), tol, _tptr(out), ctypes.byref(it), ctypes.byref(tr),
                                             _stream()), (ENOCONV,) if allow_noconv else ())
        return out, it.value, tr.value

    def apply_preconditioner(self, r, precision=None):
        import torch
        _need_device(r, self.n, "r")
        z = torch.empty_like(r)
        prec = self.precision if precision is None else precision
        _check(lib.asmg_apply_preconditioner_device(self.h, _tptr(r), _tptr(z), prec, _stream()))
        return z

    def matvec(self, x):
        import torch
        _need_device(x, self.n, "x")
        y = torch.empty_like(x)
        _check(lib.asmg_matvec_device(self.h, _tptr(x), _tptr(y), _stream()))
        return y

    def element_gradient(self, u, lam):
        import torch
        _need_device(u, self.n, "u")
        _need_device(lam, self.n, "lam")
        g = torch.empty(self.n_elements, dtype=torch.float64, device=u.device)
        _check(lib.asmg_element_gradient_device(self.h, _tptr(u), _tptr(lam), _tptr(g), _stream()))
        return g

    def adjoint_gradient(self, u, lam):
        """dJ/dm per element (kappa = exp(m)) from u and the adjoint state lam of A lam = dJ/du."""
        import torch
        _need_device(u, self.n, "u")
        _need_device(lam, self.n, "lam")
        g = torch.empty(self.n_elements, dtype=torch.float64, device=u.device)
        _check(lib.asmg_adjoint_gradient_device(self.h, _tptr(u), _tptr(lam), _tptr(g), _stream()))
        return g

    def solve_stats(self):
        """(iterations, restarts from the true residual) of the last solve."""
        it, rs = self.export("solve_stats").tolist()
        return it, rs

    def time_kernel(self, which, reps=20, precision=None):
        ms = ctypes.c_double()
        by = ctypes.c_double()
        prec = self.precision if precision is None else precision
        _check(lib.asmg_time_kernel(self.h, which, reps, prec, _stream(), ctypes.byref(ms), ctypes.byref(by)))
        return ms.value, by.value

    # -- exports --------------------------------------------------------------
    def export(self, name, level=0, dtype=None):
        cnt = ctypes.c_int64()
        _check(lib.asmg_export(self.h, name.encode(), level, None, ctypes.byref(cnt)))
        if dtype is None:
            dtype = (np.float64 if name.endswith("_val") or name in ("setup_seconds", "leaf_kappa", "coarse_inv",
                                                                       "tune_times") else np.int64)
        buf = np.empty(cnt.value, dtype=dtype)
        if cnt.value:
            _check(lib.asmg_export(self.h, name.encode(), level, _ptr(buf), ctypes.byref(cnt)))
        return buf

    def tuned_shapes(self, precision=PREC_FP64):
        """(threads per block, XCD order, kernel variant) picked by the autotuner per slice-kernel
        launch site."""
        return self.export("tuned_shapes", precision).reshape(-1, 3)

    def tune_times(self, precision=PREC_FP64):
        """The autotuner's best ms per (launch site, candidate shape); -1 = not timed."""
        t = self.export("tune_times", precision, dtype=np.float64)
        return t.reshape(-1, N_SHAPES) if len(t) else t

    def setup_seconds(self):
        """Wall time of the setup phases (s): fine, tree, levels, transfer, colourings, coarse, upload."""
        keys = ["fine", "tree", "levels", "transfer", "colourings", "coarse", "upload"]
        return dict(zip(keys, self.export("setup_seconds").tolist()))

    def info(self):
        v = self.export("info")
        keys = ["dim", "n", "J", "lc", "n_levels", "nnz_A", "nnz_Pi", "n_refined", "n_leaves", "n_colours_fine",
                "n_elements", "n_vertices"]
        return {k: int(x) for k, x in zip(keys, v)}

    def export_csr(self, mat, level=0, shape=None):
        import scipy.sparse as sp
        rp = self.export(f"{mat}_rowptr", level)
        ci = self.export(f"{mat}_col", level)
        v = self.export(f"{mat}_val", level)
        n = len(rp) - 1
        if shape is None:
            shape = (n, int(ci.max()) + 1 if len(ci) else 0)
        return sp.csr_matrix((v, ci, rp), shape=shape)


class BatchSolver:
    """Many meshes, solved together (asmg_setup_batch / asmg_solve_batch_device).

    ``meshes`` is a list of (coords, elems, kappa). Right-hand sides and solutions
    are device tensors laid out [mesh][rhs][unknown] (see ``offsets``).
    """

    def __init__(self, meshes, *, device=0, precision=PREC_FP64, n_min=0, nu_aux=2, nu_fine=1,
                 coarse_max_dofs=1024, max_iter=1000, smoothing=0, autotune=1, nested=0):
        dim = np.asarray(meshes[0][0]).shape[1]
        coords = np.ascontiguousarray(np.concatenate([np.asarray(m[0], dtype=np.float64) for m in meshes]))
        elems = np.ascontiguousarray(np.concatenate([np.asarray(m[1], dtype=np.int32) for m in meshes]))
        kappa = np.ascontiguousarray(np.concatenate([np.asarray(m[2], dtype=np.float64) for m in meshes]))
        vo = np.zeros(len(meshes) + 1, dtype=np.int64)
        eo = np.zeros(len(meshes) + 1, dtype=np.int64)
        vo[1:] = np.cumsum([len(m[0]) for m in meshes])
        eo[1:] = np.cumsum([len(m[1]) for m in meshes])
        opt = Options()
        lib.asmg_default_options(ctypes.byref(opt))
        opt.n_min, opt.nu_aux, opt.nu_fine = n_min, nu_aux, nu_fine
        opt.coarse_max_dofs, opt.max_iter, opt.precision, opt.device = coarse_max_dofs, max_iter, precision, device
        opt.smoothing = smoothing
        opt.autotune = autotune
        opt.nested = nested
        h = ctypes.c_void_p()
        _check(lib.asmg_setup_batch(len(meshes), dim, _ptr(vo), _ptr(coords), _ptr(eo), _ptr(elems), _ptr(kappa),
                                    ctypes.byref(opt), ctypes.byref(h)))
        self.h = h
        self.n_meshes = len(meshes)
        cnt = ctypes.c_int64(self.n_meshes)
        self.n_per_mesh = np.empty(self.n_meshes, dtype=np.int64)
        _check(lib.asmg_export(self.h, b"batch_n", 0, _ptr(self.n_per_mesh), ctypes.byref(cnt)))
        self.n_total = int(self.n_per_mesh.sum())
        self.precision = precision

    def close(self):
        if getattr(self, "h", None) and lib is not None:
            lib.asmg_destroy(self.h)
            self.h = None

    __del__ = close

    def _export(self, name, level, dtype):
        cnt = ctypes.c_int64()
        _check(lib.asmg_export(self.h, name, level, None, ctypes.byref(cnt)))
        buf = np.empty(cnt.value, dtype=dtype)
        if cnt.value:
            _check(lib.asmg_export(self.h, name, level, _ptr(buf), ctypes.byref(cnt)))
        return buf

    def tuned_shapes(self, n_rhs, precision=PREC_FP64):
        """(threads per block, XCD order, kernel variant) picked by the autotuner per slice-kernel
        launch site."""
        return self._export(b"batch_shapes", n_rhs + 8 * precision, np.int64).reshape(-1, 3)

    def tune_times(self, n_rhs, precision=PREC_FP64):
        """The autotuner's best ms per (launch site, candidate shape); -1 = not timed."""
        t = self._export(b"batch_tune_times", n_rhs + 8 * precision, np.float64)
        return t.reshape(-1, N_SHAPES) if len(t) else t

    def offsets(self, n_rhs):
        o = np.zeros(self.n_meshes + 1, dtype=np.int64)
        o[1:] = np.cumsum(self.n_per_mesh * n_rhs)
        return o

    def set_precision(self, precision):
        _check(lib.asmg_set_precision(self.h, precision))
        self.precision = precision

    def solve(self, F, n_rhs, tol=1e-8, out=None):
        import torch
        if n_rhs not in (1, 2, 4):
            raise ValueError("n_rhs must be 1, 2 or 4")
        _need_device(F, self.n_total * n_rhs, "F")
        U = torch.empty_like(F) if out is None else _need_device(out, self.n_total * n_rhs, "out")
        it = np.zeros(self.n_meshes * n_rhs, dtype=np.int32)
        tr = np.zeros(self.n_meshes * n_rhs)
        _check(lib.asmg_solve_batch_device(self.h, n_rhs, _tptr(F), tol, _tptr(U), _ptr(it), _ptr(tr), _stream()))
        return U, it.reshape(self.n_meshes, n_rhs), tr.reshape(self.n_meshes, n_rhs)

    def time_kernel(self, which, n_rhs, reps=10, precision=None):
        """asmg_time_batch_kernel: 0 = B_co as graph replays (median ms, bytes per application),
        1 = Gauss-Seidel colour passes timed per launch (mean ms and bytes per launch)."""
        ms = ctypes.c_double()
        by = ctypes.c_double()
        prec = self.precision if precision is None else precision
        _check(lib.asmg_time_batch_kernel(self.h, which, n_rhs, reps, prec, _stream(), ctypes.byref(ms),
                                          ctypes.byref(by)))
        return ms.value, by.value

    def time_preconditioner(self, n_rhs, reps=10, precision=None):
        ms = ctypes.c_double()
        by = ctypes.c_double()
        prec = self.precision if precision is None else precision
        _check(lib.asmg_time_batch(self.h, n_rhs, reps, prec, _stream(), ctypes.byref(ms), ctypes.byref(by)))
        return ms.value, by.value


class LogCoefficientSolve:
    """u(m) = A(exp(m))^{-1} f as a torch.autograd.Function over per-element log-coefficients m.

    Forward: the library refreshes A from kappa = exp(m) on the device (the auxiliary
    hierarchy of the last setup is kept as the preconditioner), then the PCG solve.
    Backward: one more PCG solve with the same symmetric matrix, A lam = dJ/du, then the
    library's adjoint element kernel dJ/dm_e = -kappa_e lam_e^T K1_e u_e. If the solver's
    coefficient changed after this forward (another forward on the same solver), backward
    first restores A(exp(m)) from the saved m.
    """

    @staticmethod
    def function():
        import torch

        class _Fn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, m, f, solver, tol):
                md = m.detach().contiguous()
                solver.set_log_coefficient_device(md)
                u, _, _ = solver.solve_device(f.contiguous(), tol)
                ctx.solver = solver
                ctx.tol = tol
                ctx.version = solver.coef_version
                ctx.save_for_backward(u, md)
                return u

            @staticmethod
            def backward(ctx, gu):
                u, md = ctx.saved_tensors
                S = ctx.solver
                if S.coef_version != ctx.version:
                    S.set_log_coefficient_device(md)
                    ctx.version = S.coef_version
                lam, _, _ = S.solve_device(gu.contiguous(), ctx.tol)
                return S.adjoint_gradient(u, lam), None, None, None

        return _Fn
