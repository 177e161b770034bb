"""Write the stored expected values of the full-size graded-mesh parity test.

Calls only the oracle (``oracle/``) and the seeded input generators (``workloads/``):
no value here comes from the HIP path. Run from the repository root:

    python tests/golden/make_graded1m.py [scale]

Workload: the graded 2-D Delaunay mesh of the unit square (density 1/(r + 0.01) + 1
towards (0, 0), about 1.0 M vertices and 2.0 M triangles at scale 1), kappa = exp(N(0,
0.5^2)) per element, f ~ U[-1, 1] per unknown, homogeneous Dirichlet data.

Stored (``graded1m.npz``, or ``graded<scale>.npz`` for another scale):
  * SHA-256 digests of every index map of the hierarchy in a canonical int64 form
    (``hierarchy_digests``): box keys, refined set, leaves, level sizes, level vertices,
    simplices and unknowns, the patterns of A, A_l, P_l and Pi, the colourings;
  * one FP64 application z = B_co f (Algorithm 1) at 4096 seeded unknowns, with |z|_inf;
  * the FP64 PCG solve of Section 5.2 to ||r|| <= 1e-8 ||f|| from u_0 = 0: the iteration
    count, u at the same unknowns and |u|_inf;
  * the FP64 solve to 1e-12 (the reference of the mixed-precision bar), at the same unknowns.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

N_SAMPLES = 4096


def digest(a) -> str:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int64))
    return hashlib.sha256(a.tobytes()).hexdigest()


def boxes(tuples, d):
    """A set or list of (level, i_0, .., i_{d-1}) boxes as a sorted (k, d + 1) int64 array."""
    arr = np.array(sorted(tuples), dtype=np.int64).reshape(-1, d + 1)
    return arr


def hierarchy_digests(H) -> dict:
    """Canonical digests of the oracle hierarchy's index maps (see module docstring)."""
    d = H.d
    out = {"keys": digest(H.tree.keys), "refined": digest(boxes(H.tree.R, d)),
           "leaves": digest(boxes(H.tree.leaves, d)),
           "level_n": digest([H.meshes.level(l).n for l in range(1, H.tree.J + 1)]),
           "A_pattern": digest(np.concatenate([H.A.indptr, H.A.indices])),
           "Pi_pattern": digest(np.concatenate([H.Pi.tocsr().indptr, H.Pi.tocsr().indices])),
           "colour_fine": digest(H.colour_fine)}
    for l in range(H.aux.lc, H.tree.J + 1):
        lm = H.meshes.level(l)
        out[f"level_verts_{l}"] = digest(lm.verts)
        out[f"level_simp_{l}"] = digest(lm.simp)
        out[f"level_dofs_{l}"] = digest(lm.dof_vert)
        Al = H.aux.A[l].tocsr()
        out[f"Al_pattern_{l}"] = digest(np.concatenate([Al.indptr, Al.indices]))
    for l in range(H.aux.lc + 1, H.tree.J + 1):
        P = H.aux.P[l].tocsr()
        out[f"P_pattern_{l}"] = digest(np.concatenate([P.indptr, P.indices]))
        out[f"colour_aux_{l}"] = digest(H.colour_aux[l])
    return out


def sample_indices(n: int) -> np.ndarray:
    return np.sort(np.random.default_rng([1, 99, 0]).choice(n, size=min(N_SAMPLES, n), replace=False))


def main(scale: float = 1.0):
    import workloads as W
    from oracle.hierarchy import Hierarchy

    t0 = time.perf_counter()
    c = W.make_config(1, scale=scale)
    print(f"mesh: {len(c['coords'])} vertices, {len(c['elems'])} triangles ({time.perf_counter() - t0:.0f} s)",
          flush=True)
    t0 = time.perf_counter()
    H = Hierarchy(c["coords"], c["elems"], c["kappa"])
    print(f"oracle hierarchy: {H.n} unknowns, J = {H.tree.J}, l_c = {H.aux.lc} ({time.perf_counter() - t0:.0f} s)",
          flush=True)
    f = c["f_vertex"][H.dofs]
    idx = sample_indices(H.n)
    t0 = time.perf_counter()
    z = H.preconditioner()(f)
    print(f"B_co f ({time.perf_counter() - t0:.0f} s)", flush=True)
    t0 = time.perf_counter()
    u, it, info = H.solve(f, 1e-8)
    print(f"solve 1e-8: {it} iterations, true residual {info['true_rel_residual']:.3e} "
          f"({time.perf_counter() - t0:.0f} s)", flush=True)
    t0 = time.perf_counter()
    u12, it12, info12 = H.solve(f, 1e-12)
    print(f"solve 1e-12: {it12} iterations ({time.perf_counter() - t0:.0f} s)", flush=True)
    dig = hierarchy_digests(H)
    name = "graded1m" if scale == 1.0 else f"graded{scale:g}"
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}.npz")
    np.savez_compressed(
        path, scale=np.float64(scale), n=np.int64(H.n), J=np.int64(H.tree.J), lc=np.int64(H.aux.lc),
        idx=idx.astype(np.int64), z=z[idx], z_inf=np.float64(np.abs(z).max()), z_norm=np.float64(np.linalg.norm(z)),
        iters=np.int64(it), u=u[idx], u_inf=np.float64(np.abs(u).max()),
        true_rel_residual=np.float64(info["true_rel_residual"]),
        iters12=np.int64(it12), u12=u12[idx], u12_inf=np.float64(np.abs(u12).max()),
        hierarchy_digests=np.array(json.dumps(dig, sort_keys=True)))
    print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    main(float(sys.argv[1]) if len(sys.argv) > 1 else 1.0)
