"""Seeded synthetic inputs for the ASMG-PCG solve (meshes, coefficients, right-hand sides).

This module only builds inputs: meshes, per-element coefficients, per-vertex
right-hand-side draws. It contains none of the solver's arithmetic, and both the
oracle and the HIP path take their inputs from here.

Every random draw comes from ``numpy.random.default_rng([cfg, stream, item])``
and is made in a fixed order, so a (config, item) pair always yields the same
arrays.

Workload families (shapes follow the paper's experiments, Section 5: a 2-D
Poisson problem on the unit square with homogeneous Dirichlet data, on
shape-regular unstructured meshes with local refinement):

* ``square_mesh``  -- an n x n grid of the unit square, each cell split by a
  diagonal picked by a seeded coin, interior nodes jittered by U(-j h, j h).
  This is the jittered structured mesh family (64^2 small case, 724^2 adjoint
  case, 32..512 sides in the batched case).
* ``graded_mesh``  -- a Delaunay mesh of the unit square whose point density is
  proportional to 1/(r + 0.01) + 1, with r the distance to the corner (0, 0).
  The points are the jittered centres of a balanced quadtree refined until each
  leaf is no larger than the local target spacing, plus the leaf corners on the
  boundary. This stands in for the paper's locally refined Baltic Sea mesh,
  which is not available.
* ``kuhn_cube_mesh`` -- an n^3 grid of the unit cube, six Kuhn tetrahedra per
  cell, interior nodes jittered.
"""
from __future__ import annotations

import numpy as np
import scipy.spatial

# ----------------------------------------------------------------------------
# seeded streams
# ----------------------------------------------------------------------------


def rng(cfg: int, stream: int, item: int = 0) -> np.random.Generator:
    return np.random.default_rng([int(cfg), int(stream), int(item)])


# stream numbers (fixed)
S_JITTER, S_DIAG, S_RHS, S_REPAIR, S_COEF, S_COEF2, S_NOISE, S_DIR, S_SIDES = range(9)


# ----------------------------------------------------------------------------
# helpers
# ----------------------------------------------------------------------------


def boundary_vertices(coords: np.ndarray) -> np.ndarray:
    """Vertices with some coordinate equal to the bounding-box min or max."""
    lo = coords.min(axis=0)
    hi = coords.max(axis=0)
    return np.any((coords == lo) | (coords == hi), axis=1)


def triangle_min_angles(coords: np.ndarray, tris: np.ndarray) -> np.ndarray:
    p = coords[tris]
    out = np.full(len(tris), 180.0)
    for k in range(3):
        u = p[:, (k + 1) % 3] - p[:, k]
        v = p[:, (k + 2) % 3] - p[:, k]
        c = (u * v).sum(1) / (np.linalg.norm(u, axis=1) * np.linalg.norm(v, axis=1))
        out = np.minimum(out, np.degrees(np.arccos(np.clip(c, -1.0, 1.0))))
    return out


def _orient_ccw(coords, tris):
    p = coords[tris]
    det = (p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1]) - (p[:, 1, 1] - p[:, 0, 1]) * (
        p[:, 2, 0] - p[:, 0, 0])
    tris = tris.copy()
    neg = det < 0
    tris[neg, 1], tris[neg, 2] = tris[neg, 2].copy(), tris[neg, 1].copy()
    return tris


def _morton2(ix: np.ndarray, iy: np.ndarray) -> np.ndarray:
    key = np.zeros(len(ix), dtype=np.uint64)
    ix = ix.astype(np.uint64)
    iy = iy.astype(np.uint64)
    for b in range(31):
        key |= ((ix >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b + 1)
        key |= ((iy >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b)
    return key


# ----------------------------------------------------------------------------
# 2-D jittered structured mesh
# ----------------------------------------------------------------------------


def square_mesh(n: int, jitter: float = 0.3, cfg: int = 0, item: int = 0,
                diagonals: str = "random", min_angle: float = 5.0):
    """n x n cells on [0,1]^2, two triangles per cell.

    Returns (coords (V,2) float64, elems (2 n^2, 3) int32, n_repaired).
    Vertices are numbered row-major (x fastest). ``diagonals`` is "random"
    (seeded coin per cell, row-major) or "ur" (every cell split from its
    lower-left to its upper-right corner). Interior nodes get a U(-jitter h,
    jitter h) offset per coordinate (row-major); any interior node touching a
    triangle with an angle below ``min_angle`` degrees is redrawn from the
    repair stream until no such triangle is left.
    """
    h = 1.0 / n
    g = np.arange(n + 1, dtype=np.float64) * h
    g[-1] = 1.0
    X, Y = np.meshgrid(g, g, indexing="xy")
    coords = np.stack([X.ravel(), Y.ravel()], axis=1)
    vid = np.arange((n + 1) * (n + 1)).reshape(n + 1, n + 1)  # [j, i]
    ll = vid[:-1, :-1].ravel()
    lr = vid[:-1, 1:].ravel()
    ul = vid[1:, :-1].ravel()
    ur = vid[1:, 1:].ravel()
    if diagonals == "random":
        flip = rng(cfg, S_DIAG, item).random(n * n) < 0.5
    elif diagonals == "ur":
        flip = np.zeros(n * n, dtype=bool)
    else:
        raise ValueError(diagonals)
    # diagonal ll-ur: (ll, lr, ur), (ll, ur, ul); diagonal lr-ul: (ll, lr, ul), (lr, ur, ul)
    t0 = np.where(flip[:, None], np.stack([ll, lr, ul], 1), np.stack([ll, lr, ur], 1))
    t1 = np.where(flip[:, None], np.stack([lr, ur, ul], 1), np.stack([ll, ur, ul], 1))
    elems = np.empty((2 * n * n, 3), dtype=np.int32)
    elems[0::2] = t0
    elems[1::2] = t1
    interior = ~boundary_vertices(coords)
    repaired = 0
    if jitter > 0:
        idx = np.nonzero(interior)[0]
        base = coords.copy()
        coords = coords.copy()
        coords[idx] += rng(cfg, S_JITTER, item).uniform(-jitter * h, jitter * h, (len(idx), 2))
        rep = rng(cfg, S_REPAIR, item)
        for _ in range(100):
            bad = triangle_min_angles(coords, elems) < min_angle
            if not bad.any():
                break
            nodes = np.unique(elems[bad].ravel())
            nodes = nodes[interior[nodes]]
            repaired += len(nodes)
            coords[nodes] = base[nodes] + rep.uniform(-jitter * h, jitter * h, (len(nodes), 2))
        else:  # pragma: no cover - never reached for jitter <= 0.3
            raise RuntimeError("square_mesh: repair did not converge")
    return coords, elems, repaired


# ----------------------------------------------------------------------------
# 2-D meshes of non-box domains (the general-domain Dirichlet grids of Section 3.4)
# ----------------------------------------------------------------------------


def mesh_boundary(elems: np.ndarray, n_vertices: int) -> np.ndarray:
    """Vertices on an edge that belongs to a single triangle."""
    e = np.sort(np.concatenate([elems[:, [0, 1]], elems[:, [1, 2]], elems[:, [2, 0]]]), axis=1)
    u, c = np.unique(e, axis=0, return_counts=True)
    m = np.zeros(n_vertices, dtype=bool)
    m[u[c == 1].ravel()] = True
    return m


def _compact(coords, elems):
    used = np.unique(elems.ravel())
    new = np.full(len(coords), -1, dtype=np.int64)
    new[used] = np.arange(len(used))
    return coords[used], new[elems].astype(np.int32)


def _jitter_interior(coords, elems, h, jitter, cfg, item, min_angle=5.0):
    bnd = mesh_boundary(elems, len(coords))
    idx = np.nonzero(~bnd)[0]
    base = coords.copy()
    coords = coords.copy()
    coords[idx] += rng(cfg, S_JITTER, item).uniform(-jitter * h, jitter * h, (len(idx), 2))
    rep = rng(cfg, S_REPAIR, item)
    for _ in range(100):
        bad = triangle_min_angles(coords, elems) < min_angle
        if not bad.any():
            return coords
        nodes = np.unique(elems[bad].ravel())
        nodes = nodes[~bnd[nodes]]
        coords[nodes] = base[nodes] + rep.uniform(-jitter * h, jitter * h, (len(nodes), 2))
    raise RuntimeError("repair did not converge")


def lshape_mesh(n: int, jitter: float = 0.3, cfg: int = 5, item: int = 0):
    """L-shaped domain [0,1]^2 minus (1/2,1)^2: the square mesh of side n (n even) without the
    cells of the removed quadrant; interior vertices jittered as in ``square_mesh``.
    Returns (coords, elems, dirichlet) with Dirichlet data on the whole boundary."""
    if n % 2:
        raise ValueError("n must be even")
    coords, elems, _ = square_mesh(n, 0.0, cfg=cfg, item=item)
    cen = coords[elems].mean(axis=1)
    keep = ~((cen[:, 0] > 0.5) & (cen[:, 1] > 0.5))
    coords, elems = _compact(coords, elems[keep])
    if jitter > 0:
        coords = _jitter_interior(coords, elems, 1.0 / n, jitter, cfg, item)
    return coords, elems, mesh_boundary(elems, len(coords))


def annulus_mesh(n: int, r_in: float = 0.2, r_out: float = 0.5, cfg: int = 6, item: int = 0):
    """Annulus centred at (1/2, 1/2): n points on the outer circle, proportionally fewer on the
    inner one, jittered interior points at spacing ~ 2 pi r_out / n, Delaunay, triangles with
    centroid in the hole dropped. Its polygonal boundary lies on no dyadic line.
    Returns (coords, elems, dirichlet) with Dirichlet data on both boundary circles."""
    from scipy.spatial import Delaunay
    h = 2 * np.pi * r_out / n
    c = np.array([0.5, 0.5])
    t_out = 2 * np.pi * np.arange(n) / n
    n_in = max(8, int(round(n * r_in / r_out)))
    t_in = 2 * np.pi * (np.arange(n_in) + 0.5) / n_in
    outer = c + r_out * np.stack([np.cos(t_out), np.sin(t_out)], 1)
    inner = c + r_in * np.stack([np.cos(t_in), np.sin(t_in)], 1)
    g = np.arange(-r_out, r_out + h, h)
    X, Y = np.meshgrid(g, g)
    P = np.stack([X.ravel(), Y.ravel()], 1)
    P += rng(cfg, S_JITTER, item).uniform(-0.25 * h, 0.25 * h, P.shape)
    r = np.hypot(P[:, 0], P[:, 1])
    P = c + P[(r < r_out - 0.5 * h) & (r > r_in + 0.5 * h)]
    coords = np.concatenate([outer, inner, P])
    tri = Delaunay(coords).simplices
    cen = coords[tri].mean(axis=1)
    rc = np.hypot(cen[:, 0] - 0.5, cen[:, 1] - 0.5)
    elems = tri[rc > r_in * np.cos(np.pi / n_in)].astype(np.int32)
    coords, elems = _compact(coords, elems)
    # counter-clockwise orientation
    a = coords[elems]
    det = (a[:, 1, 0] - a[:, 0, 0]) * (a[:, 2, 1] - a[:, 0, 1]) - (a[:, 1, 1] - a[:, 0, 1]) * (a[:, 2, 0] - a[:, 0, 0])
    elems[det < 0] = elems[det < 0][:, [0, 2, 1]]
    return coords, elems, mesh_boundary(elems, len(coords))


# ----------------------------------------------------------------------------
# 2-D graded Delaunay mesh
# ----------------------------------------------------------------------------


def _graded_spacing(x, y, c):
    r = np.hypot(x, y)
    return 1.0 / np.sqrt(c * (1.0 / (r + 0.01) + 1.0))


def _graded_leaves(c, max_level=24):
    out = []
    ix = np.zeros(1, np.int64)
    iy = np.zeros(1, np.int64)
    lev = 0
    while len(ix):
        s = 2.0 ** -lev
        ref = (s > _graded_spacing((ix + 0.5) * s, (iy + 0.5) * s, c)) & (lev < max_level)
        out.append((lev, ix[~ref], iy[~ref]))
        a, b = ix[ref], iy[ref]
        ix = np.concatenate([2 * a, 2 * a + 1, 2 * a, 2 * a + 1])
        iy = np.concatenate([2 * b, 2 * b, 2 * b + 1, 2 * b + 1])
        lev += 1
    return out


def graded_point_count(c):
    return sum(len(a) for _, a, _ in _graded_leaves(c))


def graded_mesh(n_points: int = 1_000_000, cfg: int = 1, item: int = 0, jitter: float = 0.1,
                min_angle: float = 20.0):
    """Delaunay mesh of [0,1]^2 graded towards (0,0); about ``n_points`` vertices.

    Density is proportional to 1/(r+0.01) + 1. The spacing scale c is found by
    bisection so that the quadtree has n_points leaves (within 0.5 %). Each leaf
    contributes its centre jittered by U(-jitter s, jitter s) (s = leaf side);
    leaf corners on the boundary of the square are added so that the hull is
    the square. Vertices are sorted in Morton order of their position.
    Asserts that every triangle has all angles above ``min_angle`` degrees
    after at most a few repair rounds (offending centres redrawn with half the
    jitter). Returns (coords, elems int32, n_repaired).
    """
    lo, hi = 1.0, 1e9
    for _ in range(200):
        mid = np.sqrt(lo * hi)
        cnt = graded_point_count(mid)
        if abs(cnt - n_points) <= 0.005 * n_points:
            break
        if cnt < n_points:
            lo = mid
        else:
            hi = mid
    leaves = _graded_leaves(mid)
    g = rng(cfg, S_JITTER, item)
    centres, sides, bnd = [], [], []
    for lev, ix, iy in leaves:
        if len(ix) == 0:
            continue
        s = 2.0 ** -lev
        centres.append(np.stack([(ix + 0.5) * s, (iy + 0.5) * s], 1))
        sides.append(np.full(len(ix), s))
        for X, Y in ((ix, iy), (ix + 1, iy), (ix, iy + 1), (ix + 1, iy + 1)):
            q = np.stack([X * s, Y * s], 1)
            m = (q[:, 0] == 0) | (q[:, 0] == 1) | (q[:, 1] == 0) | (q[:, 1] == 1)
            bnd.append(q[m])
    C = np.concatenate(centres)
    S = np.concatenate(sides)
    B = np.unique(np.concatenate(bnd), axis=0)
    P = C + g.uniform(-1.0, 1.0, C.shape) * (jitter * S)[:, None]
    # Morton order of position (on a 2^30 grid) for a local vertex numbering
    allp = np.concatenate([P, B])
    q = np.minimum((allp * 2.0 ** 30).astype(np.int64), 2 ** 30 - 1)
    order = np.argsort(_morton2(q[:, 0], q[:, 1]), kind="stable")
    n_c = len(P)
    rep = rng(cfg, S_REPAIR, item)
    repaired = 0
    for _ in range(20):
        coords = allp[order]
        tris = scipy.spatial.Delaunay(coords).simplices.astype(np.int32)
        tris = _orient_ccw(coords, tris)
        bad = triangle_min_angles(coords, tris) <= min_angle
        if not bad.any():
            break
        nodes = order[np.unique(tris[bad].ravel())]
        nodes = nodes[nodes < n_c]
        repaired += len(nodes)
        allp[nodes] = C[nodes] + rep.uniform(-1.0, 1.0, (len(nodes), 2)) * (0.5 * jitter * S[nodes])[:, None]
    else:  # pragma: no cover
        raise RuntimeError("graded_mesh: minimum-angle repair did not converge")
    return coords, tris, repaired


# ----------------------------------------------------------------------------
# 3-D Kuhn cube mesh
# ----------------------------------------------------------------------------

_KUHN_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


def kuhn_cube_mesh(n: int, jitter: float = 0.2, cfg: int = 2, item: int = 0):
    """n^3 cells on [0,1]^3, six Kuhn tetrahedra per cell sharing the main diagonal.

    Vertex (i, j, k) has id i + (n+1) (j + (n+1) k). Cells are visited with i
    fastest; tetrahedra follow the permutation order (0,1,2), (0,2,1), (1,0,2),
    (1,2,0), (2,0,1), (2,1,0): vertices 0, e_p0, e_p0 + e_p1, (1,1,1).
    Returns (coords, elems int32 (6 n^3, 4), cell index of each element (n^3*6,3)).
    """
    h = 1.0 / n
    g = np.arange(n + 1, dtype=np.float64) * h
    g[-1] = 1.0
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    coords = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    m = n + 1

    def vid(i, j, k):
        return i + m * (j + m * k)

    kk, jj, ii = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ii, jj, kk = ii.ravel(), jj.ravel(), kk.ravel()
    elems = np.empty((6 * n ** 3, 4), dtype=np.int32)
    e = np.eye(3, dtype=np.int64)
    for t, p in enumerate(_KUHN_PERMS):
        a = np.zeros(3, np.int64)
        verts = [a.copy()]
        a = a + e[p[0]]
        verts.append(a.copy())
        a = a + e[p[1]]
        verts.append(a.copy())
        verts.append(np.ones(3, np.int64))
        for q, v in enumerate(verts):
            elems[t::6, q] = vid(ii + v[0], jj + v[1], kk + v[2])
    cells = np.repeat(np.stack([ii, jj, kk], 1), 6, axis=0)
    if jitter > 0:
        interior = ~boundary_vertices(coords)
        idx = np.nonzero(interior)[0]
        coords = coords.copy()
        coords[idx] += rng(cfg, S_JITTER, item).uniform(-jitter * h, jitter * h, (len(idx), 3))
    return coords, elems, cells


def checkerboard_kappa(cells: np.ndarray, n: int, blocks: int = 8, cfg: int = 2, item: int = 0,
                       high: float = 10.0) -> np.ndarray:
    """Coefficient in {1, high} on a blocks^3 checkerboard of cells with a seeded phase."""
    b = cells // (n // blocks)
    s = int(rng(cfg, S_COEF, item).integers(0, 2))
    return np.where(((b.sum(1) + s) % 2) == 0, high, 1.0)


# ----------------------------------------------------------------------------
# right-hand sides and coefficients
# ----------------------------------------------------------------------------


def rhs_per_vertex(n_vertices: int, cfg: int, item: int = 0, n_rhs: int = 1) -> np.ndarray:
    """f ~ U[-1, 1], drawn per vertex (a solver keeps the entries of its unknowns)."""
    f = rng(cfg, S_RHS, item).uniform(-1.0, 1.0, (n_rhs, n_vertices))
    return f[0] if n_rhs == 1 else f


def lognormal_kappa(n_elems: int, sigma: float, cfg: int, item: int = 0, stream: int = S_COEF):
    """kappa = exp(g), g ~ N(0, sigma^2) per element. Returns (g, kappa)."""
    g = rng(cfg, stream, item).normal(0.0, sigma, n_elems)
    return g, np.exp(g)


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------


def make_config(cfg: int, scale: float = 1.0, item: int = 0) -> dict:
    """Build workload ``cfg`` (0..4). ``scale`` shrinks the mesh for tests (1.0 = full size).

    Returns a dict with keys: dim, coords, elems, kappa, f_vertex (per-vertex
    draw), name, and extras per workload.
    """
    if cfg == 0:
        n = max(4, int(round(64 * scale)))
        coords, elems, rep = square_mesh(n, 0.3, cfg=0, item=item)
        kappa = np.ones(len(elems))
        name = f"square{n}x{n} jitter0.3 kappa1"
        out = dict(dim=2, n=n, repaired=rep)
    elif cfg == 1:
        npts = max(200, int(round(1_000_000 * scale)))
        coords, elems, rep = graded_mesh(npts, cfg=1, item=item)
        _, kappa = lognormal_kappa(len(elems), 0.5, cfg=1, item=item)
        name = f"graded-delaunay {len(coords)} vertices, kappa=exp(N(0,0.5^2))"
        out = dict(dim=2, repaired=rep)
    elif cfg == 2:
        n = max(8, int(round(128 * scale)))
        n = 8 * max(1, n // 8)
        coords, elems, cells = kuhn_cube_mesh(n, 0.2, cfg=2, item=item)
        kappa = checkerboard_kappa(cells, n, 8, cfg=2, item=item)
        name = f"kuhn-cube {n}^3 x6 jitter0.2 checkerboard8^3 kappa{{1,10}}"
        out = dict(dim=3, n=n)
    elif cfg == 4:
        n = max(4, int(round(724 * scale)))
        coords, elems, rep = square_mesh(n, 0.3, cfg=4, item=item)
        m, kappa = lognormal_kappa(len(elems), 0.3, cfg=4, item=item, stream=S_COEF)
        m2, _ = lognormal_kappa(len(elems), 0.3, cfg=4, item=item, stream=S_COEF2)
        noise = rng(4, S_NOISE, item).normal(0.0, 1e-3, len(coords))
        dirs = rng(4, S_DIR, item).normal(0.0, 1.0, (20, len(elems)))
        name = f"square{n}x{n} jitter0.3 adjoint m~N(0,0.3^2)"
        out = dict(dim=2, n=n, m=m, m_obs=m2, noise_vertex=noise, directions=dirs, repaired=rep)
    elif cfg == 3:
        raise ValueError("use batched_config() for the batched workload")
    else:
        raise ValueError(cfg)
    out.update(coords=coords, elems=elems.astype(np.int32), kappa=kappa,
               f_vertex=rhs_per_vertex(len(coords), cfg, item), name=name, cfg=cfg)
    return out


def batched_config(n_meshes: int = 256, side_lo: int = 32, side_hi: int = 512, n_rhs: int = 4,
                   item: int = 0) -> list:
    """The batched workload: ``n_meshes`` jittered square meshes, sides ~ U{side_lo..side_hi}.

    Mesh m uses item = m of the config-3 streams; each carries ``n_rhs``
    per-vertex right-hand sides.
    """
    sides = rng(3, S_SIDES, item).integers(side_lo, side_hi + 1, n_meshes)
    out = []
    for m, s in enumerate(sides):
        coords, elems, rep = square_mesh(int(s), 0.3, cfg=3, item=m)
        out.append(dict(dim=2, n=int(s), coords=coords, elems=elems, kappa=np.ones(len(elems)),
                        f_vertex=rhs_per_vertex(len(coords), 3, m, n_rhs), repaired=rep))
    return out
