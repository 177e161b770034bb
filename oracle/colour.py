"""Deterministic multicolour ordering for Gauss-Seidel (oracle).

Section 4.1 takes S = (D - L)^(-1), Gauss-Seidel, as the smoother. A sequential
sweep cannot run in parallel, so both the oracle and the GPU path run
Gauss-Seidel in a colour-major ordering pi. Inside a colour the unknowns are
pairwise uncoupled, so S = (D - L_pi)^(-1) can be applied one colour at a time.
The colouring is part of the method's definition here and both sides compute the
same one.

* Unknowns are coloured greedily. Each one takes the smallest colour not used
  by an already-coloured neighbour in the stored sparsity pattern.
* Order "natural": ascending unknown index. The unknowns are numbered in Morton
  order of position on the auxiliary grids, and in the mesh's own order on the
  original grid. This gives the checkerboard on uniform 5-point regions.
* Order "hash": descending priority w(i) = (fmix32(i XOR seed), i),
  compared lexicographically, where fmix32 is the public-domain MurmurHash3
  32-bit finaliser. This is the order Jones-Plassmann reproduces in parallel.
* Order "smallest_last" (Matula and Beck's smallest-last ordering; the default
  of the solver, ``Hierarchy``):
  repeatedly remove the remaining unknown of smallest (current degree, index),
  degrees counted in the graph of the remaining unknowns, and colour greedily in
  the reverse of the removal order. Every unknown then has at most the graph's
  degeneracy of neighbours coloured before it, so at most degeneracy + 1 colours
  are used (at most 6 on a planar graph); fewer colours mean fewer passes.

Pins: the colouring is proper; the ordering reproduces the textbook GS bounds
(Jacobi continuity ||v||_A^2 <= K <D v, v>, and the Gauss-Seidel continuity
lemma (1/K) <(D-L) x, x> <= <D x, x> <= 2 <(D-L) x, x>) on random vectors.
"""
from __future__ import annotations

import numpy as np

M32 = 0xFFFFFFFF


def fmix32(h: np.ndarray) -> np.ndarray:
    h = np.asarray(h, dtype=np.uint64) & M32
    h ^= h >> np.uint64(16)
    h = (h * np.uint64(0x85EBCA6B)) & np.uint64(M32)
    h ^= h >> np.uint64(13)
    h = (h * np.uint64(0xC2B2AE35)) & np.uint64(M32)
    h ^= h >> np.uint64(16)
    return h


def greedy_colouring(A, seed: int = 0, mode: str = "natural") -> np.ndarray:
    """Colour of every row of the square sparse matrix A (pattern only, diagonal ignored)."""
    A = A.tocsr()
    n = A.shape[0]
    idx = np.arange(n, dtype=np.int64)
    if mode == "natural":
        order = idx
    elif mode == "smallest_last":
        order = smallest_last_order(A)
    elif mode == "hash":
        w = fmix32((idx ^ int(seed)) & M32)
        order = np.lexsort((idx, w))[::-1]      # descending (w, i)
    else:
        raise ValueError(mode)
    colour = np.full(n, -1, dtype=np.int64)
    ip, ix = A.indptr, A.indices
    for i in order:
        nb = ix[ip[i]:ip[i + 1]]
        used = set(colour[nb].tolist())
        c = 0
        while c in used:
            c += 1
        colour[i] = c
    return colour


def smallest_last_order(A):
    """Colouring order of the smallest-last rule: the reverse of the removal order, where each
    step removes the remaining row of smallest (degree among remaining rows, row index)."""
    import heapq
    A = A.tocsr()
    n = A.shape[0]
    ip, ix = A.indptr, A.indices
    nbrs = [[int(j) for j in ix[ip[i]:ip[i + 1]] if j != i] for i in range(n)]
    deg = [len(nb) for nb in nbrs]
    removed = [False] * n
    heap = [(deg[i], i) for i in range(n)]
    heapq.heapify(heap)
    removal = []
    while heap:
        d, i = heapq.heappop(heap)
        if removed[i] or d != deg[i]:
            continue                      # stale entry: i's degree has dropped since
        removed[i] = True
        removal.append(i)
        for j in nbrs[i]:
            if not removed[j]:
                deg[j] -= 1
                heapq.heappush(heap, (deg[j], j))
    return np.array(removal[::-1], dtype=np.int64)


def colour_classes(colour: np.ndarray):
    """Unknowns of each colour, ascending index."""
    C = int(colour.max()) + 1 if len(colour) else 0
    return [np.nonzero(colour == c)[0] for c in range(C)]
