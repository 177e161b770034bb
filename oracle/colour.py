"""Deterministic multicolour ordering for Gauss-Seidel (oracle).

Section 4.1 takes S = (D - L)^(-1), Gauss-Seidel, as the smoother. A sequential
sweep cannot run in parallel, so both the oracle and the GPU path run
Gauss-Seidel in a colour-major ordering pi. Inside a colour the unknowns are
pairwise uncoupled, so S = (D - L_pi)^(-1) can be applied one colour at a time.
The colouring is part of the method's definition here and both sides compute the
same one.

* Unknowns are coloured greedily. Each one takes the smallest colour not used
  by an already-coloured neighbour in the stored sparsity pattern.
* Default order ("natural"): ascending unknown index. The unknowns are numbered
  in Morton order of position on the auxiliary grids, and in the mesh's own
  order on the original grid. This gives the checkerboard on uniform 5-point
  regions and few colours elsewhere.
* Alternative order ("hash"): descending priority w(i) = (fmix32(i XOR seed), i),
  compared lexicographically, where fmix32 is the public-domain MurmurHash3
  32-bit finaliser. This is the order Jones-Plassmann reproduces in parallel.

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


def colour_classes(colour: np.ndarray):
    """Unknowns of each colour, ascending index."""
    C = int(colour.max()) + 1 if len(colour) else 0
    return [np.nonzero(colour == c)[0] for c in range(C)]
