"""Everything the solve needs for one mesh, assembled by the oracle modules.

``domain="box"`` builds the Dirichlet auxiliary grids on the root box (every simplex of
sigma^(l)); ``domain="mesh"`` keeps only the simplices inside the mesh's own domain
(``domain``, 2-D); ``domain="mixed"`` builds the mixed Dirichlet/Neumann grids (simplices that
meet the domain and not its Dirichlet boundary, 2-D).

``Hierarchy(coords, elems, kappa)`` builds the fine matrix (``fem``), the closed
box tree (``cluster``), the level meshes (``auxgrid``), the auxiliary operators
(``auxops``), the transfer Pi (``transfer``) and the colourings (``colour``).
``solve(f, tol)`` runs PCG (``pcg``) with B_co (``asmg``).
"""
from __future__ import annotations

import numpy as np

from . import asmg, auxgrid, auxops, cluster, colour, fem, pcg, transfer


class Hierarchy:
    def __init__(self, coords, elems, kappa, dirichlet=None, n_min=None, coarse_max_dofs=1024,
                 colour_seed=0, check_literal=False, colouring="smallest_last", domain="box"):
        coords = np.asarray(coords, dtype=np.float64)
        elems = np.asarray(elems, dtype=np.int64)
        self.coords = coords
        self.elems = elems
        self.kappa = np.asarray(kappa, dtype=np.float64)
        self.d = coords.shape[1]
        if domain in ("mesh", "mixed") and dirichlet is None:
            from .domain import boundary_vertices
            dirichlet = boundary_vertices(elems, len(coords))
        self.A, self.dofs = fem.assemble(coords, elems, self.kappa, dirichlet)
        # no Dirichlet vertex: a pure Neumann problem (A singular, constants in its kernel)
        self.pure_neumann = len(self.dofs) == len(coords)
        self.tree = cluster.BoxTree(coords, elems, n_min, check_literal=check_literal)
        if domain not in ("box", "mesh", "mixed"):
            raise ValueError(domain)
        dom = None
        if domain == "mesh":       # Section 3.4 on the mesh's own (2-D polygonal) domain
            from .domain import Domain
            dom = Domain(coords, elems)
        if domain == "mixed":      # the mixed Dirichlet/Neumann grids (remark of Section 3.5)
            from .domain import Domain
            mask = np.zeros(len(coords), dtype=bool)
            mask[np.setdiff1d(np.arange(len(coords)), self.dofs)] = True
            dom = Domain(coords, elems, mask)
        self.meshes = auxgrid.AuxMeshes(self.tree, dom, mixed=(domain == "mixed"))
        self.aux = auxops.AuxOperators(self.tree, self.meshes, self.kappa, coarse_max_dofs)
        self.Pi = transfer.transfer(self.tree, self.meshes, coords, elems, self.dofs)
        self.colour_fine = colour.greedy_colouring(self.A, colour_seed, colouring)
        self.colour_aux = {l: colour.greedy_colouring(self.aux.A[l], colour_seed, colouring)
                           for l in range(self.aux.lc + 1, self.aux.J + 1)}
        self._B = {}

    @property
    def n(self):
        return len(self.dofs)

    def preconditioner(self, dtype=np.float64, nu_aux=2, nu_fine=1, smoothing="full", nb_layers=0):
        key = (np.dtype(dtype).name, nu_aux, nu_fine, smoothing, nb_layers)
        if key not in self._B:
            self._B[key] = asmg.ASMGPreconditioner(self, dtype, nu_aux, nu_fine, smoothing, nb_layers)
        return self._B[key]

    def solve(self, f, tol=1e-8, max_iter=1000, mixed=False, record=False, nu_aux=2, nu_fine=1,
              smoothing="full", nested=0, nb_layers=0):
        """PCG with B_co; ``nested`` > 0 starts from the nested iteration's guess with that many
        V-cycles per auxiliary level (in the preconditioner's precision); ``nb_layers`` > 0 adds
        the near-boundary correction with that many layers.

        Pure Neumann problem (every vertex an unknown, A singular with the constants as its
        kernel): the solvable part of f is solved, f minus its mean (the projection onto the
        range of A), and u is returned with zero mean; the stopping rule is relative to the
        projected f."""
        if self.pure_neumann:
            f = np.asarray(f, dtype=np.float64)
            f = f - f.mean()
        B = self.preconditioner(np.float32 if mixed else np.float64, nu_aux, nu_fine, smoothing, nb_layers)
        if mixed:
            def Bm(r):
                return B(r.astype(np.float32)).astype(np.float64)
        else:
            Bm = B
        u0 = None
        if nested > 0 and np.any(np.asarray(f) != 0):
            u0 = np.asarray(B.nested_guess(f, nested)).astype(np.float64)
        u, it, info = pcg.pcg(self.A, f, Bm, tol, max_iter, record, u0=u0)
        if self.pure_neumann:
            u = u - u.mean()
        return u, it, info

    def level_sizes(self):
        return {l: self.meshes.level(l).n for l in range(1, self.tree.J + 1)}
