// Setup steps on the device (tree.hip, assemble.hip), option setup_device.
#pragma once

#include "setup.hpp"

namespace asmg {

// Root box, element keys, refined sets R0 and R (closure), leaves, J and kappa~ of h, as
// build_tree computes them on the host, built on HIP device `ordinal`.
void build_tree_device(Hierarchy &h, int ordinal);

// Dirichlet mask and unknown numbering (host, fine_dofs), then the pattern and values of the
// fine matrix A on HIP device `ordinal`, bit-identical to build_fine.
void build_fine_device(Hierarchy &h, int ordinal);

// Level meshes sigma^(l) from J down to the bottom level l_c (and the kappa~ means per Kuhn
// simplex) on HIP device `ordinal`, identical to build_level_meshes; returns false without
// building anything on a general domain or when vertex keys exceed 64 bits ((J+1) d > 64).
bool build_level_meshes_device(Hierarchy &h, int ordinal);

// A_l of every level l_c..J (Section 4.1: the P1 stiffness matrix of sigma^(l) with the
// auxiliary coefficient kappa~ per Kuhn simplex) from the level meshes already built on the host
// (build_level_meshes), assembled on HIP device `ordinal`, bit-identical to the host assembly.
void assemble_levels_device(Hierarchy &h, int ordinal);

// P_l of every level l_c < l <= J (nodal interpolation by exact point location) on HIP device
// `ordinal`, bit-identical to the host's; returns false without building anything when the
// integer coordinates are too large for exact int64 determinants (2-D: J > 30, 3-D: J > 19).
bool prolongations_device(Hierarchy &h, int ordinal);

// The Scott-Zhang transfer Pi (one thread per unknown: sigma_i, the leaves meeting it, exact
// clipping against sigma^(J) and quadrature) on HIP device `ordinal`, identical to
// build_transfer; returns false without building anything when the sizes exceed 32-bit indices
// (the caller then builds Pi on the host).
bool build_transfer_device(Hierarchy &h, int ordinal);

// Colourings of the original grid and the smoothed auxiliary levels in the hash order (option
// colouring = 1) on HIP device `ordinal` by Jones-Plassmann rounds: identical to
// build_colourings. Throws ASMG_EINVAL for the other orders.
void build_colourings_device(Hierarchy &h, int ordinal);

}  // namespace asmg
