// Cluster tree on the device (tree.hip).
#pragma once

#include "setup.hpp"

namespace asmg {

// Root box, element keys, refined sets R0 and R (closure), leaves, J and kappa~ of h, as
// build_tree computes them on the host, built on HIP device `ordinal`.
void build_tree_device(Hierarchy &h, int ordinal);

}  // namespace asmg
