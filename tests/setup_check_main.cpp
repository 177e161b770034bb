// Host-only driver of the whole host setup (setup.cpp, domain.cpp, nearbnd.cpp), for runs under
// AddressSanitizer and UndefinedBehaviorSanitizer: no HIP code is built into it.
//
// Usage: setup_check <mesh.bin>
//   mesh.bin: int32 dim, int64 n_vertices, int64 n_elements, int32 domain, int32 has_mask;
//   then coords (n_vertices*dim doubles), elems (n_elements*(dim+1) int32), kappa (n_elements
//   doubles) and, if has_mask, one uint8 Dirichlet flag per vertex.
// Prints the hierarchy's sizes; exits non-zero on a setup error.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "setup.hpp"

using namespace asmg;

int main(int argc, char **argv) {
  if (argc != 2) {
    std::fprintf(stderr, "usage: %s mesh.bin\n", argv[0]);
    return 2;
  }
  std::FILE *f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t dim = 0, domain = 0, has_mask = 0;
  int64_t nv = 0, ne = 0;
  bool ok = std::fread(&dim, 4, 1, f) == 1 && std::fread(&nv, 8, 1, f) == 1 && std::fread(&ne, 8, 1, f) == 1 &&
            std::fread(&domain, 4, 1, f) == 1 && std::fread(&has_mask, 4, 1, f) == 1;
  Hierarchy h;
  if (ok) {
    h.d = dim;
    h.nv = nv;
    h.ne = ne;
    h.coords.resize((size_t)nv * dim);
    h.elems.resize((size_t)ne * (dim + 1));
    h.kappa.resize((size_t)ne);
    ok = std::fread(h.coords.data(), 8, h.coords.size(), f) == h.coords.size() &&
         std::fread(h.elems.data(), 4, h.elems.size(), f) == h.elems.size() &&
         std::fread(h.kappa.data(), 8, h.kappa.size(), f) == h.kappa.size();
    if (ok && has_mask) {
      h.dirichlet.resize((size_t)nv);
      ok = std::fread(h.dirichlet.data(), 1, h.dirichlet.size(), f) == h.dirichlet.size();
    }
  }
  std::fclose(f);
  if (!ok) return 2;
  // the library's defaults (asmg_default_options lives with the device code)
  h.opt = asmg_options{};
  h.opt.nu_aux = 2;
  h.opt.nu_fine = 1;
  h.opt.coarse_max_dofs = 1024;
  h.opt.max_iter = 1000;
  h.opt.colouring = 2;
  h.opt.autotune = 1;
  h.opt.domain = domain;
  h.opt.device = -1;
  h.opt.nb_layers = 2;  // the near-boundary sets and their exact solvers are built too
  try {
    build_fine(h);
    build_tree(h);
    if (domain >= 1) build_domain(h);
    build_levels(h);
    build_transfer(h);
    build_colourings(h);
    build_local_sets(h);
    build_coarse(h);
    build_near_boundary(h);
  } catch (const AsmgError &e) {
    std::fprintf(stderr, "setup error %d: %s\n", e.code, e.msg.c_str());
    return 1;
  }
  std::printf("n %lld J %d lc %d nnz_A %lld\n", (long long)h.n(), h.J, h.lc, (long long)h.A.nnz());
  return 0;
}
