// Host-side setup of the ASMG hierarchy: data structures shared by the setup,
// the device upload and the C ABI. Everything here is plain C++17.
#pragma once

#include <array>
#include <cstdint>
#include <memory>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/asmg.h"

namespace asmg {

struct AsmgError {
  int code;
  std::string msg;
};

// Compressed sparse rows with int64 row pointers, int32 columns, FP64 values.
struct Csr {
  int64_t nrows = 0, ncols = 0;
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<double> v;
  int64_t nnz() const { return rp.empty() ? 0 : rp.back(); }
};

// Box of the regular box tree, encoded as a locational code:
// (1 << d*(level-1)) | Morton(index), axis 0 most significant in each bit group.
using BoxCode = uint64_t;
using KuhnW = std::array<double, 6>;  // one value per Kuhn simplex of a box (2 in 2-D, 6 in 3-D)

// One auxiliary triangulation sigma^(level) (Section 3.3).
struct LevelMesh {
  int level = 0;
  std::vector<int64_t> verts;       // nv * d integer coordinates (units of L 2^-J), Morton order
  std::vector<int64_t> simp;        // ns * (d+1) vertex indices
  std::vector<int32_t> simp_box;    // box index of each simplex
  std::vector<int8_t> simp_tmpl;    // template position (Kuhn permutation for non-fan boxes)
  std::vector<BoxCode> boxes;       // active boxes, Morton order of lower corners
  std::vector<uint8_t> fan;         // fan flag per box
  std::vector<int64_t> box_simp;    // simplex range per box (nb + 1)
  std::unordered_map<BoxCode, int32_t> box_index;
  std::vector<uint8_t> kept;        // general domain: simplex inside the domain (empty = all kept)
  std::vector<int64_t> dof_vert;    // vertex index of each unknown
  std::vector<int64_t> dof_of_vert; // unknown index of each vertex (-1 on the boundary)
  int64_t nverts() const { return (int64_t)dof_of_vert.size(); }
  int64_t n() const { return (int64_t)dof_vert.size(); }
};

struct DomainIndex;  // boundary edges and bucket grids of a general 2-D domain (domain.cpp)

// Near-boundary set J_{l,j} of one auxiliary level (Section 3.5) and the exact solver of A_l
// restricted to it (nearbnd.cpp)
struct NearBnd {
  std::vector<int64_t> J;        // level unknowns in the solver's order
  bool dense = true;             // dense: `inv` is the |J|^2 inverse (regularised where singular)
  std::vector<double> inv;
  // domain decomposition: interiors of the pieces [poff[p], poff[p+1]) of J, then the separator
  // [nI, |J|); dense inverses of the interior blocks at boff[p]; couplings A_SI (rows separator,
  // columns interior position) and A_IS (rows interior, columns separator position); the inverse
  // of the Schur complement on the separator
  int nI = 0;
  std::vector<int64_t> poff, boff;
  std::vector<double> blocks;
  Csr ASI, AIS;
  std::vector<double> sinv;
};

struct Hierarchy {
  // input
  int d = 2;
  int64_t nv = 0, ne = 0;
  std::vector<double> coords;
  std::vector<int32_t> elems;
  std::vector<double> kappa;
  std::vector<uint8_t> dirichlet;
  asmg_options opt{};
  int threads = 0;  // host threads for the setup (0 = all cores)
  // setup stages that ran on the device (bits: 1 fine matrix, 2 cluster tree, 4 level meshes,
  // 8 A_l, 16 P_l, 32 Pi, 64 colourings)
  int64_t device_stages = 0;
  std::vector<double> setup_seconds;  // wall time of the setup phases: fine, tree, levels,
                                      // transfer, colourings, coarse, upload

  // fine problem (Section 2)
  std::vector<int64_t> dofs;          // vertex id per unknown
  std::vector<int64_t> dof_of_vertex; // -1 for Dirichlet vertices
  Csr A;                              // unknown order, diagonal included
  std::vector<double> K1;             // per-element stiffness at kappa = 1, ne * (d+1)^2

  // cluster tree (Sections 3.1-3.2)
  double a[3] = {0, 0, 0};
  double L = 1;
  std::vector<int64_t> keys;          // ne * d
  std::unordered_set<BoxCode> R0, R;  // refined boxes before / after closure
  std::vector<BoxCode> leaves;        // sorted by (level, index)
  std::unordered_map<BoxCode, double> leaf_kappa;
  std::unordered_map<BoxCode, KuhnW> kuhn_w;  // mean coefficient per Kuhn simplex of a box
  int J = 1;

  // auxiliary hierarchy (Sections 3.3-3.4, 4.1)
  std::shared_ptr<DomainIndex> domain;  // general domain (option domain = 1), else null
  std::unordered_map<int, LevelMesh> meshes;
  std::vector<int64_t> level_n;       // unknowns of levels 1..J (index level-1)
  int lc = 1;
  std::unordered_map<int, Csr> Al;    // lc..J
  std::unordered_map<int, Csr> P;     // lc+1..J
  Csr Pi;                             // fine unknowns x level-J unknowns
  std::vector<int32_t> colour_fine;
  std::unordered_map<int, std::vector<int32_t>> colour_aux;  // lc+1..J
  std::unordered_map<int, std::vector<uint8_t>> local_set;   // N~_l, lc+1..J (1 = smoothed locally)
  int64_t nc = 0;
  std::vector<double> coarse_inv;     // nc * nc, row-major, explicit inverse of A_lc (regularised
                                      // on components with zero row sums: pure Neumann problems)
  std::unordered_map<int, NearBnd> nb;  // near-boundary correction, lc+1..J (option nb_layers)

  int64_t n() const { return (int64_t)dofs.size(); }
};

// setup steps (setup.cpp)
void fine_dofs(Hierarchy &h);   // Dirichlet mask (default rules), unknown numbering
void build_fine(Hierarchy &h);  // fine_dofs, then the pattern and values of A
void assemble_fine_values(Hierarchy &h);
void build_tree(Hierarchy &h);
void build_levels(Hierarchy &h);  // build_level_meshes, then build_level_operators(h, true)
// kappa~ means per Kuhn simplex, the level meshes sigma^(l) from J down to the bottom level l_c
void build_level_meshes(Hierarchy &h);
// kappa~ means per Kuhn simplex of every box (the level matrices' coefficients)
void compute_level_means(Hierarchy &h);
// A_l (l_c <= l <= J) and P_l (l_c < l <= J); `assemble` / `prolong` false: that one is
// already built (on the device)
void build_level_operators(Hierarchy &h, bool assemble, bool prolong = true);
void assemble_aux_values(Hierarchy &h);
void build_transfer(Hierarchy &h);
void build_colourings(Hierarchy &h);
void build_local_sets(Hierarchy &h);
void build_domain(Hierarchy &h);
std::vector<uint8_t> domain_keeps(const Hierarchy &h, const LevelMesh &lm);
// mixed Dirichlet/Neumann grids: kept (meets the domain, not Gamma_D) and touch (meets Gamma_D)
void domain_mixed(const Hierarchy &h, const LevelMesh &lm, std::vector<uint8_t> &kept,
                  std::vector<uint8_t> &touch);
void build_coarse(Hierarchy &h);
// near-boundary correction (nearbnd.cpp): J_{l,j} of a level, and every level's set and solver
std::vector<int64_t> near_boundary_set(Hierarchy &h, int level, int layers);
void build_near_boundary(Hierarchy &h);
// M (n x n symmetric, row-major) replaced by its inverse; with `regularised`, each connected
// component whose rows sum to zero first gets gamma 1 1^T (gamma = mean diagonal / size)
void spd_inverse(std::vector<double> &M, int64_t n, int threads, bool regularised);
const LevelMesh &level_mesh(Hierarchy &h, int level);
// position of every unknown of the original grid in Morton order of its vertex (device layout)
std::vector<int> morton_rank(const Hierarchy &h);
// element stiffness at kappa = 1 (|tau| grad(lambda_i).grad(lambda_j))
void element_unit_stiffness(const Hierarchy &h, int64_t e, double K[4][4]);

// helpers
int box_level(BoxCode c, int d);
void box_index(BoxCode c, int d, int64_t *idx);
BoxCode box_code(int level, const int64_t *idx, int d);

}  // namespace asmg
