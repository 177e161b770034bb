// Host-side construction of the ASMG hierarchy.
//
//   build_fine        P1 stiffness pattern and values, Dirichlet elimination (Section 2, eq. (2))
//   build_tree        barycenters, box keys, cluster tree and closure (Sections 3.1-3.2)
//   level_mesh        nested conforming auxiliary triangulations sigma^(l) (Section 3.3),
//                     Dirichlet auxiliary grids of a box domain (Section 3.4)
//   build_levels      choice of the V-cycle bottom, A_l and P_l patterns (Section 4.1)
//   build_transfer    Scott-Zhang transfer Pi (Section 4.1)
//   build_colourings  multicolour orderings for Gauss-Seidel
//   build_coarse      Cholesky factor and explicit inverse of the bottom matrix (Algorithm 2, B_0)
//
// Index maps (keys, refined boxes, vertices, simplices, unknown numbering, patterns,
// colourings) are exact integer computations. The floating-point steps that feed
// them (barycenters, keys) use plain IEEE operations in a fixed order and are
// compiled without floating-point contraction.
#include "setup.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <atomic>
#include <exception>
#include <mutex>
#include <numeric>
#include <queue>
#include <thread>

namespace asmg {

[[noreturn]] static void fail(int code, const std::string &m) { throw AsmgError{code, m}; }

// run f(i) for i in [0, n) on up to h.threads host threads (0 = all cores); the first error is rethrown
template <class F>
static void parallel_for(const Hierarchy &h, int64_t n, F f) {
  int nt = h.threads > 0 ? h.threads : (int)std::thread::hardware_concurrency();
  nt = (int)std::max<int64_t>(1, std::min<int64_t>(nt, n));
  if (nt == 1) {
    for (int64_t i = 0; i < n; ++i) f(i);
    return;
  }
  std::atomic<int64_t> next{0};
  std::mutex mu;
  std::exception_ptr err;
  auto work = [&]() {
    try {
      while (true) {
        const int64_t i = next.fetch_add(1);
        if (i >= n) return;
        f(i);
      }
    } catch (...) {
      std::lock_guard<std::mutex> g(mu);
      if (!err) err = std::current_exception();
      next = n;
    }
  };
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t) th.emplace_back(work);
  for (auto &t : th) t.join();
  if (err) std::rethrow_exception(err);
}

static constexpr int key_bits(int d) { return d == 2 ? 30 : 20; }

// ---------------------------------------------------------------------------
// box codes
// ---------------------------------------------------------------------------

BoxCode box_code(int level, const int64_t *idx, int d) {
  BoxCode m = 0;
  const int bits = level - 1;
  for (int b = 0; b < bits; ++b)
    for (int k = 0; k < d; ++k) m |= (BoxCode)((idx[k] >> b) & 1) << (b * d + (d - 1 - k));
  return m | ((BoxCode)1 << (d * bits));
}

int box_level(BoxCode c, int d) { return (63 - __builtin_clzll(c)) / d + 1; }

void box_index(BoxCode c, int d, int64_t *idx) {
  const int bits = box_level(c, d) - 1;
  for (int k = 0; k < d; ++k) idx[k] = 0;
  for (int b = 0; b < bits; ++b)
    for (int k = 0; k < d; ++k) idx[k] |= (int64_t)((c >> (b * d + (d - 1 - k))) & 1) << b;
}

// same-level offsets of boxes sharing a facet, or (3-D) an edge
static std::vector<std::array<int, 3>> touch_offsets(int d) {
  std::vector<std::array<int, 3>> out;
  for (int x = -1; x <= 1; ++x)
    for (int y = -1; y <= 1; ++y)
      for (int z = (d == 3 ? -1 : 0); z <= (d == 3 ? 1 : 0); ++z) {
        int nz = (x != 0) + (y != 0) + (z != 0);
        if (nz == 1 || (d == 3 && nz == 2)) out.push_back({x, y, z});
      }
  return out;
}

static inline bool offset_box(BoxCode b, const std::array<int, 3> &o, int d, BoxCode *out) {
  int64_t idx[3];
  box_index(b, d, idx);
  const int lev = box_level(b, d);
  const int64_t n = (int64_t)1 << (lev - 1);
  for (int k = 0; k < d; ++k) {
    idx[k] += o[k];
    if (idx[k] < 0 || idx[k] >= n) return false;
  }
  *out = box_code(lev, idx, d);
  return true;
}

// Morton key of integer points with `bits` bits per axis (axis 0 most significant)
static inline unsigned __int128 morton_point(const int64_t *X, int d, int bits) {
  unsigned __int128 m = 0;
  for (int b = 0; b < bits; ++b)
    for (int k = 0; k < d; ++k) m |= (unsigned __int128)((X[k] >> b) & 1) << (b * d + (d - 1 - k));
  return m;
}

// bit b of x moved to bit d*b (x below 2^32 for d = 2, below 2^21 for d = 3): mask-and-shift
// bit interleaving
static inline uint64_t spread_bits(uint64_t x, int d) {
  if (d == 2) {
    x &= 0xffffffffULL;
    x = (x | (x << 16)) & 0x0000ffff0000ffffULL;
    x = (x | (x << 8)) & 0x00ff00ff00ff00ffULL;
    x = (x | (x << 4)) & 0x0f0f0f0f0f0f0f0fULL;
    x = (x | (x << 2)) & 0x3333333333333333ULL;
    x = (x | (x << 1)) & 0x5555555555555555ULL;
  } else {
    x &= 0x1fffffULL;
    x = (x | (x << 32)) & 0x001f00000000ffffULL;
    x = (x | (x << 16)) & 0x001f0000ff0000ffULL;
    x = (x | (x << 8)) & 0x100f00f00f00f00fULL;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ULL;
    x = (x | (x << 2)) & 0x1249249249249249ULL;
  }
  return x;
}

// morton_point for keys of at most 64 bits (same bit layout)
static inline uint64_t morton_point64(const int64_t *X, int d) {
  uint64_t m = 0;
  for (int k = 0; k < d; ++k) m |= spread_bits((uint64_t)X[k], d) << (d - 1 - k);
  return m;
}

// ---------------------------------------------------------------------------
// fine problem (Section 2)
// ---------------------------------------------------------------------------

// gradients of the barycentric coordinates and |det| of one element
static double element_grads(const Hierarchy &h, int64_t e, double G[4][3]) {
  const int d = h.d;
  const int32_t *ev = &h.elems[e * (d + 1)];
  const double *p0 = &h.coords[(int64_t)ev[0] * d];
  double M[3][3];  // columns = edges p_k - p_0
  for (int k = 0; k < d; ++k) {
    const double *pk = &h.coords[(int64_t)ev[k + 1] * d];
    for (int r = 0; r < d; ++r) M[r][k] = pk[r] - p0[r];
  }
  double det, inv[3][3];
  if (d == 2) {
    det = M[0][0] * M[1][1] - M[0][1] * M[1][0];
    inv[0][0] = M[1][1] / det;
    inv[0][1] = -M[0][1] / det;
    inv[1][0] = -M[1][0] / det;
    inv[1][1] = M[0][0] / det;
  } else {
    double c[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        int r0 = (j + 1) % 3, r1 = (j + 2) % 3, c0 = (i + 1) % 3, c1 = (i + 2) % 3;
        c[i][j] = M[r0][c0] * M[r1][c1] - M[r0][c1] * M[r1][c0];  // cofactor (j,i) -> adj(i,j)
      }
    det = M[0][0] * c[0][0] + M[0][1] * c[1][0] + M[0][2] * c[2][0];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) inv[i][j] = c[i][j] / det;
  }
  if (!(det != 0.0) || !std::isfinite(det)) fail(ASMG_EINVAL, "degenerate element " + std::to_string(e));
  for (int k = 0; k < d; ++k)
    for (int r = 0; r < d; ++r) G[k + 1][r] = inv[k][r];
  for (int r = 0; r < d; ++r) {
    double s = 0;
    for (int k = 0; k < d; ++k) s += inv[k][r];
    G[0][r] = -s;
  }
  return std::fabs(det);
}

// CSR pattern from element lists: rows = unknowns; `ev` maps element-local slots to unknowns (-1 = none)
template <class F>
static void pattern_from_elements(int64_t n, int64_t ne, int k, F unknown_of, Csr &A) {
  A.nrows = A.ncols = n;
  std::vector<int64_t> cnt(n + 1, 0);
  std::vector<int64_t> u(k);
  for (int64_t e = 0; e < ne; ++e) {
    for (int i = 0; i < k; ++i) u[i] = unknown_of(e, i);
    for (int i = 0; i < k; ++i)
      if (u[i] >= 0)
        for (int j = 0; j < k; ++j)
          if (u[j] >= 0) cnt[u[i] + 1]++;
  }
  for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
  std::vector<int32_t> tmp(cnt[n]);
  std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
  for (int64_t e = 0; e < ne; ++e) {
    for (int i = 0; i < k; ++i) u[i] = unknown_of(e, i);
    for (int i = 0; i < k; ++i)
      if (u[i] >= 0)
        for (int j = 0; j < k; ++j)
          if (u[j] >= 0) tmp[pos[u[i]]++] = (int32_t)u[j];
  }
  A.rp.assign(n + 1, 0);
  A.ci.clear();
  A.ci.reserve(cnt[n] / 3 + n);
  for (int64_t i = 0; i < n; ++i) {
    auto b = tmp.begin() + cnt[i], e = tmp.begin() + cnt[i + 1];
    std::sort(b, e);
    auto last = std::unique(b, e);
    A.ci.insert(A.ci.end(), b, last);
    A.rp[i + 1] = (int64_t)A.ci.size();
  }
  A.v.assign(A.ci.size(), 0.0);
}

static inline int64_t find_col(const Csr &A, int64_t row, int32_t col) {
  const int32_t *b = A.ci.data() + A.rp[row], *e = A.ci.data() + A.rp[row + 1];
  const int32_t *p = std::lower_bound(b, e, col);
  return (int64_t)(p - A.ci.data());
}

void element_unit_stiffness(const Hierarchy &h, int64_t e, double K[4][4]) {
  const int d = h.d;
  double G[4][3];
  const double vol = element_grads(h, e, G) / (d == 2 ? 2.0 : 6.0);
  for (int i = 0; i <= d; ++i)
    for (int j = 0; j <= d; ++j) {
      double g = 0;
      for (int r = 0; r < d; ++r) g += G[i][r] * G[j][r];
      K[i][j] = vol * g;
    }
}

void fine_dofs(Hierarchy &h) {
  const int d = h.d;
  if (h.dirichlet.empty() && h.opt.domain >= 1) {
    // the mesh's own domain: Dirichlet data on its boundary vertices (edges of one triangle)
    std::vector<std::pair<int64_t, int64_t>> e;
    for (int64_t t = 0; t < h.ne; ++t)
      for (int i = 0; i <= d; ++i)
        for (int j = i + 1; j <= d; ++j) {
          int64_t a = h.elems[t * (d + 1) + i], b = h.elems[t * (d + 1) + j];
          e.push_back({std::min(a, b), std::max(a, b)});
        }
    std::sort(e.begin(), e.end());
    h.dirichlet.assign(h.nv, 0);
    for (size_t i = 0; i < e.size();) {
      size_t j = i;
      while (j < e.size() && e[j] == e[i]) ++j;
      if (j - i == 1) h.dirichlet[e[i].first] = h.dirichlet[e[i].second] = 1;
      i = j;
    }
  }
  if (h.dirichlet.empty()) {
    double lo[3], hi[3];
    for (int k = 0; k < d; ++k) lo[k] = hi[k] = h.coords[k];
    for (int64_t v = 0; v < h.nv; ++v)
      for (int k = 0; k < d; ++k) {
        lo[k] = std::min(lo[k], h.coords[v * d + k]);
        hi[k] = std::max(hi[k], h.coords[v * d + k]);
      }
    h.dirichlet.assign(h.nv, 0);
    for (int64_t v = 0; v < h.nv; ++v)
      for (int k = 0; k < d; ++k) {
        double x = h.coords[v * d + k];
        if (x == lo[k] || x == hi[k]) h.dirichlet[v] = 1;
      }
  }
  h.dof_of_vertex.assign(h.nv, -1);
  h.dofs.clear();
  for (int64_t v = 0; v < h.nv; ++v)
    if (!h.dirichlet[v]) {
      h.dof_of_vertex[v] = (int64_t)h.dofs.size();
      h.dofs.push_back(v);
    }
}

void build_fine(Hierarchy &h) {
  const int d = h.d;
  fine_dofs(h);
  pattern_from_elements(h.n(), h.ne, d + 1,
                        [&](int64_t e, int i) { return h.dof_of_vertex[h.elems[e * (d + 1) + i]]; }, h.A);
  assemble_fine_values(h);
}

void assemble_fine_values(Hierarchy &h) {
  const int d = h.d, k = d + 1;
  std::fill(h.A.v.begin(), h.A.v.end(), 0.0);
  const double fact = d == 2 ? 2.0 : 6.0;
  double G[4][3];
  for (int64_t e = 0; e < h.ne; ++e) {
    const double vol = element_grads(h, e, G) / fact;
    const double w = h.kappa[e] * vol;
    const int32_t *ev = &h.elems[e * k];
    for (int i = 0; i < k; ++i) {
      int64_t ui = h.dof_of_vertex[ev[i]];
      if (ui < 0) continue;
      for (int j = 0; j < k; ++j) {
        int64_t uj = h.dof_of_vertex[ev[j]];
        if (uj < 0) continue;
        double g = 0;
        for (int r = 0; r < d; ++r) g += G[i][r] * G[j][r];
        h.A.v[find_col(h.A, ui, (int32_t)uj)] += w * g;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// cluster tree and closure (Sections 3.1-3.2)
// ---------------------------------------------------------------------------

static void split_clusters(Hierarchy &h, const std::vector<BoxCode> &mc, BoxCode b, int level, int64_t lo,
                           int64_t hi, int n_min) {
  const int d = h.d, D = key_bits(d);
  if (hi - lo <= n_min || level > D) return;
  h.R0.insert(b);
  const int sh = d * (D - level);  // shift of a level-(level+1) code inside a max-level code
  int64_t start = lo;
  for (int ci = 0; ci < (1 << d); ++ci) {
    BoxCode cb = (b << d) | (BoxCode)ci;
    BoxCode upper = (cb + 1) << sh;
    int64_t end = std::lower_bound(mc.begin() + start, mc.begin() + hi, upper) - mc.begin();
    if (end > start) split_clusters(h, mc, cb, level + 1, start, end, n_min);
    start = end;
  }
}

static bool in_tree(const Hierarchy &h, BoxCode b) {
  return box_level(b, h.d) == 1 || h.R.count(b >> h.d);
}

void build_tree(Hierarchy &h) {
  const int d = h.d, D = key_bits(d), k = d + 1;
  const int n_min = h.opt.n_min > 0 ? h.opt.n_min : (d == 2 ? 3 : 7);
  // root box B^1: anchored at the minimum corner, side = largest extent
  double lo[3], hi[3];
  for (int q = 0; q < d; ++q) lo[q] = hi[q] = h.coords[q];
  for (int64_t v = 0; v < h.nv; ++v)
    for (int q = 0; q < d; ++q) {
      lo[q] = std::min(lo[q], h.coords[v * d + q]);
      hi[q] = std::max(hi[q], h.coords[v * d + q]);
    }
  h.L = 0;
  for (int q = 0; q < d; ++q) {
    h.a[q] = lo[q];
    h.L = std::max(h.L, hi[q] - lo[q]);
  }
  if (!(h.L > 0)) fail(ASMG_EINVAL, "mesh has zero extent");
  // barycenters and integer keys
  h.keys.assign(h.ne * d, 0);
  const double scale = std::ldexp(1.0, D);
  const int64_t kmax = ((int64_t)1 << D) - 1;
  std::vector<BoxCode> code(h.ne);
  for (int64_t e = 0; e < h.ne; ++e) {
    const int32_t *ev = &h.elems[e * k];
    int64_t kk[3];
    for (int q = 0; q < d; ++q) {
      volatile double s = h.coords[(int64_t)ev[0] * d + q] + h.coords[(int64_t)ev[1] * d + q];
      for (int m = 2; m < k; ++m) s = s + h.coords[(int64_t)ev[m] * d + q];
      volatile double xi = s / (double)k;
      volatile double t = (xi - h.a[q]) / h.L;
      volatile double ts = t * scale;
      double f = std::floor(ts);
      int64_t ki = f < 0 ? 0 : (int64_t)f;
      if (ki > kmax) ki = kmax;
      kk[q] = ki;
      h.keys[e * d + q] = ki;
    }
    code[e] = box_code(D + 1, kk, d);
  }
  std::vector<int64_t> order(h.ne);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int64_t x, int64_t y) {
    return code[x] < code[y] || (code[x] == code[y] && x < y);
  });
  std::vector<BoxCode> mc(h.ne);
  std::vector<double> ksorted(h.ne);
  for (int64_t i = 0; i < h.ne; ++i) {
    mc[i] = code[order[i]];
    ksorted[i] = h.kappa[order[i]];
  }
  h.R0.clear();
  split_clusters(h, mc, (BoxCode)1, 1, 0, h.ne, n_min);

  // closure: the paper's level-by-level Mark / Close / Refine (Section 3.2)
  std::vector<std::vector<BoxCode>> byLevel(D + 2);
  for (BoxCode b : h.R0) byLevel[box_level(b, d)].push_back(b);
  for (auto &v : byLevel) std::sort(v.begin(), v.end());
  const auto offs = touch_offsets(d);
  h.R.clear();
  for (int lev = 1; lev <= D + 1; ++lev) {
    const std::vector<BoxCode> &marked = byLevel[lev];
    if (marked.empty()) continue;
    std::unordered_set<BoxCode> allm(marked.begin(), marked.end());
    std::vector<BoxCode> newly(marked.begin(), marked.end());
    while (!newly.empty()) {
      std::vector<BoxCode> lst;
      for (BoxCode b : newly) {
        if (box_level(b, d) < 2) continue;
        for (const auto &o : offs) {
          BoxCode q;
          if (!offset_box(b, o, d, &q)) continue;
          BoxCode p = q >> d;
          if (h.R.count(p) || allm.count(p) || !in_tree(h, p)) continue;
          allm.insert(p);
          lst.push_back(p);
        }
      }
      newly.swap(lst);
    }
    h.R.insert(allm.begin(), allm.end());
  }
  // leaves
  h.leaves.clear();
  if (h.R.empty()) {
    h.leaves.push_back((BoxCode)1);
  } else {
    for (BoxCode b : h.R)
      for (int ci = 0; ci < (1 << d); ++ci) {
        BoxCode c = (b << d) | (BoxCode)ci;
        if (!h.R.count(c)) h.leaves.push_back(c);
      }
  }
  // leaves in (level, index tuple) order: one 128-bit key per leaf (level above bit 64, then the
  // index components, each below 2^(64/d))
  {
    std::vector<std::pair<unsigned __int128, BoxCode>> kl(h.leaves.size());
    for (size_t i = 0; i < h.leaves.size(); ++i) {
      const BoxCode b = h.leaves[i];
      int64_t ix[3];
      box_index(b, d, ix);
      const int w = 64 / d;
      unsigned __int128 k = (unsigned __int128)box_level(b, d) << 64;
      for (int q = 0; q < d; ++q) k |= (unsigned __int128)ix[q] << (w * (d - 1 - q));
      kl[i] = {k, b};
    }
    std::sort(kl.begin(), kl.end());
    for (size_t i = 0; i < kl.size(); ++i) h.leaves[i] = kl[i].second;
  }
  h.J = 1;
  for (BoxCode b : h.leaves) h.J = std::max(h.J, box_level(b, d));
  if (h.J > 31 || (d == 3 && h.J > 21)) fail(ASMG_EINVAL, "tree too deep");

  // kappa~ per leaf: mean over the cluster, or over the nearest non-empty ancestor cluster
  h.leaf_kappa.clear();
  for (BoxCode b : h.leaves) {
    BoxCode q = b;
    while (true) {
      int lev = box_level(q, d);
      int sh = d * (D + 1 - lev);
      int64_t s = std::lower_bound(mc.begin(), mc.end(), q << sh) - mc.begin();
      int64_t e = std::lower_bound(mc.begin(), mc.end(), (q + 1) << sh) - mc.begin();
      if (e > s) {
        double sum = 0;
        for (int64_t i = s; i < e; ++i) sum += ksorted[i];
        h.leaf_kappa[b] = sum / (double)(e - s);
        break;
      }
      q >>= d;
    }
  }
}

// mean coefficient of every Kuhn simplex of every box (leaf: kappa~; refined: mean of the
// 2^d child Kuhn simplices inside)
static const int PERM2[2][2] = {{0, 1}, {1, 0}};
static const int PERM3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

static inline int perm_at(int d, int t, int m) { return d == 2 ? PERM2[t][m] : PERM3[t][m]; }

static void compute_kuhn_means(Hierarchy &h) {
  const int d = h.d, nperm = d == 2 ? 2 : 6;
  // child Kuhn simplices inside each parent Kuhn simplex: child position a in {0,1}^d, child simplex s
  std::vector<std::vector<std::pair<int, int>>> inside(nperm);
  for (int t = 0; t < nperm; ++t)
    for (int ci = 0; ci < (1 << d); ++ci) {
      int a[3];
      for (int q = 0; q < d; ++q) a[q] = (ci >> (d - 1 - q)) & 1;
      for (int s = 0; s < nperm; ++s) {
        bool ok = true;
        for (int m = 0; m + 1 < d && ok; ++m) {
          int p = perm_at(d, t, m), q = perm_at(d, t, m + 1);
          if (a[p] > a[q]) continue;
          if (a[p] < a[q]) { ok = false; break; }
          int ip = -1, iq = -1;
          for (int r = 0; r < d; ++r) {
            if (perm_at(d, s, r) == p) ip = r;
            if (perm_at(d, s, r) == q) iq = r;
          }
          if (ip > iq) ok = false;
        }
        if (ok) inside[t].push_back({ci, s});
      }
    }
  h.kuhn_w.clear();
  h.kuhn_w.reserve(h.leaf_kappa.size() + h.R.size());
  for (auto &kv : h.leaf_kappa) {
    KuhnW w{};
    for (int t = 0; t < nperm; ++t) w[t] = kv.second;
    h.kuhn_w.emplace(kv.first, w);
  }
  // finer boxes first (each box's means come from its children's)
  std::vector<std::pair<int, BoxCode>> Rs;
  Rs.reserve(h.R.size());
  for (BoxCode b : h.R) Rs.push_back({box_level(b, d), b});
  std::sort(Rs.begin(), Rs.end(), [](const std::pair<int, BoxCode> &x, const std::pair<int, BoxCode> &y) {
    return x.first > y.first;
  });
  for (const auto &lb : Rs) {
    const BoxCode b = lb.second;
    KuhnW w{};
    for (int t = 0; t < nperm; ++t) {
      double s = 0;
      for (auto &cs : inside[t]) s += h.kuhn_w.at((b << d) | (BoxCode)cs.first)[cs.second];
      w[t] = s / (double)(1 << d);
    }
    h.kuhn_w.emplace(b, w);
  }
}

// ---------------------------------------------------------------------------
// level meshes (Section 3.3)
// ---------------------------------------------------------------------------

struct SimpBuilder {
  int d;
  std::vector<int64_t> pts;  // (d+1)*d per simplex
  std::vector<int32_t> box;
  std::vector<int8_t> tmpl;
  void add(const int64_t *v, int nvtx, int32_t b, int t) {
    pts.insert(pts.end(), v, v + nvtx * d);
    box.push_back(b);
    tmpl.push_back((int8_t)t);
  }
};

static void kuhn_simplices(int d, const int64_t *c, int64_t S, int32_t bi, SimpBuilder &sb) {
  const int nperm = d == 2 ? 2 : 6;
  for (int t = 0; t < nperm; ++t) {
    int64_t v[4][3];
    for (int q = 0; q < d; ++q) v[0][q] = c[q];
    for (int m = 0; m < d - 1; ++m) {
      for (int q = 0; q < d; ++q) v[m + 1][q] = v[m][q];
      v[m + 1][perm_at(d, t, m)] += S;
    }
    for (int q = 0; q < d; ++q) v[d][q] = c[q] + S;
    int64_t flat[12];
    for (int m = 0; m <= d; ++m)
      for (int q = 0; q < d; ++q) flat[m * d + q] = v[m][q];
    sb.add(flat, d + 1, bi, t);
  }
}

static bool neighbour_refined(const Hierarchy &h, BoxCode b, int ox, int oy, int oz) {
  BoxCode nb;
  std::array<int, 3> o{ox, oy, oz};
  if (!offset_box(b, o, h.d, &nb)) return false;
  return h.R.count(nb) > 0;
}

static void fan2(const Hierarchy &h, BoxCode b, const int64_t *c, int64_t S, int32_t bi, SimpBuilder &sb) {
  const int64_t H = S / 2;
  int64_t LL[2] = {c[0], c[1]}, LR[2] = {c[0] + S, c[1]}, UR[2] = {c[0] + S, c[1] + S}, UL[2] = {c[0], c[1] + S};
  int64_t C[2] = {c[0] + H, c[1] + H};
  const int64_t *E[4][2] = {{LL, LR}, {LR, UR}, {UR, UL}, {UL, LL}};
  const int O[4][2] = {{0, -1}, {1, 0}, {0, 1}, {-1, 0}};
  int t = 0;
  for (int e = 0; e < 4; ++e) {
    const int64_t *v0 = E[e][0], *v1 = E[e][1];
    if (neighbour_refined(h, b, O[e][0], O[e][1], 0)) {
      int64_t m[2] = {(v0[0] + v1[0]) / 2, (v0[1] + v1[1]) / 2};
      int64_t t1[6] = {v0[0], v0[1], m[0], m[1], C[0], C[1]};
      int64_t t2[6] = {m[0], m[1], v1[0], v1[1], C[0], C[1]};
      sb.add(t1, 3, bi, t++);
      sb.add(t2, 3, bi, t++);
    } else {
      int64_t t1[6] = {v0[0], v0[1], v1[0], v1[1], C[0], C[1]};
      sb.add(t1, 3, bi, t++);
    }
  }
}

static void fan3(const Hierarchy &h, BoxCode b, const int64_t *c, int64_t S, int32_t bi, SimpBuilder &sb) {
  const int64_t H = S / 2;
  int64_t C[3] = {c[0] + H, c[1] + H, c[2] + H};
  int t = 0;
  for (int ax = 0; ax < 3; ++ax) {
    int u = ax == 0 ? 1 : 0, v = ax == 2 ? 1 : 2;
    for (int s = 0; s < 2; ++s) {
      int of[3] = {0, 0, 0};
      of[ax] = 2 * s - 1;
      int64_t base[3] = {c[0], c[1], c[2]};
      base[ax] += s * S;
      auto P = [&](int al2, int be2, int64_t *out) {
        for (int q = 0; q < 3; ++q) out[q] = base[q];
        out[u] += al2 * H;
        out[v] += be2 * H;
      };
      auto inR = [&](const int *o) { return neighbour_refined(h, b, o[0], o[1], o[2]); };
      // face edges counter-clockwise in (u, v): bottom, right, top, left (half-units)
      const int ea[4][4] = {{0, 0, 2, 0}, {2, 0, 2, 2}, {2, 2, 0, 2}, {0, 2, 0, 0}};
      int ip[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
      ip[0][v] = -1;
      ip[1][u] = 1;
      ip[2][v] = 1;
      ip[3][u] = -1;
      bool mid[4], anymid = false;
      for (int e = 0; e < 4; ++e) {
        int both[3] = {of[0] + ip[e][0], of[1] + ip[e][1], of[2] + ip[e][2]};
        mid[e] = inR(of) || inR(ip[e]) || inR(both);
        anymid = anymid || mid[e];
      }
      std::vector<std::array<int64_t, 9>> tris;
      auto push = [&](const int64_t *p, const int64_t *q, const int64_t *r) {
        std::array<int64_t, 9> a{p[0], p[1], p[2], q[0], q[1], q[2], r[0], r[1], r[2]};
        tris.push_back(a);
      };
      if (inR(of)) {
        for (int be0 = 0; be0 < 2; ++be0)
          for (int al0 = 0; al0 < 2; ++al0) {
            int64_t p00[3], p10[3], p11[3], p01[3];
            P(al0, be0, p00);
            P(al0 + 1, be0, p10);
            P(al0 + 1, be0 + 1, p11);
            P(al0, be0 + 1, p01);
            push(p00, p10, p11);
            push(p00, p01, p11);
          }
      } else if (anymid) {
        int64_t FC[3];
        P(1, 1, FC);
        for (int e = 0; e < 4; ++e) {
          int64_t p0[3], p1[3];
          P(ea[e][0], ea[e][1], p0);
          P(ea[e][2], ea[e][3], p1);
          if (mid[e]) {
            int64_t pm[3] = {(p0[0] + p1[0]) / 2, (p0[1] + p1[1]) / 2, (p0[2] + p1[2]) / 2};
            push(p0, pm, FC);
            push(pm, p1, FC);
          } else {
            push(p0, p1, FC);
          }
        }
      } else {
        int64_t p00[3], p20[3], p22[3], p02[3];
        P(0, 0, p00);
        P(2, 0, p20);
        P(2, 2, p22);
        P(0, 2, p02);
        push(p00, p20, p22);
        push(p00, p02, p22);
      }
      for (auto &tr : tris) {
        int64_t flat[12];
        for (int q = 0; q < 9; ++q) flat[q] = tr[q];
        for (int q = 0; q < 3; ++q) flat[9 + q] = C[q];
        sb.add(flat, 4, bi, t++);
      }
    }
  }
}

static bool is_fan(const Hierarchy &h, BoxCode b, int level) {
  if (box_level(b, h.d) >= level) return false;
  static thread_local std::vector<std::array<int, 3>> offs2 = touch_offsets(2), offs3 = touch_offsets(3);
  const auto &offs = h.d == 2 ? offs2 : offs3;
  for (const auto &o : offs) {
    BoxCode nb;
    if (offset_box(b, o, h.d, &nb) && h.R.count(nb)) return true;
  }
  return false;
}

static LevelMesh make_level_mesh(const Hierarchy &h, int level) {
  const int d = h.d, J = h.J;
  LevelMesh lm;
  lm.level = level;
  // active boxes: tree boxes of this level, leaves of coarser levels
  std::vector<BoxCode> act;
  for (BoxCode b : h.leaves)
    if (box_level(b, d) < level) act.push_back(b);
  if (level == 1) {
    act.push_back((BoxCode)1);
  } else {
    for (BoxCode b : h.R)
      if (box_level(b, d) == level - 1)
        for (int ci = 0; ci < (1 << d); ++ci) act.push_back((b << d) | (BoxCode)ci);
  }
  std::vector<std::pair<unsigned __int128, BoxCode>> keyed(act.size());
  for (size_t i = 0; i < act.size(); ++i) {
    int64_t idx[3], cor[3];
    box_index(act[i], d, idx);
    const int sh = J - box_level(act[i], d) + 1;
    for (int q = 0; q < d; ++q) cor[q] = idx[q] << sh;
    keyed[i] = {morton_point(cor, d, J + 1), act[i]};
  }
  std::sort(keyed.begin(), keyed.end());
  lm.boxes.resize(act.size());
  lm.fan.resize(act.size());
  SimpBuilder sb{d, {}, {}, {}};
  for (size_t i = 0; i < keyed.size(); ++i) {
    BoxCode b = keyed[i].second;
    lm.boxes[i] = b;
    lm.box_index[b] = (int32_t)i;
    int64_t idx[3], cor[3];
    box_index(b, d, idx);
    const int64_t S = (int64_t)1 << (J - box_level(b, d) + 1);
    for (int q = 0; q < d; ++q) cor[q] = idx[q] * S;
    bool f = is_fan(h, b, level);
    lm.fan[i] = f;
    if (!f)
      kuhn_simplices(d, cor, S, (int32_t)i, sb);
    else if (d == 2)
      fan2(h, b, cor, S, (int32_t)i, sb);
    else
      fan3(h, b, cor, S, (int32_t)i, sb);
  }
  const int64_t ns = (int64_t)sb.box.size(), nvtx = ns * (d + 1);
  // vertex numbering: rank of the vertex's Morton key among the distinct keys
  lm.simp.resize(nvtx);
  int64_t nv = 0;
  if ((J + 1) * d <= 64) {
    // keys of at most 64 bits: LSD radix sort of (key, position), 11 bits per pass
    std::vector<uint64_t> key(nvtx), k2(nvtx);
    std::vector<int64_t> pos(nvtx), p2(nvtx);
    for (int64_t i = 0; i < nvtx; ++i) {
      key[i] = morton_point64(&sb.pts[i * d], d);
      pos[i] = i;
    }
    std::vector<int64_t> cnt(2048);
    for (int sh = 0; sh < (J + 1) * d; sh += 11) {
      std::fill(cnt.begin(), cnt.end(), 0);
      for (int64_t i = 0; i < nvtx; ++i) cnt[(key[i] >> sh) & 2047]++;
      int64_t run = 0;
      for (int64_t &c : cnt) {
        const int64_t t = c;
        c = run;
        run += t;
      }
      for (int64_t i = 0; i < nvtx; ++i) {
        const int64_t o = cnt[(key[i] >> sh) & 2047]++;
        k2[o] = key[i];
        p2[o] = pos[i];
      }
      key.swap(k2);
      pos.swap(p2);
    }
    std::vector<int64_t> first;  // position of one vertex with each key
    for (int64_t j = 0; j < nvtx; ++j) {
      if (j == 0 || key[j] != key[j - 1]) first.push_back(pos[j]);
      lm.simp[pos[j]] = (int64_t)first.size() - 1;
    }
    nv = (int64_t)first.size();
    lm.verts.assign(nv * d, 0);
    for (int64_t r = 0; r < nv; ++r)
      for (int q = 0; q < d; ++q) lm.verts[r * d + q] = sb.pts[first[r] * d + q];
  } else {
    std::vector<unsigned __int128> vk(nvtx);
    for (int64_t i = 0; i < nvtx; ++i) vk[i] = morton_point(&sb.pts[i * d], d, J + 1);
    std::vector<unsigned __int128> uk(vk);
    std::sort(uk.begin(), uk.end());
    uk.erase(std::unique(uk.begin(), uk.end()), uk.end());
    nv = (int64_t)uk.size();
    lm.verts.assign(nv * d, 0);
    for (int64_t i = 0; i < nvtx; ++i) {
      int64_t r = std::lower_bound(uk.begin(), uk.end(), vk[i]) - uk.begin();
      lm.simp[i] = r;
      for (int q = 0; q < d; ++q) lm.verts[r * d + q] = sb.pts[i * d + q];
    }
  }
  lm.simp_box = std::move(sb.box);
  lm.simp_tmpl = std::move(sb.tmpl);
  lm.box_simp.assign(lm.boxes.size() + 1, 0);
  for (int64_t s = 0; s < ns; ++s) lm.box_simp[lm.simp_box[s] + 1]++;
  for (size_t i = 0; i < lm.boxes.size(); ++i) lm.box_simp[i + 1] += lm.box_simp[i];
  const int64_t top = (int64_t)1 << J;
  // general domain (Section 3.4): keep the simplices inside the domain; an unknown needs its
  // whole star kept
  std::vector<uint8_t> outside(nv, 0);
  const bool mixed = h.domain && h.opt.domain == 2;
  std::vector<uint8_t> inkept;  // mixed grids: vertex of a kept simplex
  if (mixed) {
    // mixed Dirichlet/Neumann grids: every vertex of a kept simplex is an unknown (natural
    // conditions, on the root box too) except the vertices of simplices meeting Gamma_D
    std::vector<uint8_t> touch;
    domain_mixed(h, lm, lm.kept, touch);
    inkept.assign(nv, 0);
    for (int64_t s = 0; s < ns; ++s)
      for (int i = 0; i <= d; ++i) {
        if (lm.kept[s]) inkept[lm.simp[s * (d + 1) + i]] = 1;
        if (touch[s]) outside[lm.simp[s * (d + 1) + i]] = 1;
      }
  } else if (h.domain) {
    lm.kept = domain_keeps(h, lm);
    for (int64_t s = 0; s < ns; ++s)
      if (!lm.kept[s])
        for (int i = 0; i <= d; ++i) outside[lm.simp[s * (d + 1) + i]] = 1;
  }
  lm.dof_of_vert.assign(nv, -1);
  for (int64_t v = 0; v < nv; ++v) {
    bool in = !outside[v];
    if (mixed) {
      in = in && inkept[v];
    } else {
      for (int q = 0; q < d; ++q) {
        int64_t x = lm.verts[v * d + q];
        in = in && x > 0 && x < top;
      }
    }
    if (in) {
      lm.dof_of_vert[v] = (int64_t)lm.dof_vert.size();
      lm.dof_vert.push_back(v);
    }
  }
  return lm;
}

const LevelMesh &level_mesh(Hierarchy &h, int level) {
  auto it = h.meshes.find(level);
  if (it != h.meshes.end()) return it->second;
  return h.meshes.emplace(level, make_level_mesh(h, level)).first->second;
}

// ---------------------------------------------------------------------------
// auxiliary operators (Section 4.1)
// ---------------------------------------------------------------------------

static int64_t idet(int d, const int64_t E[3][3]) {
  if (d == 2) return E[0][0] * E[1][1] - E[0][1] * E[1][0];
  return E[0][0] * (E[1][1] * E[2][2] - E[1][2] * E[2][1]) - E[0][1] * (E[1][0] * E[2][2] - E[1][2] * E[2][0]) +
         E[0][2] * (E[1][0] * E[2][1] - E[1][1] * E[2][0]);
}

// integer cofactor vectors a_0..a_d of a simplex in units of half its box side
static int64_t aux_cofactors(const Hierarchy &h, const LevelMesh &lm, int64_t s, int64_t a[4][3], int64_t *half) {
  const int d = h.d;
  BoxCode b = lm.boxes[lm.simp_box[s]];
  *half = (int64_t)1 << (h.J - box_level(b, d));
  const int64_t *v0 = &lm.verts[lm.simp[s * (d + 1)] * d];
  int64_t M[3][3];  // M[r][k] = component r of edge k
  for (int k = 0; k < d; ++k) {
    const int64_t *vk = &lm.verts[lm.simp[s * (d + 1) + k + 1] * d];
    for (int r = 0; r < d; ++r) M[r][k] = (vk[r] - v0[r]) / *half;
  }
  const int64_t det = idet(d, M);
  // rows of adj(M): a_{k+1}
  if (d == 2) {
    a[1][0] = M[1][1];
    a[1][1] = -M[0][1];
    a[2][0] = -M[1][0];
    a[2][1] = M[0][0];
  } else {
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        int r0 = (j + 1) % 3, r1 = (j + 2) % 3, c0 = (i + 1) % 3, c1 = (i + 2) % 3;
        a[i + 1][j] = M[r0][c0] * M[r1][c1] - M[r0][c1] * M[r1][c0];
      }
  }
  for (int r = 0; r < d; ++r) {
    int64_t sum = 0;
    for (int k = 1; k <= d; ++k) sum += a[k][r];
    a[0][r] = -sum;
  }
  return det;
}

static void assemble_level(Hierarchy &h, int level, Csr &A, bool pattern) {
  const int d = h.d, k = d + 1;
  const LevelMesh &lm = h.meshes.at(level);
  const int64_t ns = (int64_t)lm.simp_box.size();
  // the grid is the kept simplices (all of sigma^(l) unless a general domain drops some)
  auto in_grid = [&](int64_t s) { return lm.kept.empty() || lm.kept[s]; };
  if (pattern)
    pattern_from_elements(lm.n(), ns, k, [&](int64_t s, int i) {
      return in_grid(s) ? lm.dof_of_vert[lm.simp[s * k + i]] : (int64_t)-1;
    }, A);
  else
    std::fill(A.v.begin(), A.v.end(), 0.0);
  const double fact = d == 2 ? 2.0 : 6.0;
  const double unit = std::ldexp(h.L, -h.J);
  for (int64_t s = 0; s < ns; ++s) {
    if (!in_grid(s)) continue;
    int64_t a[4][3], half;
    const int64_t det = aux_cofactors(h, lm, s, a, &half);
    const double denom = fact * (double)std::llabs(det);
    BoxCode b = lm.boxes[lm.simp_box[s]];
    const KuhnW &w = h.kuhn_w.at(b);
    const double kap = lm.fan[lm.simp_box[s]] ? w[0] : w[lm.simp_tmpl[s]];
    for (int i = 0; i < k; ++i) {
      int64_t ui = lm.dof_of_vert[lm.simp[s * k + i]];
      if (ui < 0) continue;
      for (int j = 0; j < k; ++j) {
        int64_t uj = lm.dof_of_vert[lm.simp[s * k + j]];
        if (uj < 0) continue;
        int64_t dot = 0;
        for (int r = 0; r < d; ++r) dot += a[i][r] * a[j][r];
        double val = (double)dot / denom;
        if (d == 3) val = val * ((double)half * unit);
        val = val * kap;
        A.v[find_col(A, ui, (int32_t)uj)] += val;
      }
    }
  }
  if (pattern) {
    // drop couplings that are exactly zero (right angles): the pattern is geometric
    Csr B;
    B.nrows = A.nrows;
    B.ncols = A.ncols;
    B.rp.assign(A.nrows + 1, 0);
    for (int64_t i = 0; i < A.nrows; ++i) {
      for (int64_t p = A.rp[i]; p < A.rp[i + 1]; ++p)
        if (A.v[p] != 0.0 || A.ci[p] == i) {
          B.ci.push_back(A.ci[p]);
          B.v.push_back(A.v[p]);
        }
      B.rp[i + 1] = (int64_t)B.ci.size();
    }
    A = std::move(B);
  }
}

// exact barycentric coordinates of integer point X in simplex s; false if outside
static bool bary_exact(const LevelMesh &lm, int d, int64_t s, const int64_t *X, double *lam) {
  const int64_t *V[4];
  for (int m = 0; m <= d; ++m) V[m] = &lm.verts[lm.simp[s * (d + 1) + m] * d];
  auto det = [&](const int64_t *P[4]) -> __int128 {
    __int128 E[3][3];
    for (int k = 0; k < d; ++k)
      for (int r = 0; r < d; ++r) E[r][k] = (__int128)(P[k + 1][r] - P[0][r]);
    if (d == 2) return E[0][0] * E[1][1] - E[0][1] * E[1][0];
    return E[0][0] * (E[1][1] * E[2][2] - E[1][2] * E[2][1]) - E[0][1] * (E[1][0] * E[2][2] - E[1][2] * E[2][0]) +
           E[0][2] * (E[1][0] * E[2][1] - E[1][1] * E[2][0]);
  };
  __int128 tot = det(V);
  __int128 num[4];
  for (int m = 0; m <= d; ++m) {
    const int64_t *Q[4];
    for (int r = 0; r <= d; ++r) Q[r] = r == m ? X : V[r];
    num[m] = det(Q);
    if (tot < 0) num[m] = -num[m];
    if (num[m] < 0) return false;
  }
  if (tot < 0) tot = -tot;
  for (int m = 0; m <= d; ++m) lam[m] = (double)num[m] / (double)tot;
  return true;
}

static void build_prolongation(Hierarchy &h, int level, Csr &P) {
  const int d = h.d, J = h.J;
  const LevelMesh &fine = h.meshes.at(level);
  const LevelMesh &coarse = h.meshes.at(level - 1);
  P.nrows = fine.n();
  P.ncols = coarse.n();
  P.rp.assign(P.nrows + 1, 0);
  P.ci.clear();
  P.v.clear();
  std::vector<std::pair<int32_t, double>> row;
  for (int64_t i = 0; i < fine.n(); ++i) {
    const int64_t *X = &fine.verts[fine.dof_vert[i] * d];
    int32_t bi = -1;
    for (int k = 1; k <= level - 1 && bi < 0; ++k) {
      int64_t idx[3];
      const int sh = J - k + 1;
      const int64_t nmax = ((int64_t)1 << (k - 1)) - 1;
      for (int q = 0; q < d; ++q) idx[q] = std::min(X[q] >> sh, nmax);
      auto it = coarse.box_index.find(box_code(k, idx, d));
      if (it != coarse.box_index.end()) bi = it->second;
    }
    if (bi < 0) fail(ASMG_EINVAL, "prolongation: point location failed");
    double lam[4];
    int64_t sfound = -1;
    for (int64_t s = coarse.box_simp[bi]; s < coarse.box_simp[bi + 1]; ++s)
      if (bary_exact(coarse, d, s, X, lam)) {
        sfound = s;
        break;
      }
    if (sfound < 0) fail(ASMG_EINVAL, "prolongation: no containing simplex");
    row.clear();
    for (int m = 0; m <= d; ++m) {
      if (lam[m] == 0.0) continue;
      int64_t j = coarse.dof_of_vert[coarse.simp[sfound * (d + 1) + m]];
      if (j < 0) continue;
      row.push_back({(int32_t)j, lam[m]});
    }
    std::sort(row.begin(), row.end());
    for (auto &e : row) {
      if (!P.ci.empty() && (int64_t)P.ci.size() > P.rp[i] && P.ci.back() == e.first) {
        P.v.back() += e.second;
      } else {
        P.ci.push_back(e.first);
        P.v.push_back(e.second);
      }
    }
    P.rp[i + 1] = (int64_t)P.ci.size();
  }
}

void compute_level_means(Hierarchy &h) { compute_kuhn_means(h); }

void build_level_meshes(Hierarchy &h) {
  compute_kuhn_means(h);
  const int J = h.J;
  const int Nc = h.opt.coarse_max_dofs > 0 ? h.opt.coarse_max_dofs : 1024;
  h.level_n.assign(J, -1);
  // level sizes shrink going down; build meshes from J downwards in parallel batches until one
  // has at most Nc unknowns
  h.lc = 1;
  int l = J;
  bool found = false;
  while (!found && l >= 1) {
    const int nb = std::min(l, std::max(1, h.threads > 0 ? h.threads : (int)std::thread::hardware_concurrency()));
    std::vector<LevelMesh> got(nb);
    parallel_for(h, nb, [&](int64_t i) {
      if (!h.meshes.count(l - (int)i)) got[i] = make_level_mesh(h, l - (int)i);
    });
    for (int i = 0; i < nb; ++i) {
      const int li = l - i;
      if (!h.meshes.count(li)) h.meshes.emplace(li, std::move(got[i]));
      h.level_n[li - 1] = h.meshes.at(li).n();
    }
    for (int i = 0; i < nb; ++i) {
      const int li = l - i;
      if (h.level_n[li - 1] <= Nc) {
        h.lc = li;
        found = true;
        break;
      }
    }
    l -= nb;
  }
  // meshes below the bottom are not needed
  for (auto it = h.meshes.begin(); it != h.meshes.end();)
    it = it->first < h.lc ? h.meshes.erase(it) : std::next(it);
  for (int li = 1; li < h.lc; ++li) h.level_n[li - 1] = -1;
}

void build_level_operators(Hierarchy &h, bool assemble, bool prolong) {
  const int J = h.J;
  if (assemble) {
    h.Al.clear();
    for (int li = J; li >= h.lc; --li) h.Al[li];
    parallel_for(h, J - h.lc + 1, [&](int64_t i) { assemble_level(h, J - (int)i, h.Al.at(J - (int)i), true); });
  }
  if (!prolong) return;
  h.P.clear();
  for (int li = J; li > h.lc; --li) h.P[li];
  parallel_for(h, J - h.lc, [&](int64_t i) { build_prolongation(h, J - (int)i, h.P.at(J - (int)i)); });
}

void build_levels(Hierarchy &h) {
  build_level_meshes(h);
  build_level_operators(h, true);
}

void assemble_aux_values(Hierarchy &h) {
  h.leaf_kappa.clear();
  // recompute kappa~ from the sorted clusters: rebuilt by build_tree's logic on the new kappa
  const int d = h.d, D = key_bits(d);
  std::vector<BoxCode> code(h.ne);
  for (int64_t e = 0; e < h.ne; ++e) code[e] = box_code(D + 1, &h.keys[e * d], d);
  std::vector<int64_t> order(h.ne);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int64_t x, int64_t y) {
    return code[x] < code[y] || (code[x] == code[y] && x < y);
  });
  std::vector<BoxCode> mc(h.ne);
  for (int64_t i = 0; i < h.ne; ++i) mc[i] = code[order[i]];
  for (BoxCode b : h.leaves) {
    BoxCode q = b;
    while (true) {
      int lev = box_level(q, d);
      int sh = d * (D + 1 - lev);
      int64_t s = std::lower_bound(mc.begin(), mc.end(), q << sh) - mc.begin();
      int64_t e = std::lower_bound(mc.begin(), mc.end(), (q + 1) << sh) - mc.begin();
      if (e > s) {
        double sum = 0;
        for (int64_t i = s; i < e; ++i) sum += h.kappa[order[i]];
        h.leaf_kappa[b] = sum / (double)(e - s);
        break;
      }
      q >>= d;
    }
  }
  compute_kuhn_means(h);
  parallel_for(h, h.J - h.lc + 1, [&](int64_t i) { assemble_level(h, h.J - (int)i, h.Al.at(h.J - (int)i), false); });
}

// ---------------------------------------------------------------------------
// Scott-Zhang transfer (Section 4.1)
// ---------------------------------------------------------------------------

static void collect_leaves(const Hierarchy &h, BoxCode b, const double *lo, const double *hi,
                           std::vector<BoxCode> &out) {
  const int d = h.d;
  int64_t idx[3];
  box_index(b, d, idx);
  const int lev = box_level(b, d);
  const double side = std::ldexp(h.L, -(lev - 1));
  for (int q = 0; q < d; ++q) {
    double b0 = h.a[q] + (double)idx[q] * side, b1 = h.a[q] + (double)(idx[q] + 1) * side;
    if (b0 > hi[q] || b1 < lo[q]) return;
  }
  if (!h.R.count(b)) {
    out.push_back(b);
    return;
  }
  for (int ci = 0; ci < (1 << d); ++ci) collect_leaves(h, (b << d) | (BoxCode)ci, lo, hi, out);
}

static inline double det3(const double *u, const double *v, const double *w) {
  return u[0] * (v[1] * w[2] - v[2] * w[1]) - u[1] * (v[0] * w[2] - v[2] * w[0]) + u[2] * (v[0] * w[1] - v[1] * w[0]);
}

void build_transfer(Hierarchy &h) {
  const int d = h.d, k = d + 1;
  const LevelMesh &lm = level_mesh(h, h.J);
  const double unit = std::ldexp(h.L, -h.J);
  const int64_t n = h.n();
  // sigma_i: 2-D the edge to the smallest-id neighbour, 3-D the lexicographically smallest face
  std::vector<int64_t> sj(h.nv, INT64_MAX), sk(h.nv, INT64_MAX);
  for (int64_t e = 0; e < h.ne; ++e) {
    const int32_t *ev = &h.elems[e * k];
    for (int a = 0; a < k; ++a) {
      int64_t v = ev[a];
      if (d == 2) {
        for (int b = 0; b < k; ++b)
          if (b != a) sj[v] = std::min<int64_t>(sj[v], ev[b]);
      } else {
        int o[3], c = 0;
        for (int b = 0; b < 4; ++b)
          if (b != a) o[c++] = ev[b];
        for (int x = 0; x < 3; ++x)
          for (int y = x + 1; y < 3; ++y) {
            int64_t j = std::min(o[x], o[y]), kk = std::max(o[x], o[y]);
            if (j < sj[v] || (j == sj[v] && kk < sk[v])) {
              sj[v] = j;
              sk[v] = kk;
            }
          }
      }
    }
  }
  Csr &Pi = h.Pi;
  Pi.nrows = n;
  Pi.ncols = lm.n();
  // A piece of sigma_i lying in the facet of simplex s opposite its vertex m is met by the two
  // simplices sharing that facet and counts 1/2 from each; a facet on the boundary of the root
  // box belongs to one simplex and counts fully.
  const int64_t top = (int64_t)1 << h.J;
  auto facet_weight = [&](int64_t s, int m) {
    for (int q = 0; q < d; ++q) {
      bool lo_all = true, hi_all = true;
      for (int a = 0; a < k; ++a) {
        if (a == m) continue;
        const int64_t x = lm.verts[lm.simp[s * k + a] * d + q];
        lo_all = lo_all && x == 0;
        hi_all = hi_all && x == top;
      }
      if (lo_all || hi_all) return 1.0;
    }
    return 0.5;
  };
  // rows in chunks on parallel threads, concatenated in order
  const int64_t CH = 4096;
  const int64_t nch = (n + CH - 1) / CH;
  std::vector<std::vector<int32_t>> cci(nch);
  std::vector<std::vector<double>> cv(nch);
  std::vector<std::vector<int64_t>> crl(nch);
  parallel_for(h, nch, [&](int64_t ch) {
  std::vector<BoxCode> lv;
  std::vector<std::pair<int32_t, double>> acc;
  std::vector<int32_t> &oci = cci[ch];
  std::vector<double> &ov = cv[ch];
  std::vector<int64_t> &orl = crl[ch];
  for (int64_t i = ch * CH; i < std::min(n, (ch + 1) * CH); ++i) {
    const int64_t vi = h.dofs[i];
    double P[3][3];
    int64_t sv[3] = {vi, sj[vi], sk[vi]};
    for (int m = 0; m < d; ++m)
      for (int q = 0; q < d; ++q) P[m][q] = h.coords[sv[m] * d + q];
    double lo[3], hi[3];
    for (int q = 0; q < d; ++q) {
      lo[q] = hi[q] = P[0][q];
      for (int m = 1; m < d; ++m) {
        lo[q] = std::min(lo[q], P[m][q]);
        hi[q] = std::max(hi[q], P[m][q]);
      }
    }
    lv.clear();
    collect_leaves(h, (BoxCode)1, lo, hi, lv);
    acc.clear();
    for (BoxCode b : lv) {
      auto it = lm.box_index.find(b);
      if (it == lm.box_index.end()) continue;
      const int32_t bi = it->second;
      for (int64_t s = lm.box_simp[bi]; s < lm.box_simp[bi + 1]; ++s) {
        double T[4][3];
        int64_t cols[4];
        for (int m = 0; m < k; ++m) {
          int64_t vv = lm.simp[s * k + m];
          cols[m] = lm.dof_of_vert[vv];
          for (int q = 0; q < d; ++q) T[m][q] = h.a[q] + (double)lm.verts[vv * d + q] * unit;
        }
        if (d == 2) {
          // barycentric coordinates of the segment ends; lambda_m(t) affine in t
          auto cross = [](double ux, double uy, double vx, double vy) { return ux * vy - uy * vx; };
          const double a2 = cross(T[1][0] - T[0][0], T[1][1] - T[0][1], T[2][0] - T[0][0], T[2][1] - T[0][1]);
          double l0[3], l1[3];
          for (int e = 0; e < 2; ++e) {
            const double x = P[e][0], y = P[e][1];
            double *l = e == 0 ? l0 : l1;
            l[0] = cross(T[1][0] - x, T[1][1] - y, T[2][0] - x, T[2][1] - y) / a2;
            l[1] = cross(T[2][0] - x, T[2][1] - y, T[0][0] - x, T[0][1] - y) / a2;
            l[2] = cross(T[0][0] - x, T[0][1] - y, T[1][0] - x, T[1][1] - y) / a2;
          }
          double t0 = 0.0, t1 = 1.0;
          bool empty = false;
          int on_facet = -1;
          for (int m = 0; m < 3; ++m) {
            const double sl = l1[m] - l0[m];
            if (l0[m] == 0.0 && l1[m] == 0.0 && on_facet < 0) on_facet = m;
            if (sl == 0.0) {
              if (l0[m] < 0.0) empty = true;
              continue;
            }
            const double tc = -l0[m] / sl;
            if (sl > 0)
              t0 = std::max(t0, tc);
            else
              t1 = std::min(t1, tc);
          }
          if (empty || !(t1 > t0)) continue;
          const double wgt = on_facet >= 0 ? facet_weight(s, on_facet) : 1.0, tm = 0.5 * (t0 + t1);
          for (int m = 0; m < 3; ++m) {
            if (cols[m] < 0) continue;
            auto f = [&](double t) { return (4.0 - 6.0 * t) * (l0[m] + t * (l1[m] - l0[m])); };
            const double val = (t1 - t0) / 6.0 * (f(t0) + 4.0 * f(tm) + f(t1)) * wgt;
            if (val != 0.0) acc.push_back({(int32_t)cols[m], val});
          }
        } else {
          // barycentric coordinates of the face corners; clip the reference triangle in (s, t)
          double c[4][3];
          double e1[3], e2[3], e3[3];
          for (int q = 0; q < 3; ++q) {
            e1[q] = T[1][q] - T[0][q];
            e2[q] = T[2][q] - T[0][q];
            e3[q] = T[3][q] - T[0][q];
          }
          const double vol = det3(e1, e2, e3);
          for (int corner = 0; corner < 3; ++corner) {
            const double *x = P[corner];
            for (int m = 0; m < 4; ++m) {
              double Q[4][3];
              for (int r = 0; r < 4; ++r)
                for (int q = 0; q < 3; ++q) Q[r][q] = r == m ? x[q] : T[r][q];
              double f1[3], f2[3], f3[3];
              for (int q = 0; q < 3; ++q) {
                f1[q] = Q[1][q] - Q[0][q];
                f2[q] = Q[2][q] - Q[0][q];
                f3[q] = Q[3][q] - Q[0][q];
              }
              c[m][corner] = det3(f1, f2, f3) / vol;
            }
          }
          std::vector<std::array<double, 2>> poly{{0.0, 0.0}, {1.0, 0.0}, {0.0, 1.0}}, out;
          int on_facet = -1;
          for (int m = 0; m < 4 && poly.size() >= 3; ++m) {
            const double c0 = c[m][0], c1 = c[m][1], c2 = c[m][2];
            if (c0 == 0.0 && c1 == 0.0 && c2 == 0.0 && on_facet < 0) on_facet = m;
            auto f = [&](const std::array<double, 2> &p) { return c0 + p[0] * (c1 - c0) + p[1] * (c2 - c0); };
            out.clear();
            const size_t np = poly.size();
            for (size_t q = 0; q < np; ++q) {
              const auto &A_ = poly[q];
              const auto &B_ = poly[(q + 1) % np];
              const double fa = f(A_), fb = f(B_);
              if (fa >= 0) out.push_back(A_);
              if ((fa > 0 && fb < 0) || (fa < 0 && fb > 0)) {
                const double t = fa / (fa - fb);
                out.push_back({A_[0] + t * (B_[0] - A_[0]), A_[1] + t * (B_[1] - A_[1])});
              }
            }
            poly.swap(out);
          }
          if (poly.size() < 3) continue;
          const double wgt = on_facet >= 0 ? facet_weight(s, on_facet) : 1.0;
          for (int m = 0; m < 4; ++m) {
            if (cols[m] < 0) continue;
            const double c0 = c[m][0], c1 = c[m][1], c2 = c[m][2];
            auto f = [&](double s_, double t_) {
              return (18.0 - 24.0 * (s_ + t_)) * (c0 + s_ * (c1 - c0) + t_ * (c2 - c0));
            };
            double val = 0.0;
            for (size_t q = 1; q + 1 < poly.size(); ++q) {
              const auto &A_ = poly[0], &B_ = poly[q], &C_ = poly[q + 1];
              const double area =
                  0.5 * std::fabs((B_[0] - A_[0]) * (C_[1] - A_[1]) - (B_[1] - A_[1]) * (C_[0] - A_[0]));
              if (area == 0.0) continue;
              val += area *
                     (f(0.5 * (A_[0] + B_[0]), 0.5 * (A_[1] + B_[1])) + f(0.5 * (B_[0] + C_[0]), 0.5 * (B_[1] + C_[1])) +
                      f(0.5 * (C_[0] + A_[0]), 0.5 * (C_[1] + A_[1]))) /
                     3.0;
            }
            val *= wgt;
            if (val != 0.0) acc.push_back({(int32_t)cols[m], val});
          }
        }
      }
    }
    // by column, equal columns in the order they were met (summed in that order below)
    std::stable_sort(acc.begin(), acc.end(), [](const std::pair<int32_t, double> &x,
                                                const std::pair<int32_t, double> &y) { return x.first < y.first; });
    const size_t before = oci.size();
    for (size_t q = 0; q < acc.size(); ++q) {
      if (q > 0 && acc[q].first == acc[q - 1].first)
        ov.back() += acc[q].second;
      else {
        oci.push_back(acc[q].first);
        ov.push_back(acc[q].second);
      }
    }
    orl.push_back((int64_t)(oci.size() - before));
  }
  });
  Pi.rp.assign(n + 1, 0);
  Pi.ci.clear();
  Pi.v.clear();
  int64_t row = 0;
  for (int64_t ch = 0; ch < nch; ++ch) {
    Pi.ci.insert(Pi.ci.end(), cci[ch].begin(), cci[ch].end());
    Pi.v.insert(Pi.v.end(), cv[ch].begin(), cv[ch].end());
    for (int64_t len : crl[ch]) {
      Pi.rp[row + 1] = Pi.rp[row] + len;
      ++row;
    }
  }
}

// ---------------------------------------------------------------------------
// multicolour ordering
// ---------------------------------------------------------------------------

static inline uint32_t fmix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x85ebca6bu;
  x ^= x >> 13;
  x *= 0xc2b2ae35u;
  x ^= x >> 16;
  return x;
}

// Smallest-last order (Matula and Beck): repeatedly remove the remaining row of smallest
// (degree among the remaining rows, row index); colour in the reverse removal order. The
// lazy-deletion heap pops exactly that minimum, so the order is unique.
static std::vector<int64_t> smallest_last_order(const Csr &A) {
  const int64_t n = A.nrows;
  std::vector<int32_t> deg(n, 0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t p = A.rp[i]; p < A.rp[i + 1]; ++p) deg[i] += A.ci[p] != i;
  using Item = std::pair<int32_t, int64_t>;
  std::vector<Item> init(n);
  for (int64_t i = 0; i < n; ++i) init[i] = {deg[i], i};
  std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap(std::greater<Item>(), std::move(init));
  std::vector<uint8_t> removed(n, 0);
  std::vector<int64_t> order;
  order.reserve(n);
  while (!heap.empty()) {
    const Item it = heap.top();
    heap.pop();
    const int64_t i = it.second;
    if (removed[i] || it.first != deg[i]) continue;
    removed[i] = 1;
    order.push_back(i);
    for (int64_t p = A.rp[i]; p < A.rp[i + 1]; ++p) {
      const int64_t j = A.ci[p];
      if (j == i || removed[j]) continue;
      heap.push({--deg[j], j});
    }
  }
  std::reverse(order.begin(), order.end());
  return order;
}

// greedy colouring (each row takes the smallest colour unused by its coloured neighbours) in
// ascending index (mode 0), descending (fmix32(i ^ seed), i) (mode 1) or smallest-last order (mode 2)
static std::vector<int32_t> greedy_colouring(const Csr &A, uint32_t seed, int mode) {
  const int64_t n = A.nrows;
  std::vector<int64_t> order(n);
  std::iota(order.begin(), order.end(), 0);
  if (mode == 2) order = smallest_last_order(A);
  if (mode == 1) {
    std::vector<uint32_t> w(n);
    for (int64_t i = 0; i < n; ++i) w[i] = fmix32((uint32_t)i ^ seed);
    std::sort(order.begin(), order.end(), [&](int64_t x, int64_t y) {
      return w[x] > w[y] || (w[x] == w[y] && x > y);
    });
  }
  std::vector<int32_t> col(n, -1);
  std::vector<int64_t> mark(64, -1);
  for (int64_t i : order) {
    for (int64_t p = A.rp[i]; p < A.rp[i + 1]; ++p) {
      int32_t c = col[A.ci[p]];
      if (c >= 0) {
        if (c >= (int32_t)mark.size()) mark.resize(c + 1, -1);
        mark[c] = i;
      }
    }
    int32_t c = 0;
    while (c < (int32_t)mark.size() && mark[c] == i) ++c;
    col[i] = c;
  }
  return col;
}

void build_colourings(Hierarchy &h) {
  // one matrix per task: the original grid and the smoothed auxiliary levels
  std::vector<int> lv{0};
  for (int l = h.lc + 1; l <= h.J; ++l) lv.push_back(l);
  std::vector<std::vector<int32_t>> out(lv.size());
  parallel_for(h, (int64_t)lv.size(), [&](int64_t t) {
    const Csr &A = lv[t] == 0 ? h.A : h.Al.at(lv[t]);
    out[t] = greedy_colouring(A, h.opt.colour_seed, h.opt.colouring);
  });
  h.colour_fine = std::move(out[0]);
  h.colour_aux.clear();
  for (size_t t = 1; t < lv.size(); ++t) h.colour_aux[lv[t]] = std::move(out[t]);
}

// N~_l (Section 4.3): unknowns of level l that are new, or whose nodal basis function changed
// from level l-1. In the level-l basis phi_{k,l-1} = sum_i P[i,k] phi_{i,l}; an unknown that
// already existed has the single entry 1 in its row of P_l, and its function is unchanged
// exactly when that entry is alone in its column.
void build_local_sets(Hierarchy &h) {
  h.local_set.clear();
  for (int l = h.lc + 1; l <= h.J; ++l) {
    const Csr &P = h.P.at(l);
    std::vector<int32_t> colcount(P.ncols, 0);
    for (int32_t c : P.ci) ++colcount[c];
    std::vector<uint8_t> m(P.nrows, 1);
    for (int64_t i = 0; i < P.nrows; ++i) {
      const bool old = P.rp[i + 1] - P.rp[i] == 1 && P.v[P.rp[i]] == 1.0;
      if (old) m[i] = colcount[P.ci[P.rp[i]]] > 1;
    }
    h.local_set[l] = std::move(m);
  }
}

// ---------------------------------------------------------------------------
// bottom of the V-cycle: Cholesky factor A_lc = L L^T and the explicit inverse
// ---------------------------------------------------------------------------

void build_coarse(Hierarchy &h) {
  const Csr &A = h.Al.at(h.lc);
  const int64_t n = A.nrows;
  h.nc = n;
  h.coarse_inv.assign(n * n, 0.0);
  if (n == 0) return;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t p = A.rp[i]; p < A.rp[i + 1]; ++p) h.coarse_inv[i * n + A.ci[p]] = A.v[p];
  // Cholesky factor and explicit inverse; a singular component (a pure Neumann problem: rows
  // summing to zero) is regularised by its rank-one term first
  spd_inverse(h.coarse_inv, n, h.threads, true);
}

// ---------------------------------------------------------------------------
// Morton rank of every unknown of the original grid: its position when the unknowns are sorted
// by the Morton code of their vertex (quantised in the root box of the cluster tree, ties by id)
std::vector<int> morton_rank(const Hierarchy &h) {
  const int64_t n = h.n();
  const int d = h.d;
  const int bits = d == 2 ? 31 : 21;
  const double scale = std::ldexp(1.0, bits);
  std::vector<std::pair<uint64_t, int64_t>> key(n);
  for (int64_t i = 0; i < n; ++i) {
    const double *x = &h.coords[h.dofs[i] * d];
    uint64_t q[3] = {0, 0, 0};
    for (int k = 0; k < d; ++k) {
      double t = (x[k] - h.a[k]) / h.L * scale;
      t = std::min(std::max(t, 0.0), scale - 1.0);
      q[k] = (uint64_t)t;
    }
    uint64_t m = 0;
    for (int b = bits - 1; b >= 0; --b)
      for (int k = 0; k < d; ++k) m = (m << 1) | ((q[k] >> b) & 1u);
    key[i] = {m, i};
  }
  std::sort(key.begin(), key.end());
  std::vector<int> rank(n);
  for (int64_t k = 0; k < n; ++k) rank[key[k].second] = (int)k;
  return rank;
}

}  // namespace asmg
