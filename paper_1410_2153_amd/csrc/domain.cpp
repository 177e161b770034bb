// Dirichlet auxiliary grids on a general 2-D polygonal domain (Section 3.4).
//
// Section 3.4 keeps on level l the simplices of sigma^(l) that lie in the domain. The domain is
// the closed union of the mesh's triangles. An auxiliary vertex with integer coordinate X on the
// finest box grid sits at the double a_k + L * (X_k * 2^-J) (round to nearest, the product
// first; this file is compiled without contraction). A simplex is kept iff no boundary edge of
// the mesh (an edge of one triangle) meets its open interior and its interior point
// (2 v0 + v1 + v2) / 4 lies in a closed mesh triangle: with no boundary edge inside, the
// connected interior lies entirely in the domain or entirely outside its closure. A closed
// segment and an open triangle are disjoint iff the line of one edge of the triangle, or the
// segment's own line, separates them weakly (separating axes of two convex polygons).
//
// Every decision is a sign of an orientation determinant of doubles, evaluated exactly with
// floating-point expansions (Shewchuk, "Adaptive precision floating-point arithmetic and fast
// robust geometric predicates", 1997): a filtered double evaluation, and an exact expansion
// when the filter cannot decide.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "setup.hpp"

namespace asmg {

namespace {

// ---- exact orientation ------------------------------------------------------------------

inline void two_sum(double a, double b, double &x, double &y) {
  x = a + b;
  const double bv = x - a, av = x - bv;
  y = (a - av) + (b - bv);
}

inline void two_diff(double a, double b, double &x, double &y) {
  x = a - b;
  const double bv = a - x, av = x + bv;
  y = (a - av) + (bv - b);
}

inline void split(double a, double &hi, double &lo) {
  const double c = 134217729.0 * a;  // 2^27 + 1
  const double abig = c - a;
  hi = c - abig;
  lo = a - hi;
}

inline void two_product(double a, double b, double &x, double &y) {
  x = a * b;
  double ahi, alo, bhi, blo;
  split(a, ahi, alo);
  split(b, bhi, blo);
  const double e1 = x - ahi * bhi, e2 = e1 - alo * bhi, e3 = e2 - ahi * blo;
  y = alo * blo - e3;
}

// h = e * b for a nonoverlapping expansion e (increasing magnitude); zero components dropped
int scale_expansion(int elen, const double *e, double b, double *h) {
  double bhi, blo;
  split(b, bhi, blo);
  int hi = 0;
  double q, hh;
  auto prod = [&](double a, double &x, double &y) {
    x = a * b;
    double ahi, alo;
    split(a, ahi, alo);
    const double e1 = x - ahi * bhi, e2 = e1 - alo * bhi, e3 = e2 - ahi * blo;
    y = alo * blo - e3;
  };
  prod(e[0], q, hh);
  if (hh != 0) h[hi++] = hh;
  for (int i = 1; i < elen; ++i) {
    double p1, p0, sum;
    prod(e[i], p1, p0);
    two_sum(q, p0, sum, hh);
    if (hh != 0) h[hi++] = hh;
    two_sum(p1, sum, q, hh);
    if (hh != 0) h[hi++] = hh;
  }
  if (q != 0 || hi == 0) h[hi++] = q;
  return hi;
}

// h = e + f for nonoverlapping expansions (increasing magnitude); zero components dropped
int expansion_sum(int elen, const double *e, int flen, const double *f, double *h) {
  // merge by magnitude, then accumulate with two_sum (linear expansion sum)
  std::vector<double> g(elen + flen);
  int i = 0, j = 0, k = 0;
  while (i < elen && j < flen) g[k++] = (std::fabs(e[i]) < std::fabs(f[j])) ? e[i++] : f[j++];
  while (i < elen) g[k++] = e[i++];
  while (j < flen) g[k++] = f[j++];
  int hi = 0;
  double q = g[0];
  for (int m = 1; m < k; ++m) {
    double sum, hh;
    two_sum(q, g[m], sum, hh);
    if (hh != 0) h[hi++] = hh;
    q = sum;
  }
  if (q != 0 || hi == 0) h[hi++] = q;
  return hi;
}

// sign of (b - a) x (c - a), exact for double inputs
int orient2d(const double *a, const double *b, const double *c) {
  const double detl = (a[0] - c[0]) * (b[1] - c[1]);
  const double detr = (a[1] - c[1]) * (b[0] - c[0]);
  const double det = detl - detr;
  const double sum = std::fabs(detl) + std::fabs(detr);
  const double eps = std::ldexp(1.0, -53);
  if (std::fabs(det) > (3.0 + 16.0 * eps) * eps * sum) return (det > 0) - (det < 0);
  // exact: (acx)(bcy) - (acy)(bcx) with every difference a two-term expansion
  double acx[2], acy[2], bcx[2], bcy[2];
  two_diff(a[0], c[0], acx[1], acx[0]);
  two_diff(a[1], c[1], acy[1], acy[0]);
  two_diff(b[0], c[0], bcx[1], bcx[0]);
  two_diff(b[1], c[1], bcy[1], bcy[0]);
  double t1[4], t2[4], L[8], r1[4], r2[4], R[8], D[16];
  int n1 = scale_expansion(2, acx, bcy[0], t1), n2 = scale_expansion(2, acx, bcy[1], t2);
  const int nl = expansion_sum(n1, t1, n2, t2, L);
  n1 = scale_expansion(2, acy, -bcx[0], r1);
  n2 = scale_expansion(2, acy, -bcx[1], r2);
  const int nr = expansion_sum(n1, r1, n2, r2, R);
  const int nd = expansion_sum(nl, L, nr, R, D);
  for (int i = nd - 1; i >= 0; --i)
    if (D[i] != 0) return D[i] > 0 ? 1 : -1;
  return 0;
}

// ---- the domain ---------------------------------------------------------------------------

struct Grid {  // uniform bucket grid over the root box: items listed per cell
  int g = 1;
  double a0 = 0, a1 = 0, L = 1;
  std::vector<int64_t> start;
  std::vector<int64_t> items;
  int cell(double x, int k) const {
    const double t = (x - (k ? a1 : a0)) / L * g;
    return std::min(g - 1, std::max(0, (int)std::floor(t)));
  }
};

}  // namespace

struct DomainIndex {
  std::vector<int64_t> bedge;   // boundary edges, 2 vertex ids each
  std::vector<double> ebox;     // lo_x, lo_y, hi_x, hi_y per boundary edge
  std::vector<double> tbox;     // per triangle
  std::vector<int64_t> gedge;   // Gamma_D: boundary edges with both vertices Dirichlet
  std::vector<double> gbox;
  Grid eg, tg, gg;
};

namespace {

Grid make_grid(const Hierarchy &h, const std::vector<double> &box, int64_t n) {
  Grid G;
  G.a0 = h.a[0];
  G.a1 = h.a[1];
  G.L = h.L;
  G.g = std::max(1, std::min(4096, (int)std::sqrt((double)std::max<int64_t>(n, 1))));
  std::vector<int64_t> cnt((size_t)G.g * G.g + 1, 0);
  auto cells = [&](int64_t i, auto &&f) {
    const int x0 = G.cell(box[i * 4 + 0], 0), x1 = G.cell(box[i * 4 + 2], 0);
    const int y0 = G.cell(box[i * 4 + 1], 1), y1 = G.cell(box[i * 4 + 3], 1);
    for (int y = y0; y <= y1; ++y)
      for (int x = x0; x <= x1; ++x) f((int64_t)y * G.g + x);
  };
  for (int64_t i = 0; i < n; ++i) cells(i, [&](int64_t c) { ++cnt[c + 1]; });
  for (size_t c = 0; c + 1 < cnt.size(); ++c) cnt[c + 1] += cnt[c];
  G.items.resize(cnt.back());
  std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
  for (int64_t i = 0; i < n; ++i) cells(i, [&](int64_t c) { G.items[pos[c]++] = i; });
  G.start = std::move(cnt);
  return G;
}

template <class F>
void query(const Grid &G, const double *lo, const double *hi, std::vector<int64_t> &seen, int64_t stamp, F &&f) {
  const int x0 = G.cell(lo[0], 0), x1 = G.cell(hi[0], 0), y0 = G.cell(lo[1], 1), y1 = G.cell(hi[1], 1);
  for (int y = y0; y <= y1; ++y)
    for (int x = x0; x <= x1; ++x) {
      const int64_t c = (int64_t)y * G.g + x;
      for (int64_t p = G.start[c]; p < G.start[c + 1]; ++p) {
        const int64_t i = G.items[p];
        if (seen[i] == stamp) continue;
        seen[i] = stamp;
        if (!f(i)) return;
      }
    }
}

inline bool boxes_meet(const double *b, const double *lo, const double *hi) {
  return b[0] <= hi[0] && lo[0] <= b[2] && b[1] <= hi[1] && lo[1] <= b[3];
}

// does the closed segment pq meet the open triangle T (3 points)?
bool segment_meets_open(const double *p, const double *q, const double T[3][2]) {
  for (int i = 0; i < 3; ++i) {
    const double *a = T[i], *b = T[(i + 1) % 3], *c = T[(i + 2) % 3];
    const int side = orient2d(a, b, c);
    if (orient2d(a, b, p) * side <= 0 && orient2d(a, b, q) * side <= 0) return false;
  }
  const int o0 = orient2d(p, q, T[0]), o1 = orient2d(p, q, T[1]), o2 = orient2d(p, q, T[2]);
  if ((o0 >= 0 && o1 >= 0 && o2 >= 0) || (o0 <= 0 && o1 <= 0 && o2 <= 0)) return false;
  return true;
}

// does the closed segment pq meet the closed triangle T? (disjoint iff an edge line of T has both
// ends strictly outside, or the segment's line has the three vertices strictly on one side)
bool segment_meets_closed(const double *p, const double *q, const double T[3][2]) {
  for (int i = 0; i < 3; ++i) {
    const double *a = T[i], *b = T[(i + 1) % 3], *c = T[(i + 2) % 3];
    const int side = orient2d(a, b, c);
    if (orient2d(a, b, p) * side < 0 && orient2d(a, b, q) * side < 0) return false;
  }
  const int o0 = orient2d(p, q, T[0]), o1 = orient2d(p, q, T[1]), o2 = orient2d(p, q, T[2]);
  if ((o0 > 0 && o1 > 0 && o2 > 0) || (o0 < 0 && o1 < 0 && o2 < 0)) return false;
  return true;
}

void aux_point(const Hierarchy &h, const int64_t *X, int extra_bits, double *x) {
  const double s = std::ldexp(1.0, -(h.J + extra_bits));
  for (int k = 0; k < 2; ++k) x[k] = h.a[k] + h.L * ((double)X[k] * s);
}

}  // namespace

void build_domain(Hierarchy &h) {
  if (h.d != 2) throw AsmgError{ASMG_EINVAL, "general domains are 2-D"};
  auto D = std::make_shared<DomainIndex>();
  // boundary edges: edges of exactly one triangle
  std::vector<std::pair<int64_t, int64_t>> e;
  e.reserve(h.ne * 3);
  for (int64_t t = 0; t < h.ne; ++t)
    for (int i = 0; i < 3; ++i) {
      int64_t a = h.elems[t * 3 + i], b = h.elems[t * 3 + (i + 1) % 3];
      if (a > b) std::swap(a, b);
      e.push_back({a, b});
    }
  std::sort(e.begin(), e.end());
  for (size_t i = 0; i < e.size();) {
    size_t j = i;
    while (j < e.size() && e[j] == e[i]) ++j;
    if (j - i == 1) {
      D->bedge.push_back(e[i].first);
      D->bedge.push_back(e[i].second);
    }
    i = j;
  }
  const int64_t nb = (int64_t)D->bedge.size() / 2;
  D->ebox.resize(nb * 4);
  for (int64_t i = 0; i < nb; ++i) {
    const double *p = &h.coords[D->bedge[2 * i] * 2], *q = &h.coords[D->bedge[2 * i + 1] * 2];
    D->ebox[i * 4 + 0] = std::min(p[0], q[0]);
    D->ebox[i * 4 + 1] = std::min(p[1], q[1]);
    D->ebox[i * 4 + 2] = std::max(p[0], q[0]);
    D->ebox[i * 4 + 3] = std::max(p[1], q[1]);
  }
  D->tbox.resize(h.ne * 4);
  for (int64_t t = 0; t < h.ne; ++t) {
    double lo[2] = {INFINITY, INFINITY}, hi[2] = {-INFINITY, -INFINITY};
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 2; ++k) {
        const double x = h.coords[h.elems[t * 3 + i] * 2 + k];
        lo[k] = std::min(lo[k], x);
        hi[k] = std::max(hi[k], x);
      }
    D->tbox[t * 4 + 0] = lo[0];
    D->tbox[t * 4 + 1] = lo[1];
    D->tbox[t * 4 + 2] = hi[0];
    D->tbox[t * 4 + 3] = hi[1];
  }
  D->eg = make_grid(h, D->ebox, nb);
  D->tg = make_grid(h, D->tbox, h.ne);
  if (!h.dirichlet.empty())
    for (int64_t i = 0; i < nb; ++i)
      if (h.dirichlet[D->bedge[2 * i]] && h.dirichlet[D->bedge[2 * i + 1]]) {
        D->gedge.push_back(D->bedge[2 * i]);
        D->gedge.push_back(D->bedge[2 * i + 1]);
        for (int k = 0; k < 4; ++k) D->gbox.push_back(D->ebox[i * 4 + k]);
      }
  D->gg = make_grid(h, D->gbox, (int64_t)D->gedge.size() / 2);
  h.domain = D;
}

namespace {

bool contains_point(const Hierarchy &h, const DomainIndex &D, const double *x, std::vector<int64_t> &seen,
                    int64_t &stamp) {
  bool found = false;
  ++stamp;
  query(D.tg, x, x, seen, stamp, [&](int64_t t) {
    if (!boxes_meet(&D.tbox[t * 4], x, x)) return true;
    const double *a = &h.coords[h.elems[t * 3] * 2], *b = &h.coords[h.elems[t * 3 + 1] * 2],
                 *c = &h.coords[h.elems[t * 3 + 2] * 2];
    const int s = orient2d(a, b, c);
    if (orient2d(a, b, x) * s >= 0 && orient2d(b, c, x) * s >= 0 && orient2d(c, a, x) * s >= 0) {
      found = true;
      return false;
    }
    return true;
  });
  return found;
}

}  // namespace

// mixed grids (2-D): kept = the closed simplex meets the domain and not Gamma_D; touch = it
// meets Gamma_D. A closed simplex that no boundary edge meets lies entirely inside or entirely
// outside the domain, and its interior point (2 v0 + v1 + v2) / 4 decides which.
void domain_mixed(const Hierarchy &h, const LevelMesh &lm, std::vector<uint8_t> &kept,
                  std::vector<uint8_t> &touch) {
  const DomainIndex &D = *h.domain;
  const int64_t ns = (int64_t)lm.simp_box.size();
  kept.assign(ns, 0);
  touch.assign(ns, 0);
  std::vector<int64_t> seen_e(D.ebox.size() / 4, -1), seen_g(D.gbox.size() / 4, -1), seen_t(h.ne, -1);
  int64_t stamp_e = 0, stamp_g = 0, stamp_t = 0;
  std::vector<int64_t> cand, gcand;
  const int J = h.J;
  for (size_t bi = 0; bi < lm.boxes.size(); ++bi) {
    int64_t idx[3];
    box_index(lm.boxes[bi], 2, idx);
    const int64_t S = (int64_t)1 << (J - box_level(lm.boxes[bi], 2) + 1);
    const int64_t c0[2] = {idx[0] * S, idx[1] * S}, c1[2] = {idx[0] * S + S, idx[1] * S + S};
    double lo[2], hi[2];
    aux_point(h, c0, 0, lo);
    aux_point(h, c1, 0, hi);
    cand.clear();
    gcand.clear();
    ++stamp_e;
    query(D.eg, lo, hi, seen_e, stamp_e, [&](int64_t i) {
      if (boxes_meet(&D.ebox[i * 4], lo, hi)) cand.push_back(i);
      return true;
    });
    if (!D.gedge.empty()) {
      ++stamp_g;
      query(D.gg, lo, hi, seen_g, stamp_g, [&](int64_t i) {
        if (boxes_meet(&D.gbox[i * 4], lo, hi)) gcand.push_back(i);
        return true;
      });
    }
    for (int64_t s = lm.box_simp[bi]; s < lm.box_simp[bi + 1]; ++s) {
      const int64_t *v = &lm.simp[s * 3];
      double T[3][2];
      for (int i = 0; i < 3; ++i) aux_point(h, &lm.verts[v[i] * 2], 0, T[i]);
      bool gd = false;
      for (int64_t i : gcand)
        if (segment_meets_closed(&h.coords[D.gedge[2 * i] * 2], &h.coords[D.gedge[2 * i + 1] * 2], T)) {
          gd = true;
          break;
        }
      if (gd) {
        touch[s] = 1;
        continue;
      }
      bool meets = false;
      for (int64_t i : cand)
        if (segment_meets_closed(&h.coords[D.bedge[2 * i] * 2], &h.coords[D.bedge[2 * i + 1] * 2], T)) {
          meets = true;
          break;
        }
      if (meets) {
        kept[s] = 1;
        continue;
      }
      if (cand.empty() && s > lm.box_simp[bi]) {
        // no boundary edge meets the closed box: every simplex of the box is on the same side
        kept[s] = kept[lm.box_simp[bi]];
        continue;
      }
      int64_t inner[2];
      for (int k = 0; k < 2; ++k)
        inner[k] = 2 * lm.verts[v[0] * 2 + k] + lm.verts[v[1] * 2 + k] + lm.verts[v[2] * 2 + k];
      double x[2];
      aux_point(h, inner, 2, x);
      kept[s] = contains_point(h, D, x, seen_t, stamp_t) ? 1 : 0;
    }
  }
}

// kept flag of every simplex of a level mesh (2-D)
std::vector<uint8_t> domain_keeps(const Hierarchy &h, const LevelMesh &lm) {
  const DomainIndex &D = *h.domain;
  const int64_t ns = (int64_t)lm.simp_box.size();
  std::vector<uint8_t> kept(ns, 0);
  std::vector<int64_t> seen_e(D.ebox.size() / 4, -1), seen_t(h.ne, -1);
  int64_t stamp_e = 0, stamp_t = 0;
  std::vector<int64_t> cand;
  const int J = h.J;
  for (size_t bi = 0; bi < lm.boxes.size(); ++bi) {
    int64_t idx[3];
    box_index(lm.boxes[bi], 2, idx);
    const int64_t S = (int64_t)1 << (J - box_level(lm.boxes[bi], 2) + 1);
    const int64_t c0[2] = {idx[0] * S, idx[1] * S}, c1[2] = {idx[0] * S + S, idx[1] * S + S};
    double lo[2], hi[2];
    aux_point(h, c0, 0, lo);
    aux_point(h, c1, 0, hi);
    cand.clear();
    ++stamp_e;
    query(D.eg, lo, hi, seen_e, stamp_e, [&](int64_t i) {
      if (boxes_meet(&D.ebox[i * 4], lo, hi)) cand.push_back(i);
      return true;
    });
    for (int64_t s = lm.box_simp[bi]; s < lm.box_simp[bi + 1]; ++s) {
      const int64_t *v = &lm.simp[s * 3];
      double T[3][2];
      for (int i = 0; i < 3; ++i) aux_point(h, &lm.verts[v[i] * 2], 0, T[i]);
      bool meets = false;
      for (int64_t i : cand) {
        const double *p = &h.coords[D.bedge[2 * i] * 2], *q = &h.coords[D.bedge[2 * i + 1] * 2];
        if (segment_meets_open(p, q, T)) {
          meets = true;
          break;
        }
      }
      if (meets) continue;
      if (cand.empty() && s > lm.box_simp[bi]) {
        // no boundary edge meets the closed box: every simplex of the box is on the same side
        kept[s] = kept[lm.box_simp[bi]];
        continue;
      }
      int64_t inner[2];
      for (int k = 0; k < 2; ++k)
        inner[k] = 2 * lm.verts[v[0] * 2 + k] + lm.verts[v[1] * 2 + k] + lm.verts[v[2] * 2 + k];
      double x[2];
      aux_point(h, inner, 2, x);
      kept[s] = contains_point(h, D, x, seen_t, stamp_t) ? 1 : 0;
    }
  }
  return kept;
}

}  // namespace asmg
