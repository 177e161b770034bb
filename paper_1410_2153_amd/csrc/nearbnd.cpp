// Near-boundary correction of the auxiliary V-cycle (Section 3.5, Algorithm 3): the sets
// J_{l,j} and exact solvers for A_l restricted to them; and the regularised dense inverse that
// the singular subsystems of a pure Neumann problem need (also used for the bottom level).
//
// J_{l,j}: Gamma_l is the boundary of the union of the level's kept simplices (the facets that
// belong to one kept simplex). The grids are conforming, so a closed simplex is at distance 0
// from a set exactly when it shares a vertex with it: V_0 = the vertices on Gamma_l,
// T_(l,i) = the kept simplices with a vertex in V_i, V_(i+1) = the vertices of T_(l,i), and
// J_{l,j} = the unknowns among V_(j+1).
//
// Exact solve of A_JJ x = r:
//   * |J| <= kNbDenseMax: the explicit inverse (regularised where singular);
//   * larger sets (strips along the boundary): one level of domain decomposition. Recursive
//     coordinate bisection cuts J into pieces of at most kNbPiece unknowns; an unknown with a
//     neighbour in a piece of lower index joins the separator S, which decouples the pieces'
//     interiors I_p. With the dense inverses of A_{I_p I_p} and of the Schur complement
//     S = A_SS - sum_p A_{S I_p} A_{I_p I_p}^-1 A_{I_p S}, the solve is
//       y_I = A_II^-1 r_I,  x_S = S^-1 (r_S - A_SI y_I),  x_I = y_I - A_II^-1 A_IS x_S,
//     exact up to rounding. A set that contains a whole singular component of the level
//     (pure Neumann problems, small coarse levels) takes the dense path.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <string>
#include <vector>

#include "host_parallel.hpp"
#include "setup.hpp"

namespace asmg {

static constexpr int64_t kNbDenseMax = 2048;  // dense inverse up to this many unknowns
static constexpr int64_t kNbPiece = 256;      // unknowns per piece of the decomposition
static constexpr int64_t kNbSchurMax = 6144;  // largest separator (dense Schur inverse)

// Components of the symmetric matrix M (n x n, row-major) whose rows sum to zero get
// gamma_c 1_c 1_c^T added, gamma_c = mean(diag M_cc) / |c|: the result is SPD and acts as the
// pseudo-inverse on vectors with zero sum over each such component.
static void regularise(std::vector<double> &M, int64_t n) {
  std::vector<int64_t> comp(n, -1), stack;
  int64_t nc = 0;
  for (int64_t s = 0; s < n; ++s) {
    if (comp[s] >= 0) continue;
    comp[s] = nc;
    stack.assign(1, s);
    while (!stack.empty()) {
      const int64_t i = stack.back();
      stack.pop_back();
      for (int64_t j = 0; j < n; ++j)
        if (j != i && comp[j] < 0 && M[i * n + j] != 0.0) {
          comp[j] = nc;
          stack.push_back(j);
        }
    }
    ++nc;
  }
  std::vector<std::vector<int64_t>> members(nc);
  for (int64_t i = 0; i < n; ++i) members[comp[i]].push_back(i);
  for (const auto &idx : members) {
    double scale = 0.0, rmax = 0.0, dsum = 0.0;
    for (int64_t i : idx) {
      double rs = 0.0;
      for (int64_t j = 0; j < n; ++j) rs += M[i * n + j];
      scale = std::max(scale, std::fabs(M[i * n + i]));
      rmax = std::max(rmax, std::fabs(rs));
      dsum += M[i * n + i];
    }
    if (rmax <= 1e-10 * scale) {
      const double gamma = dsum / (double)idx.size() / (double)idx.size();
      for (int64_t i : idx)
        for (int64_t j : idx) M[i * n + j] += gamma;
    }
  }
}

// sum_k a[k] b[k] over k < n in four interleaved partial sums (independent chains that the
// compiler can keep in vector registers), combined in a fixed order
static inline double dot4(const double *a, const double *b, int64_t n) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int64_t k = 0;
  for (; k + 4 <= n; k += 4) {
    s0 += a[k] * b[k];
    s1 += a[k + 1] * b[k + 1];
    s2 += a[k + 2] * b[k + 2];
    s3 += a[k + 3] * b[k + 3];
  }
  for (; k < n; ++k) s0 += a[k] * b[k];
  return (s0 + s1) + (s2 + s3);
}

void spd_inverse(std::vector<double> &M, int64_t n, int threads, bool regularised) {
  if (n == 0) return;
  if (regularised) regularise(M, n);
  std::vector<double> Lm(n * n, 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j <= i; ++j) Lm[i * n + j] = M[i * n + j];
  // Cholesky, row by row of L: the entries left of the diagonal are dot products of rows
  for (int64_t j = 0; j < n; ++j) {
    const double *lj = &Lm[j * n];
    const double s = Lm[j * n + j] - dot4(lj, lj, j);
    if (!(s > 0)) throw AsmgError{ASMG_ENOTSPD, "matrix of an exact subsystem solve is not positive definite"};
    const double djj = std::sqrt(s);
    Lm[j * n + j] = djj;
    for (int64_t i = j + 1; i < n; ++i) Lm[i * n + j] = (Lm[i * n + j] - dot4(&Lm[i * n], lj, j)) / djj;
  }
  // inverse column by column (independent columns on host threads): L y = e_c, L^T x = y;
  // y_i = 0 for i < c, and the backward solve reads L^T by rows
  std::vector<double> Ut(n * n);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = 0; k < n; ++k) Ut[i * n + k] = Lm[k * n + i];
  host_parallel(threads, (int)std::min<int64_t>(n, 1 << 30), [&](int cc) {
    const int64_t c = cc;
    std::vector<double> y(n, 0.0), x(n);
    for (int64_t i = c; i < n; ++i)
      y[i] = ((i == c ? 1.0 : 0.0) - dot4(&Lm[i * n + c], &y[c], i - c)) / Lm[i * n + i];
    for (int64_t i = n - 1; i >= 0; --i) x[i] = (y[i] - dot4(&Ut[i * n + i + 1], &x[i + 1], n - 1 - i)) / Lm[i * n + i];
    for (int64_t i = 0; i < n; ++i) M[i * n + c] = x[i];
  });
}

std::vector<int64_t> near_boundary_set(Hierarchy &h, int level, int layers) {
  const LevelMesh &lm = level_mesh(h, level);
  const int d = h.d, k = d + 1;
  const int64_t ns = (int64_t)lm.simp_box.size(), nv = (int64_t)lm.verts.size() / d;
  auto kept = [&](int64_t s) { return lm.kept.empty() || lm.kept[s] != 0; };
  // facets of kept simplices, sorted; those that occur once form Gamma_l
  std::vector<std::array<int64_t, 3>> f;
  for (int64_t s = 0; s < ns; ++s) {
    if (!kept(s)) continue;
    for (int skip = 0; skip < k; ++skip) {
      std::array<int64_t, 3> t{-1, -1, -1};
      int c = 0;
      for (int a = 0; a < k; ++a)
        if (a != skip) t[c++] = lm.simp[s * k + a];
      std::sort(t.begin(), t.begin() + d);
      f.push_back(t);
    }
  }
  std::sort(f.begin(), f.end());
  std::vector<uint8_t> V(nv, 0);
  for (size_t i = 0; i < f.size();) {
    size_t e = i + 1;
    while (e < f.size() && f[e] == f[i]) ++e;
    if (e - i == 1)
      for (int a = 0; a < d; ++a) V[f[i][a]] = 1;
    i = e;
  }
  for (int round = 0; round <= layers; ++round) {
    std::vector<uint8_t> Vn(nv, 0);
    for (int64_t s = 0; s < ns; ++s) {
      if (!kept(s)) continue;
      bool hit = false;
      for (int a = 0; a < k && !hit; ++a) hit = V[lm.simp[s * k + a]] != 0;
      if (hit)
        for (int a = 0; a < k; ++a) Vn[lm.simp[s * k + a]] = 1;
    }
    V.swap(Vn);
  }
  std::vector<int64_t> J;
  for (int64_t v = 0; v < nv; ++v)
    if (V[v] && lm.dof_of_vert[v] >= 0) J.push_back(lm.dof_of_vert[v]);
  std::sort(J.begin(), J.end());
  return J;
}

// recursive coordinate bisection of the positions `idx` (into J) into pieces of at most kNbPiece
static void bisect(const std::vector<std::array<int64_t, 3>> &X, int d, std::vector<int64_t> idx,
                   std::vector<std::vector<int64_t>> &pieces) {
  if ((int64_t)idx.size() <= kNbPiece) {
    std::sort(idx.begin(), idx.end());
    pieces.push_back(idx);
    return;
  }
  int ax = 0;
  int64_t best = -1;
  for (int q = 0; q < d; ++q) {
    int64_t lo = INT64_MAX, hi = INT64_MIN;
    for (int64_t i : idx) {
      lo = std::min(lo, X[i][q]);
      hi = std::max(hi, X[i][q]);
    }
    if (hi - lo > best) {
      best = hi - lo;
      ax = q;
    }
  }
  std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
    return X[a][ax] != X[b][ax] ? X[a][ax] < X[b][ax] : a < b;
  });
  const size_t mid = idx.size() / 2;
  bisect(X, d, std::vector<int64_t>(idx.begin(), idx.begin() + mid), pieces);
  bisect(X, d, std::vector<int64_t>(idx.begin() + mid, idx.end()), pieces);
}

void build_near_boundary(Hierarchy &h) {
  h.nb.clear();
  const int layers = h.opt.nb_layers;
  if (layers <= 0) return;
  const int d = h.d;
  for (int l = h.lc + 1; l <= h.J; ++l) {
    const Csr &A = h.Al.at(l);
    const LevelMesh &lm = level_mesh(h, l);
    NearBnd nb;
    const std::vector<int64_t> J = near_boundary_set(h, l, layers);
    const int64_t n = (int64_t)J.size();
    if (n == 0) continue;
    std::vector<int64_t> pos(A.nrows, -1);
    for (int64_t i = 0; i < n; ++i) pos[J[i]] = i;
    // is some connected component of A_JJ singular (rows summing to zero)? then the dense path
    bool singular = false;
    {
      std::vector<int64_t> comp(n, -1), stack;
      for (int64_t s = 0; s < n && !singular; ++s) {
        if (comp[s] >= 0) continue;
        comp[s] = s;
        stack.assign(1, s);
        double scale = 0.0, rmax = 0.0;
        while (!stack.empty()) {
          const int64_t i = stack.back();
          stack.pop_back();
          double rs = 0.0;
          for (int64_t p = A.rp[J[i]]; p < A.rp[J[i] + 1]; ++p) {
            const int64_t j = pos[A.ci[p]];
            if (j < 0) continue;
            rs += A.v[p];
            if (j == i) scale = std::max(scale, std::fabs(A.v[p]));
            if (j != i && comp[j] < 0) {
              comp[j] = s;
              stack.push_back(j);
            }
          }
          rmax = std::max(rmax, std::fabs(rs));
        }
        singular = rmax <= 1e-10 * scale;
      }
    }
    if (n <= kNbDenseMax || singular) {
      if (n > 4 * kNbDenseMax)
        throw AsmgError{ASMG_EINVAL, "near-boundary set of level " + std::to_string(l) + " covers a singular component of " +
                                         std::to_string(n) + " unknowns, too many for the dense solve"};
      nb.dense = true;
      nb.J = J;
      nb.inv.assign(n * n, 0.0);
      for (int64_t i = 0; i < n; ++i)
        for (int64_t p = A.rp[J[i]]; p < A.rp[J[i] + 1]; ++p)
          if (pos[A.ci[p]] >= 0) nb.inv[i * n + pos[A.ci[p]]] = A.v[p];
      spd_inverse(nb.inv, n, h.threads, true);
      h.nb[l] = std::move(nb);
      continue;
    }
    // domain decomposition: pieces by coordinate bisection, separator, interiors
    std::vector<std::array<int64_t, 3>> X(n);
    for (int64_t i = 0; i < n; ++i) {
      X[i] = {0, 0, 0};
      for (int q = 0; q < d; ++q) X[i][q] = lm.verts[lm.dof_vert[J[i]] * d + q];
    }
    std::vector<std::vector<int64_t>> pieces;
    std::vector<int64_t> all(n);
    std::iota(all.begin(), all.end(), 0);
    bisect(X, d, all, pieces);
    const int64_t P = (int64_t)pieces.size();
    std::vector<int64_t> piece(n);
    for (int64_t p = 0; p < P; ++p)
      for (int64_t i : pieces[p]) piece[i] = p;
    std::vector<uint8_t> inS(n, 0);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t p = A.rp[J[i]]; p < A.rp[J[i] + 1]; ++p) {
        const int64_t j = pos[A.ci[p]];
        if (j >= 0 && j != i && piece[j] < piece[i]) inS[i] = 1;
      }
    // solver order: interiors piece by piece, then the separator (ascending within each)
    std::vector<int64_t> ord, loc(n, -1);
    nb.poff.push_back(0);
    for (int64_t p = 0; p < P; ++p) {
      for (int64_t i : pieces[p])
        if (!inS[i]) ord.push_back(i);
      nb.poff.push_back((int64_t)ord.size());
    }
    nb.nI = (int)ord.size();
    for (int64_t i = 0; i < n; ++i)
      if (inS[i]) ord.push_back(i);
    const int64_t nI = nb.nI, nS = n - nI;
    if (nS > kNbSchurMax)
      throw AsmgError{ASMG_EINVAL, "near-boundary set of level " + std::to_string(l) + ": separator of " +
                                       std::to_string(nS) + " unknowns exceeds the dense Schur limit"};
    for (int64_t q = 0; q < n; ++q) loc[ord[q]] = q;
    nb.J.resize(n);
    for (int64_t q = 0; q < n; ++q) nb.J[q] = J[ord[q]];
    // couplings in solver positions: A_SI (rows S, columns I), A_IS (rows I, columns S)
    auto coupling = [&](bool rows_sep, Csr &C) {
      C.nrows = rows_sep ? nS : nI;
      C.ncols = rows_sep ? nI : nS;
      C.rp.assign(C.nrows + 1, 0);
      C.ci.clear();
      C.v.clear();
      for (int64_t r = 0; r < C.nrows; ++r) {
        const int64_t q = rows_sep ? nI + r : r;
        const int64_t i = ord[q];
        std::vector<std::pair<int32_t, double>> row;
        for (int64_t p = A.rp[J[i]]; p < A.rp[J[i] + 1]; ++p) {
          const int64_t j = pos[A.ci[p]];
          if (j < 0) continue;
          const int64_t qj = loc[j];
          if (rows_sep && qj < nI) row.push_back({(int32_t)qj, A.v[p]});
          if (!rows_sep && qj >= nI) row.push_back({(int32_t)(qj - nI), A.v[p]});
        }
        std::sort(row.begin(), row.end());
        for (auto &e : row) {
          C.ci.push_back(e.first);
          C.v.push_back(e.second);
        }
        C.rp[r + 1] = (int64_t)C.ci.size();
      }
    };
    coupling(true, nb.ASI);
    coupling(false, nb.AIS);
    // interior blocks and their inverses (pieces on host threads)
    nb.boff.assign(P + 1, 0);
    for (int64_t p = 0; p < P; ++p) {
      const int64_t m = nb.poff[p + 1] - nb.poff[p];
      nb.boff[p + 1] = nb.boff[p] + m * m;
    }
    nb.blocks.assign(nb.boff[P], 0.0);
    host_parallel(h.threads, (int)P, [&](int pp) {
      const int64_t p = pp, q0 = nb.poff[p], m = nb.poff[p + 1] - q0;
      if (m == 0) return;
      std::vector<double> M(m * m, 0.0);
      for (int64_t a = 0; a < m; ++a) {
        const int64_t i = ord[q0 + a];
        for (int64_t e = A.rp[J[i]]; e < A.rp[J[i] + 1]; ++e) {
          const int64_t j = pos[A.ci[e]];
          if (j < 0) continue;
          const int64_t qb = loc[j] - q0;
          if (qb >= 0 && qb < m) M[a * m + qb] = A.v[e];
        }
      }
      spd_inverse(M, m, 1, false);
      std::copy(M.begin(), M.end(), nb.blocks.begin() + nb.boff[p]);
    });
    // Schur complement S = A_SS - A_SI A_II^-1 A_IS, accumulated piece by piece
    std::vector<double> S(nS * nS, 0.0);
    for (int64_t r = 0; r < nS; ++r) {
      const int64_t i = ord[nI + r];
      for (int64_t e = A.rp[J[i]]; e < A.rp[J[i] + 1]; ++e) {
        const int64_t j = pos[A.ci[e]];
        if (j >= 0 && loc[j] >= nI) S[r * nS + (loc[j] - nI)] = A.v[e];
      }
    }
    for (int64_t p = 0; p < P; ++p) {
      const int64_t q0 = nb.poff[p], m = nb.poff[p + 1] - q0;
      if (m == 0) continue;
      // separator columns coupled to this piece, and W = A_{I_p}^-1 A_{I_p, cols}
      std::vector<int64_t> cols;
      for (int64_t a = 0; a < m; ++a)
        for (int64_t e = nb.AIS.rp[q0 + a]; e < nb.AIS.rp[q0 + a + 1]; ++e) cols.push_back(nb.AIS.ci[e]);
      std::sort(cols.begin(), cols.end());
      cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
      const int64_t nc = (int64_t)cols.size();
      if (nc == 0) continue;
      std::vector<double> B(m * nc, 0.0), W(m * nc, 0.0);
      for (int64_t a = 0; a < m; ++a)
        for (int64_t e = nb.AIS.rp[q0 + a]; e < nb.AIS.rp[q0 + a + 1]; ++e) {
          const int64_t c = std::lower_bound(cols.begin(), cols.end(), (int64_t)nb.AIS.ci[e]) - cols.begin();
          B[a * nc + c] = nb.AIS.v[e];
        }
      const double *Ai = &nb.blocks[nb.boff[p]];
      for (int64_t a = 0; a < m; ++a)
        for (int64_t b = 0; b < m; ++b) {
          const double w = Ai[a * m + b];
          if (w != 0.0)
            for (int64_t c = 0; c < nc; ++c) W[a * nc + c] += w * B[b * nc + c];
        }
      // S[cols, cols] -= B^T W (A_SI = A_IS^T)
      for (int64_t c1 = 0; c1 < nc; ++c1)
        for (int64_t c2 = 0; c2 < nc; ++c2) {
          double t = 0.0;
          for (int64_t a = 0; a < m; ++a) t += B[a * nc + c1] * W[a * nc + c2];
          S[cols[c1] * nS + cols[c2]] -= t;
        }
    }
    spd_inverse(S, nS, h.threads, false);
    nb.sinv = std::move(S);
    nb.dense = false;
    h.nb[l] = std::move(nb);
  }
}

}  // namespace asmg
