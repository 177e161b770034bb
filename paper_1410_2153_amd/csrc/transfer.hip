// The Scott-Zhang transfer Pi on the device (Section 4.1): (Pi v)(p_i) = integral over sigma_i
// of psi_i v, with sigma_i the edge (2-D) or face (3-D) of unknown i chosen by the host's rule
// and psi_i the L2(sigma_i) dual basis function of its vertex, integrated exactly over the pieces
// of sigma_i cut by the simplices of the finest auxiliary grid sigma^(J).
//
// Identical to build_transfer in setup.cpp: one thread per unknown runs the host's steps with the
// host's floating-point operations in the host's order (this file is compiled without
// contraction): sigma_i, the leaves of the cluster tree meeting its bounding box in depth-first
// child order (a stackless walk), the simplices of those leaves in the grid's order, the clip and
// the quadrature. A counting pass sizes each row; the writing pass stores every contribution
// with the key (row, column) in the order met; a stable radix sort by key and sequential sums of
// each run give the host's result, which orders a row's contributions by column with a stable
// sort and sums equal columns in that order.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "common.hpp"
#include "setup.hpp"
#include "tree.hpp"

// every floating-point operation below rounds on its own (no fused multiply-add), as on the host
#pragma clang fp contract(off)

namespace asmg {
namespace {

constexpr int TT = 128;

__device__ __forceinline__ int tr_level(uint64_t c, int d) { return (63 - __clzll((long long)c)) / d + 1; }

__device__ __forceinline__ void tr_index(uint64_t c, int d, int64_t *idx) {
  const int bits = tr_level(c, d) - 1;
  for (int k = 0; k < d; ++k) idx[k] = 0;
  for (int b = 0; b < bits; ++b)
    for (int k = 0; k < d; ++k) idx[k] |= (int64_t)((c >> (b * d + (d - 1 - k))) & 1) << b;
}

template <class T>
__device__ __forceinline__ int64_t tr_find(const T *__restrict__ a, int64_t n, T v) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo < n && a[lo] == v ? lo : -1;
}

// std::min / std::max as the host evaluates them (the first argument unless the other is
// strictly smaller / larger)
__device__ __forceinline__ double tr_min(double a, double b) { return b < a ? b : a; }
__device__ __forceinline__ double tr_max(double a, double b) { return a < b ? b : a; }

__device__ __forceinline__ double tr_det3(const double *u, const double *v, const double *w) {
  return u[0] * (v[1] * w[2] - v[2] * w[1]) - u[1] * (v[0] * w[2] - v[2] * w[0]) + u[2] * (v[0] * w[1] - v[1] * w[0]);
}

// sigma_i of every vertex: 2-D the smallest-id neighbour, 3-D the lexicographically smallest
// face (j, k) packed as j * 2^32 + k; atomicMin over the elements
__global__ __launch_bounds__(TT) void k_sigma(int64_t ne, int d, const int *__restrict__ E,
                                              unsigned long long *__restrict__ sig) {
  const int64_t e = blockIdx.x * (int64_t)TT + threadIdx.x;
  if (e >= ne) return;
  const int k = d + 1;
  int ev[4];
  for (int a = 0; a < k; ++a) ev[a] = E[e * k + a];
  for (int a = 0; a < k; ++a) {
    if (d == 2) {
      unsigned long long m = ~0ULL;
      for (int b = 0; b < k; ++b)
        if (b != a) m = min(m, (unsigned long long)ev[b] << 32);
      atomicMin(&sig[ev[a]], m);
    } else {
      int o[3], c = 0;
      for (int b = 0; b < 4; ++b)
        if (b != a) o[c++] = ev[b];
      unsigned long long m = ~0ULL;
      for (int x = 0; x < 3; ++x)
        for (int y = x + 1; y < 3; ++y) {
          const unsigned long long j = (unsigned)min(o[x], o[y]), kk = (unsigned)max(o[x], o[y]);
          m = min(m, (j << 32) | kk);
        }
      atomicMin(&sig[ev[a]], m);
    }
  }
}

struct TrArgs {
  int d, J;
  int64_t n;
  double a[3], L, unit;
  int64_t top;
  const int64_t *dofs;
  const double *coords;
  const unsigned long long *sig;
  const uint64_t *R;  // refined boxes, sorted
  int64_t nr;
  const uint64_t *bcode;  // level-J active boxes sorted by code, with their indices
  const int *bidx;
  int64_t nb;
  const int64_t *box_simp;
  const int64_t *simp;
  const int64_t *verts;
  const int64_t *dofv;
  int64_t *cnt;         // counting pass: contributions per row
  const int64_t *off;   // writing pass: first slot of each row (null in the counting pass)
  uint64_t *key;        // (row << 32) | column
  double *val;
};

__device__ double tr_facet_weight(const TrArgs &A, int64_t s, int m) {
  const int d = A.d, k = d + 1;
  for (int q = 0; q < d; ++q) {
    bool lo_all = true, hi_all = true;
    for (int a = 0; a < k; ++a) {
      if (a == m) continue;
      const int64_t x = A.verts[A.simp[s * k + a] * d + q];
      lo_all = lo_all && x == 0;
      hi_all = hi_all && x == A.top;
    }
    if (lo_all || hi_all) return 1.0;
  }
  return 0.5;
}

__global__ __launch_bounds__(TT) void k_transfer(TrArgs A) {
  const int64_t i = blockIdx.x * (int64_t)TT + threadIdx.x;
  if (i >= A.n) return;
  const int d = A.d, k = d + 1;
  const int64_t vi = A.dofs[i];
  const unsigned long long sg = A.sig[vi];
  const int64_t sv[3] = {vi, (int64_t)(sg >> 32), (int64_t)(sg & 0xffffffffULL)};
  double P[3][3];
  for (int m = 0; m < d; ++m)
    for (int q = 0; q < d; ++q) P[m][q] = A.coords[sv[m] * d + q];
  double lo[3], hi[3];
  for (int q = 0; q < d; ++q) {
    lo[q] = hi[q] = P[0][q];
    for (int m = 1; m < d; ++m) {
      lo[q] = tr_min(lo[q], P[m][q]);
      hi[q] = tr_max(hi[q], P[m][q]);
    }
  }
  int64_t ncontrib = 0;
  const int64_t base = A.off ? A.off[i] : 0;
  auto push = [&](int c, double v) {
    if (A.off) {
      A.key[base + ncontrib] = ((uint64_t)i << 32) | (uint32_t)c;
      A.val[base + ncontrib] = v;
    }
    ++ncontrib;
  };
  // leaves of the cluster tree meeting [lo, hi], depth-first in child order, without a stack
  const uint64_t nchild = (uint64_t)1 << d;
  uint64_t b = 1;
  while (true) {
    bool meets = true;
    {
      int64_t idx[3];
      tr_index(b, d, idx);
      const int lev = tr_level(b, d);
      const double side = ldexp(A.L, -(lev - 1));
      for (int q = 0; q < d; ++q) {
        const double b0 = A.a[q] + (double)idx[q] * side, b1 = A.a[q] + (double)(idx[q] + 1) * side;
        if (b0 > hi[q] || b1 < lo[q]) meets = false;
      }
    }
    if (meets) {
      if (tr_find(A.R, A.nr, b) >= 0) {
        b = b << d;  // first child
        continue;
      }
      // a leaf meeting the box: its simplices, if it is an active box of level J
      const int64_t pos = tr_find(A.bcode, A.nb, b);
      if (pos >= 0) {
        const int bi = A.bidx[pos];
        for (int64_t s = A.box_simp[bi]; s < A.box_simp[bi + 1]; ++s) {
          double T[4][3];
          int64_t cols[4];
          for (int m = 0; m < k; ++m) {
            const int64_t vv = A.simp[s * k + m];
            cols[m] = A.dofv[vv];
            for (int q = 0; q < d; ++q) T[m][q] = A.a[q] + (double)A.verts[vv * d + q] * A.unit;
          }
          if (d == 2) {
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
                t0 = fmax(t0, tc);
              else
                t1 = fmin(t1, tc);
            }
            if (empty || !(t1 > t0)) continue;
            const double wgt = on_facet >= 0 ? tr_facet_weight(A, s, on_facet) : 1.0, tm = 0.5 * (t0 + t1);
            for (int m = 0; m < 3; ++m) {
              if (cols[m] < 0) continue;
              auto f = [&](double t) { return (4.0 - 6.0 * t) * (l0[m] + t * (l1[m] - l0[m])); };
              const double v = (t1 - t0) / 6.0 * (f(t0) + 4.0 * f(tm) + f(t1)) * wgt;
              if (v != 0.0) push((int)cols[m], v);
            }
          } else {
            double c[4][3];
            double e1[3], e2[3], e3[3];
            for (int q = 0; q < 3; ++q) {
              e1[q] = T[1][q] - T[0][q];
              e2[q] = T[2][q] - T[0][q];
              e3[q] = T[3][q] - T[0][q];
            }
            const double vol = tr_det3(e1, e2, e3);
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
                c[m][corner] = tr_det3(f1, f2, f3) / vol;
              }
            }
            // clip the reference triangle (s, t) by lambda_m >= 0, m = 0..3 (at most 7 corners)
            double px[8], py[8], qx[8], qy[8];
            int np = 3;
            px[0] = 0.0; py[0] = 0.0;
            px[1] = 1.0; py[1] = 0.0;
            px[2] = 0.0; py[2] = 1.0;
            int on_facet = -1;
            for (int m = 0; m < 4 && np >= 3; ++m) {
              const double c0 = c[m][0], c1 = c[m][1], c2 = c[m][2];
              if (c0 == 0.0 && c1 == 0.0 && c2 == 0.0 && on_facet < 0) on_facet = m;
              int no = 0;
              for (int q = 0; q < np; ++q) {
                const int q1 = (q + 1) % np;
                const double fa = c0 + px[q] * (c1 - c0) + py[q] * (c2 - c0);
                const double fb = c0 + px[q1] * (c1 - c0) + py[q1] * (c2 - c0);
                if (fa >= 0) {
                  qx[no] = px[q];
                  qy[no] = py[q];
                  ++no;
                }
                if ((fa > 0 && fb < 0) || (fa < 0 && fb > 0)) {
                  const double t = fa / (fa - fb);
                  qx[no] = px[q] + t * (px[q1] - px[q]);
                  qy[no] = py[q] + t * (py[q1] - py[q]);
                  ++no;
                }
              }
              np = no;
              for (int q = 0; q < np; ++q) {
                px[q] = qx[q];
                py[q] = qy[q];
              }
            }
            if (np < 3) continue;
            const double wgt = on_facet >= 0 ? tr_facet_weight(A, s, on_facet) : 1.0;
            for (int m = 0; m < 4; ++m) {
              if (cols[m] < 0) continue;
              const double c0 = c[m][0], c1 = c[m][1], c2 = c[m][2];
              auto f = [&](double s_, double t_) {
                return (18.0 - 24.0 * (s_ + t_)) * (c0 + s_ * (c1 - c0) + t_ * (c2 - c0));
              };
              double v = 0.0;
              for (int q = 1; q + 1 < np; ++q) {
                const double ax = px[0], ay = py[0], bx = px[q], by = py[q], cx = px[q + 1], cy = py[q + 1];
                const double area = 0.5 * fabs((bx - ax) * (cy - ay) - (by - ay) * (cx - ax));
                if (area == 0.0) continue;
                v += area *
                     (f(0.5 * (ax + bx), 0.5 * (ay + by)) + f(0.5 * (bx + cx), 0.5 * (by + cy)) +
                      f(0.5 * (cx + ax), 0.5 * (cy + ay))) /
                     3.0;
              }
              v *= wgt;
              if (v != 0.0) push((int)cols[m], v);
            }
          }
        }
      }
    }
    // next box in depth-first order: the next sibling, climbing while b is a last child
    while (b != 1 && (b & (nchild - 1)) == nchild - 1) b >>= d;
    if (b == 1) break;
    ++b;
  }
  if (!A.off) A.cnt[i] = ncontrib;
}

__global__ __launch_bounds__(TT) void k_tr_iota(int64_t n, int *__restrict__ x) {
  const int64_t i = blockIdx.x * (int64_t)TT + threadIdx.x;
  if (i < n) x[i] = (int)i;
}

// first position of each run of equal keys
__global__ __launch_bounds__(TT) void k_tr_heads(int64_t m, const uint64_t *__restrict__ key, int *__restrict__ head) {
  const int64_t i = blockIdx.x * (int64_t)TT + threadIdx.x;
  if (i < m) head[i] = (i == 0 || key[i] != key[i - 1]) ? 1 : 0;
}

// each run summed in order from its first value, written at its position
__global__ __launch_bounds__(TT) void k_tr_runs(int64_t m, const uint64_t *__restrict__ key,
                                                const double *__restrict__ val, const int *__restrict__ head,
                                                const int *__restrict__ pos, uint64_t *__restrict__ ukey,
                                                double *__restrict__ uval) {
  const int64_t i = blockIdx.x * (int64_t)TT + threadIdx.x;
  if (i >= m || !head[i]) return;
  const uint64_t kk = key[i];
  double sum = val[i];
  for (int64_t j = i + 1; j < m && key[j] == kk; ++j) sum += val[j];
  ukey[pos[i]] = kk;
  uval[pos[i]] = sum;
}

template <class T>
T *tr_alloc(std::vector<void *> &keep, int64_t n) {
  void *q = nullptr;
  HIPCHECK(hipMalloc(&q, (size_t)std::max<int64_t>(n, 1) * sizeof(T)));
  keep.push_back(q);
  return (T *)q;
}

}  // namespace

bool build_transfer_device(Hierarchy &h, int ordinal) {
  const int d = h.d, k = d + 1;
  const LevelMesh &lm = h.meshes.at(h.J);
  const int64_t n = h.n(), nb = (int64_t)lm.boxes.size(), ns = (int64_t)lm.simp_box.size();
  if (n >= ((int64_t)1 << 31) || h.nv >= ((int64_t)1 << 31) || nb >= ((int64_t)1 << 31)) return false;
  HIPCHECK(hipSetDevice(ordinal));
  std::vector<void *> keep;
  hipStream_t s = nullptr;
  struct Guard {
    std::vector<void *> &keep;
    hipStream_t &s;
    ~Guard() {
      if (s) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
      }
      for (void *q : keep) (void)hipFree(q);
    }
  } guard{keep, s};
  HIPCHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  std::vector<uint64_t> Rs(h.R.begin(), h.R.end());
  std::sort(Rs.begin(), Rs.end());
  int *E = tr_alloc<int>(keep, h.ne * k);
  unsigned long long *sig = tr_alloc<unsigned long long>(keep, h.nv);
  int64_t *dofs = tr_alloc<int64_t>(keep, n);
  double *X = tr_alloc<double>(keep, h.nv * d);
  uint64_t *R = tr_alloc<uint64_t>(keep, (int64_t)Rs.size()), *BC = tr_alloc<uint64_t>(keep, nb);
  int *BI = tr_alloc<int>(keep, nb);
  int64_t *BS = tr_alloc<int64_t>(keep, nb + 1), *SI = tr_alloc<int64_t>(keep, ns * k);
  int64_t *V = tr_alloc<int64_t>(keep, (int64_t)lm.verts.size()), *DV = tr_alloc<int64_t>(keep, lm.nverts());
  int64_t *cnt = tr_alloc<int64_t>(keep, n), *off = tr_alloc<int64_t>(keep, n + 1);
  HIPCHECK(hipMemcpyAsync(E, h.elems.data(), (size_t)h.ne * k * 4, hipMemcpyHostToDevice, s));
  HIPCHECK(hipMemsetAsync(sig, 0xff, (size_t)h.nv * 8, s));
  HIPCHECK(hipMemcpyAsync(dofs, h.dofs.data(), (size_t)n * 8, hipMemcpyHostToDevice, s));
  HIPCHECK(hipMemcpyAsync(X, h.coords.data(), (size_t)h.nv * d * 8, hipMemcpyHostToDevice, s));
  if (!Rs.empty()) HIPCHECK(hipMemcpyAsync(R, Rs.data(), Rs.size() * 8, hipMemcpyHostToDevice, s));
  // level J's active boxes sorted by code, with their indices (radix sort on the device)
  if (nb) {
    uint64_t *BC0 = tr_alloc<uint64_t>(keep, nb);
    int *BI0 = tr_alloc<int>(keep, nb);
    HIPCHECK(hipMemcpyAsync(BC0, lm.boxes.data(), (size_t)nb * 8, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_tr_iota, dim3((unsigned)((nb + TT - 1) / TT)), dim3(TT), 0, s, nb, BI0);
    size_t tb = 0;
    HIPCHECK(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, BC0, BC, BI0, BI, (int)nb, 0, 64, s));
    void *tmp = tr_alloc<char>(keep, (int64_t)tb);
    HIPCHECK(hipcub::DeviceRadixSort::SortPairs(tmp, tb, BC0, BC, BI0, BI, (int)nb, 0, 64, s));
  }
  HIPCHECK(hipMemcpyAsync(BS, lm.box_simp.data(), (size_t)(nb + 1) * 8, hipMemcpyHostToDevice, s));
  HIPCHECK(hipMemcpyAsync(SI, lm.simp.data(), (size_t)ns * k * 8, hipMemcpyHostToDevice, s));
  HIPCHECK(hipMemcpyAsync(V, lm.verts.data(), lm.verts.size() * 8, hipMemcpyHostToDevice, s));
  HIPCHECK(hipMemcpyAsync(DV, lm.dof_of_vert.data(), (size_t)lm.nverts() * 8, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_sigma, dim3((unsigned)std::max<int64_t>(1, (h.ne + TT - 1) / TT)), dim3(TT), 0, s, h.ne, d,
                     (const int *)E, sig);
  TrArgs a{};
  a.d = d;
  a.J = h.J;
  a.n = n;
  for (int q = 0; q < 3; ++q) a.a[q] = h.a[q];
  a.L = h.L;
  a.unit = std::ldexp(h.L, -h.J);
  a.top = (int64_t)1 << h.J;
  a.dofs = dofs;
  a.coords = X;
  a.sig = sig;
  a.R = R;
  a.nr = (int64_t)Rs.size();
  a.bcode = BC;
  a.bidx = BI;
  a.nb = nb;
  a.box_simp = BS;
  a.simp = SI;
  a.verts = V;
  a.dofv = DV;
  a.cnt = cnt;
  a.off = nullptr;
  const unsigned g = (unsigned)std::max<int64_t>(1, (n + TT - 1) / TT);
  Csr &Pi = h.Pi;
  Pi.nrows = n;
  Pi.ncols = lm.n();
  Pi.rp.assign((size_t)n + 1, 0);
  Pi.ci.clear();
  Pi.v.clear();
  if (n == 0) return true;
  // counting pass, offsets, writing pass
  hipLaunchKernelGGL(k_transfer, dim3(g), dim3(TT), 0, s, a);
  std::vector<int64_t> hc((size_t)n), ho((size_t)n + 1, 0);
  HIPCHECK(hipMemcpyAsync(hc.data(), cnt, (size_t)n * 8, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  for (int64_t i = 0; i < n; ++i) ho[i + 1] = ho[i] + hc[i];
  const int64_t m = ho[n];
  if (m >= ((int64_t)1 << 31)) return false;
  if (m == 0) return true;
  HIPCHECK(hipMemcpyAsync(off, ho.data(), (size_t)(n + 1) * 8, hipMemcpyHostToDevice, s));
  uint64_t *key = tr_alloc<uint64_t>(keep, m), *key_s = tr_alloc<uint64_t>(keep, m);
  double *val = tr_alloc<double>(keep, m), *val_s = tr_alloc<double>(keep, m);
  a.off = off;
  a.key = key;
  a.val = val;
  hipLaunchKernelGGL(k_transfer, dim3(g), dim3(TT), 0, s, a);
  {
    size_t tb = 0;
    HIPCHECK(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, key, key_s, val, val_s, (int)m, 0, 64, s));
    void *tmp = tr_alloc<char>(keep, (int64_t)tb);
    HIPCHECK(hipcub::DeviceRadixSort::SortPairs(tmp, tb, key, key_s, val, val_s, (int)m, 0, 64, s));
  }
  int *head = tr_alloc<int>(keep, m), *pos = tr_alloc<int>(keep, m);
  const unsigned gm = (unsigned)((m + TT - 1) / TT);
  hipLaunchKernelGGL(k_tr_heads, dim3(gm), dim3(TT), 0, s, m, (const uint64_t *)key_s, head);
  {
    size_t tb = 0;
    HIPCHECK(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, head, pos, (int)m, s));
    void *tmp = tr_alloc<char>(keep, (int64_t)tb);
    HIPCHECK(hipcub::DeviceScan::ExclusiveSum(tmp, tb, head, pos, (int)m, s));
  }
  int last_pos = 0, last_head = 0;
  HIPCHECK(hipMemcpyAsync(&last_pos, pos + (m - 1), 4, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipMemcpyAsync(&last_head, head + (m - 1), 4, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  const int64_t nnz = (int64_t)last_pos + last_head;
  uint64_t *ukey = tr_alloc<uint64_t>(keep, nnz);
  double *uval = tr_alloc<double>(keep, nnz);
  hipLaunchKernelGGL(k_tr_runs, dim3(gm), dim3(TT), 0, s, m, (const uint64_t *)key_s, (const double *)val_s,
                     (const int *)head, (const int *)pos, ukey, uval);
  HIPCHECK(hipGetLastError());
  std::vector<uint64_t> hk((size_t)nnz);
  Pi.v.resize((size_t)nnz);
  HIPCHECK(hipMemcpyAsync(hk.data(), ukey, (size_t)nnz * 8, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipMemcpyAsync(Pi.v.data(), uval, (size_t)nnz * 8, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  Pi.ci.resize((size_t)nnz);
  for (int64_t e = 0; e < nnz; ++e) {
    Pi.ci[e] = (int32_t)(hk[e] & 0xffffffffULL);
    Pi.rp[(hk[e] >> 32) + 1]++;
  }
  for (int64_t i = 0; i < n; ++i) Pi.rp[i + 1] += Pi.rp[i];
  return true;
}

}  // namespace asmg
