// Batched engine: many meshes of uneven size, each with up to 4 right-hand sides, solved
// together. One launch sequence per PCG step covers every system.
//
// Merging. Every level is a block-diagonal concatenation over the meshes that have it:
//   - the original grids of all meshes (mesh-major; colour-major inside a mesh);
//   - auxiliary level k = "k-th level below the finest" of each mesh (l = J_m - k).
// At merged level k, the meshes still above their bottom ("smoothing" meshes) come
// first, then the meshes whose bottom level is l = J_m - k. The smoothing rows are
// a prefix of the level's vector.
// A Gauss-Seidel colour pass covers colour c of every smoothing mesh: a segment
// table (one row range per mesh) maps blocks to rows.
// Right-hand sides are interleaved ([row][NR]), so every matrix entry is read once
// per NR systems.
// CG scalars live per system (mesh x rhs). Dot products are segmented per mesh: no
// block straddles two meshes, and the last block of a mesh reduces its partials.
// Converged systems are frozen; the launch sequence stops when all are done.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>
#include <thread>
#include <vector>

#include "batch.hpp"
#include "common.hpp"

namespace asmg {

enum { BST_OK = 0, BST_NOTSPD = 1, BST_NAN = 2, BST_NOCONV = 3 };

template <int NR, class T>
struct alignas(sizeof(T) * NR) VecR {
  T v[NR];
};

__device__ __forceinline__ int find_seg(const int *__restrict__ b0, int nseg, int b) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (b0[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

template <int LPR, int NR, class T>
__device__ __forceinline__ void row_dot_nr(const int *__restrict__ rp, const int *__restrict__ ci,
                                           const T *__restrict__ av, const T *__restrict__ x, int row, bool act,
                                           int lane, T acc[NR]) {
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = 0;
  if (act) {
    const VecR<NR, T> *X = reinterpret_cast<const VecR<NR, T> *>(x);
    const int b = rp[row], e = rp[row + 1];
    for (int k = b + lane; k < e; k += LPR) {
      const T a = av[k];
      const VecR<NR, T> xv = X[ci[k]];
#pragma unroll
      for (int r = 0; r < NR; ++r) acc[r] += a * xv.v[r];
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = group_sum<LPR>(acc[r]);
}

// Gauss-Seidel colour pass over a segment table
template <int LPR, int NR, class T>
__global__ __launch_bounds__(BS) void kb_gs(const int *__restrict__ s_r0, const int *__restrict__ s_r1,
                                            const int *__restrict__ s_b0, int nseg, const int *__restrict__ rp,
                                            const int *__restrict__ ci, const T *__restrict__ av,
                                            const T *__restrict__ invd, const T *__restrict__ b, T *__restrict__ x,
                                            const int *__restrict__ done) {
  if (*done) return;
  const int s = find_seg(s_b0, nseg, blockIdx.x);
  const int t = (blockIdx.x - s_b0[s]) * BS + threadIdx.x;
  const int row = s_r0[s] + t / LPR, lane = t % LPR;
  const bool act = row < s_r1[s];
  T acc[NR];
  row_dot_nr<LPR, NR>(rp, ci, av, x, row, act, lane, acc);
  if (act && lane == 0) {
    const T id = invd[row];
    VecR<NR, T> o;
    const VecR<NR, T> bv = reinterpret_cast<const VecR<NR, T> *>(b)[row];
#pragma unroll
    for (int r = 0; r < NR; ++r) o.v[r] = (bv.v[r] - acc[r]) * id;
    reinterpret_cast<VecR<NR, T> *>(x)[row] = o;
  }
}

// first pass of a sweep from zero over the smoothing rows [0, n): rows of colour 0 of their
// mesh (row < c0 of the mesh segment) get b / a_ii, others 0. Segments = meshes, 1 row per thread.
template <int NR, class T>
__global__ __launch_bounds__(BS) void kb_gs_first(const int *__restrict__ m_r0, const int *__restrict__ m_c0,
                                                  const int *__restrict__ m_r1, const int *__restrict__ m_b0,
                                                  int nseg, const T *__restrict__ b, const T *__restrict__ invd,
                                                  T *__restrict__ x, const int *__restrict__ done) {
  if (*done) return;
  const int s = find_seg(m_b0, nseg, blockIdx.x);
  const int row = m_r0[s] + (blockIdx.x - m_b0[s]) * BS + threadIdx.x;
  if (row >= m_r1[s]) return;
  VecR<NR, T> o;
  if (row < m_c0[s]) {
    const T id = invd[row];
    const VecR<NR, T> bv = reinterpret_cast<const VecR<NR, T> *>(b)[row];
#pragma unroll
    for (int r = 0; r < NR; ++r) o.v[r] = bv.v[r] * id;
  } else {
#pragma unroll
    for (int r = 0; r < NR; ++r) o.v[r] = 0;
  }
  reinterpret_cast<VecR<NR, T> *>(x)[row] = o;
}

// FP64 -> FP32 copy of the fine right-hand side (mixed precision)
template <int NR>
__global__ __launch_bounds__(BS) void kb_cvt(int n, const double *__restrict__ src, float *__restrict__ dst,
                                             const int *__restrict__ done) {
  if (*done) return;
  const int i = blockIdx.x * BS + threadIdx.x;
  if (i < n * NR) dst[i] = (float)src[i];
}

template <int LPR, int NR, class T>
__global__ __launch_bounds__(BS) void kb_residual(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                  const T *__restrict__ av, const T *__restrict__ dg,
                                                  const T *__restrict__ b, const T *__restrict__ x,
                                                  T *__restrict__ r, const int *__restrict__ done) {
  if (*done) return;
  const int t = blockIdx.x * BS + threadIdx.x;
  const int row = t / LPR, lane = t % LPR;
  const bool act = row < n;
  T acc[NR];
  row_dot_nr<LPR, NR>(rp, ci, av, x, row, act, lane, acc);
  if (act && lane == 0) {
    const T d = dg[row];
    const VecR<NR, T> bv = reinterpret_cast<const VecR<NR, T> *>(b)[row];
    const VecR<NR, T> xv = reinterpret_cast<const VecR<NR, T> *>(x)[row];
    VecR<NR, T> o;
#pragma unroll
    for (int q = 0; q < NR; ++q) o.v[q] = bv.v[q] - d * xv.v[q] - acc[q];
    reinterpret_cast<VecR<NR, T> *>(r)[row] = o;
  }
}

template <int LPR, int NR, int ADD, class T>
__global__ __launch_bounds__(BS) void kb_spmv(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                              const T *__restrict__ av, const T *__restrict__ x, T *__restrict__ y,
                                              const int *__restrict__ done) {
  if (*done) return;
  const int t = blockIdx.x * BS + threadIdx.x;
  const int row = t / LPR, lane = t % LPR;
  const bool act = row < n;
  T acc[NR];
  row_dot_nr<LPR, NR>(rp, ci, av, x, row, act, lane, acc);
  if (act && lane == 0) {
    VecR<NR, T> o;
    if (ADD) o = reinterpret_cast<const VecR<NR, T> *>(y)[row];
#pragma unroll
    for (int q = 0; q < NR; ++q) o.v[q] = ADD ? o.v[q] + acc[q] : acc[q];
    reinterpret_cast<VecR<NR, T> *>(y)[row] = o;
  }
}

// bottom solves of the meshes whose V-cycle ends on this level: y = M_m g, one wave per row
template <int NR, class T>
__global__ __launch_bounds__(BS) void kb_gemv(const int *__restrict__ rowpref, int nb, const int *__restrict__ nc,
                                              const int64_t *__restrict__ moff, const int *__restrict__ voff,
                                              const T *__restrict__ M, const T *__restrict__ g, T *__restrict__ y,
                                              const int *__restrict__ done) {
  if (*done) return;
  const int w = blockIdx.x * (BS / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (w >= rowpref[nb]) return;  // whole wave leaves together
  const int s = find_seg(rowpref, nb, w);
  const int i = w - rowpref[s], n = nc[s];
  const T *m = M + moff[s] + (int64_t)i * n;
  const VecR<NR, T> *G = reinterpret_cast<const VecR<NR, T> *>(g) + voff[s];
  T acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = 0;
  for (int j = lane; j < n; j += 64) {
    const T a = m[j];
    const VecR<NR, T> gv = G[j];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] += a * gv.v[r];
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = group_sum<64>(acc[r]);
  if (lane == 0) {
    VecR<NR, T> o;
#pragma unroll
    for (int r = 0; r < NR; ++r) o.v[r] = acc[r];
    reinterpret_cast<VecR<NR, T> *>(y)[voff[s] + i] = o;
  }
}

// ----------------------------------------------------------------------------
// batched CG (fine level, FP64). Block tables: mesh m owns blocks [b0[m], b0[m+1]) and rows
// [r0[m], r1[m]); rows per block = BS / LPR (SpMV-type) or BS (element-wise).
// ----------------------------------------------------------------------------

struct BCtl {  // device pointers of the per-system scalars (arrays of n_meshes * NR)
  double *rho, *pq, *rr, *alpha, *beta, *fn2, *tol2, *rz, *tr;
  int *iter, *dn, *status, *first;
  unsigned *ticket;  // per mesh
  int *active, *gdone;
  int maxit;
};

// Reductions: every block of a CG kernel belongs to one mesh and writes NR partials; a finalize
// kernel with one block per mesh reduces that mesh's partials in a fixed order. No atomics
// except the count of active systems.

template <int NR>
__device__ __forceinline__ void bwrite(double v[NR], double *partials) {
#pragma unroll
  for (int r = 0; r < NR; ++r) v[r] = block_sum(v[r]);
  if (threadIdx.x == 0)
#pragma unroll
    for (int r = 0; r < NR; ++r) partials[(size_t)blockIdx.x * NR + r] = v[r];
}

template <int NR>
__device__ __forceinline__ void breduce(const double *partials, int b0, int b1, double out[NR]) {
  double s[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) s[r] = 0;
  for (int b = b0 + (int)threadIdx.x; b < b1; b += BS)
#pragma unroll
    for (int r = 0; r < NR; ++r) s[r] += partials[(size_t)b * NR + r];
#pragma unroll
  for (int r = 0; r < NR; ++r) out[r] = block_sum(s[r]);
}

__device__ __forceinline__ void bretire(BCtl c, int sys, int status) {
  c.dn[sys] = 1;
  c.status[sys] = status;
  const int prev = atomicSub(c.active, 1);
  if (prev == 1) *c.gdone = 1;
}

template <int NR>
__global__ __launch_bounds__(BS) void kb_cg_init(const int *__restrict__ m_r0, const int *__restrict__ m_r1,
                                                 const int *__restrict__ m_b0, int nm, const double *__restrict__ f,
                                                 double *__restrict__ r, double *__restrict__ u,
                                                 double *__restrict__ p, double *partials) {
  const int m = find_seg(m_b0, nm, blockIdx.x);
  const int row = m_r0[m] + (blockIdx.x - m_b0[m]) * BS + threadIdx.x;
  double v[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) v[q] = 0;
  if (row < m_r1[m]) {
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const size_t i = (size_t)row * NR + q;
      const double fi = f[i];
      r[i] = fi;
      u[i] = 0.0;
      p[i] = 0.0;
      v[q] = fi * fi;
    }
  }
  bwrite<NR>(v, partials);
}

template <int NR>
__global__ __launch_bounds__(BS) void kb_fin_init(const int *__restrict__ m_b0, const double *partials, double tol,
                                                  BCtl c) {
  const int m = blockIdx.x;
  double t[NR];
  breduce<NR>(partials, m_b0[m], m_b0[m + 1], t);
  if (threadIdx.x == 0) {
    int act = 0;
    for (int q = 0; q < NR; ++q) {
      const int sys = m * NR + q;
      c.fn2[sys] = t[q];
      c.tol2[sys] = tol * tol * t[q];
      c.iter[sys] = 0;
      c.status[sys] = BST_OK;
      c.first[sys] = 1;
      c.dn[sys] = (t[q] == 0.0) ? 1 : 0;
      act += (t[q] != 0.0);
    }
    if (act) atomicAdd(c.active, act);
  }
}

template <int LPR, int NR>
__global__ __launch_bounds__(BS) void kb_cg_spmv(const int *__restrict__ m_r0, const int *__restrict__ m_r1,
                                                 const int *__restrict__ m_b0, int nm, const int *__restrict__ rp,
                                                 const int *__restrict__ ci, const double *__restrict__ av,
                                                 const double *__restrict__ dg, const double *__restrict__ p,
                                                 double *__restrict__ q, BCtl c, double *partials) {
  if (*c.gdone) return;
  const int m = find_seg(m_b0, nm, blockIdx.x);
  const int t = (blockIdx.x - m_b0[m]) * BS + threadIdx.x;
  const int row = m_r0[m] + t / LPR, lane = t % LPR;
  const bool act = row < m_r1[m];
  double acc[NR], v[NR];
  row_dot_nr<LPR, NR>(rp, ci, av, p, row, act, lane, acc);
#pragma unroll
  for (int k = 0; k < NR; ++k) v[k] = 0;
  if (act && lane == 0) {
    const double d = dg[row];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const size_t i = (size_t)row * NR + k;
      const double qi = d * p[i] + acc[k];
      q[i] = qi;
      v[k] = p[i] * qi;
    }
  }
  bwrite<NR>(v, partials);
}

template <int NR>
__global__ __launch_bounds__(BS) void kb_fin_spmv(const int *__restrict__ m_b0, const double *partials, BCtl c) {
  if (*c.gdone) return;
  const int m = blockIdx.x;
  double t[NR];
  breduce<NR>(partials, m_b0[m], m_b0[m + 1], t);
  if (threadIdx.x == 0) {
    for (int k = 0; k < NR; ++k) {
      const int sys = m * NR + k;
      if (c.dn[sys]) continue;
      c.pq[sys] = t[k];
      c.iter[sys] += 1;
      if (!(t[k] > 0.0) || !isfinite(t[k]))
        bretire(c, sys, isfinite(t[k]) ? BST_NOTSPD : BST_NAN);
      else
        c.alpha[sys] = c.rho[sys] / t[k];
    }
  }
}

template <int NR>
__global__ __launch_bounds__(BS) void kb_cg_axpy(const int *__restrict__ m_r0, const int *__restrict__ m_r1,
                                                 const int *__restrict__ m_b0, int nm, double *__restrict__ u,
                                                 double *__restrict__ r, const double *__restrict__ p,
                                                 const double *__restrict__ q, BCtl c, double *partials) {
  if (*c.gdone) return;
  const int m = find_seg(m_b0, nm, blockIdx.x);
  const int row = m_r0[m] + (blockIdx.x - m_b0[m]) * BS + threadIdx.x;
  double v[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    v[k] = 0;
    const int sys = m * NR + k;
    if (row < m_r1[m] && !c.dn[sys]) {
      const size_t i = (size_t)row * NR + k;
      const double a = c.alpha[sys];
      u[i] += a * p[i];
      const double ri = r[i] - a * q[i];
      r[i] = ri;
      v[k] = ri * ri;
    }
  }
  bwrite<NR>(v, partials);
}

template <int NR>
__global__ __launch_bounds__(BS) void kb_fin_axpy(const int *__restrict__ m_b0, const double *partials, BCtl c) {
  if (*c.gdone) return;
  const int m = blockIdx.x;
  double t[NR];
  breduce<NR>(partials, m_b0[m], m_b0[m + 1], t);
  if (threadIdx.x == 0) {
    for (int k = 0; k < NR; ++k) {
      const int sys = m * NR + k;
      if (c.dn[sys]) continue;
      c.rr[sys] = t[k];
      if (!isfinite(t[k]))
        bretire(c, sys, BST_NAN);
      else if (t[k] <= c.tol2[sys])
        bretire(c, sys, BST_OK);
      else if (c.iter[sys] >= c.maxit)
        bretire(c, sys, BST_NOCONV);
    }
  }
}

template <int NR, class T>
__global__ __launch_bounds__(BS) void kb_cg_rz(const int *__restrict__ m_r0, const int *__restrict__ m_r1,
                                               const int *__restrict__ m_b0, int nm, const double *__restrict__ r,
                                               const T *__restrict__ z, BCtl c, double *partials) {
  if (*c.gdone) return;
  const int m = find_seg(m_b0, nm, blockIdx.x);
  const int row = m_r0[m] + (blockIdx.x - m_b0[m]) * BS + threadIdx.x;
  double v[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    const size_t i = (size_t)row * NR + k;
    v[k] = row < m_r1[m] ? r[i] * (double)z[i] : 0.0;
  }
  bwrite<NR>(v, partials);
}

template <int NR>
__global__ __launch_bounds__(BS) void kb_fin_rz(const int *__restrict__ m_b0, const double *partials, BCtl c) {
  if (*c.gdone) return;
  const int m = blockIdx.x;
  double t[NR];
  breduce<NR>(partials, m_b0[m], m_b0[m + 1], t);
  if (threadIdx.x == 0) {
    for (int k = 0; k < NR; ++k) {
      const int sys = m * NR + k;
      if (c.dn[sys]) continue;
      c.rz[sys] = t[k];
      if (!(t[k] > 0.0) || !isfinite(t[k])) {
        bretire(c, sys, isfinite(t[k]) ? BST_NOTSPD : BST_NAN);
      } else if (c.first[sys]) {
        c.beta[sys] = 0.0;
        c.rho[sys] = t[k];
        c.first[sys] = 0;
      } else {
        c.beta[sys] = t[k] / c.rho[sys];
        c.rho[sys] = t[k];
      }
    }
  }
}

template <int NR, class T>
__global__ __launch_bounds__(BS) void kb_cg_p(const int *__restrict__ m_r0, const int *__restrict__ m_r1,
                                              const int *__restrict__ m_b0, int nm, const T *__restrict__ z,
                                              double *__restrict__ p, BCtl c) {
  if (*c.gdone) return;
  const int m = find_seg(m_b0, nm, blockIdx.x);
  const int row = m_r0[m] + (blockIdx.x - m_b0[m]) * BS + threadIdx.x;
  if (row >= m_r1[m]) return;
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    const int sys = m * NR + k;
    if (c.dn[sys]) continue;
    const size_t i = (size_t)row * NR + k;
    p[i] = (double)z[i] + c.beta[sys] * p[i];
  }
}

template <int LPR, int NR>
__global__ __launch_bounds__(BS) void kb_true_res(const int *__restrict__ m_r0, const int *__restrict__ m_r1,
                                                  const int *__restrict__ m_b0, int nm, const int *__restrict__ rp,
                                                  const int *__restrict__ ci, const double *__restrict__ av,
                                                  const double *__restrict__ dg, const double *__restrict__ f,
                                                  const double *__restrict__ u, double *partials) {
  const int m = find_seg(m_b0, nm, blockIdx.x);
  const int t = (blockIdx.x - m_b0[m]) * BS + threadIdx.x;
  const int row = m_r0[m] + t / LPR, lane = t % LPR;
  const bool act = row < m_r1[m];
  double acc[NR], v[NR];
  row_dot_nr<LPR, NR>(rp, ci, av, u, row, act, lane, acc);
#pragma unroll
  for (int k = 0; k < NR; ++k) v[k] = 0;
  if (act && lane == 0) {
    const double d = dg[row];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const size_t i = (size_t)row * NR + k;
      const double e = f[i] - d * u[i] - acc[k];
      v[k] = e * e;
    }
  }
  bwrite<NR>(v, partials);
}

template <int NR>
__global__ __launch_bounds__(BS) void kb_fin_tr(const int *__restrict__ m_b0, const double *partials, BCtl c) {
  const int m = blockIdx.x;
  double t[NR];
  breduce<NR>(partials, m_b0[m], m_b0[m + 1], t);
  if (threadIdx.x == 0)
    for (int k = 0; k < NR; ++k) c.tr[m * NR + k] = t[k];
}

// restart systems whose true residual is above tol (mixed precision): r = f - A u, p = 0
template <int LPR, int NR>
__global__ __launch_bounds__(BS) void kb_restart(const int *__restrict__ m_r0, const int *__restrict__ m_r1,
                                                 const int *__restrict__ m_b0, int nm, const int *__restrict__ rp,
                                                 const int *__restrict__ ci, const double *__restrict__ av,
                                                 const double *__restrict__ dg, const double *__restrict__ f,
                                                 const double *__restrict__ u, double *__restrict__ r,
                                                 double *__restrict__ p, const int *__restrict__ mask) {
  const int m = find_seg(m_b0, nm, blockIdx.x);
  const int t = (blockIdx.x - m_b0[m]) * BS + threadIdx.x;
  const int row = m_r0[m] + t / LPR, lane = t % LPR;
  const bool act = row < m_r1[m];
  double acc[NR];
  row_dot_nr<LPR, NR>(rp, ci, av, u, row, act, lane, acc);
  if (act && lane == 0) {
    const double d = dg[row];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      if (!mask[m * NR + k]) continue;
      const size_t i = (size_t)row * NR + k;
      r[i] = f[i] - d * u[i] - acc[k];
      p[i] = 0.0;
    }
  }
}

// input [mesh][rhs][dof] -> internal [row][NR]; output the reverse
template <int NR>
__global__ __launch_bounds__(BS) void kb_gather(int n, const int64_t *__restrict__ src0, const int *__restrict__ stride,
                                                const double *__restrict__ F, double *__restrict__ f) {
  const int row = blockIdx.x * BS + threadIdx.x;
  if (row >= n) return;
  const int64_t s0 = src0[row];
  const int st = stride[row];
#pragma unroll
  for (int k = 0; k < NR; ++k) f[(size_t)row * NR + k] = F[s0 + (int64_t)k * st];
}

template <int NR>
__global__ __launch_bounds__(BS) void kb_scatter(int n, const int64_t *__restrict__ src0, const int *__restrict__ stride,
                                                 const double *__restrict__ u, double *__restrict__ U) {
  const int row = blockIdx.x * BS + threadIdx.x;
  if (row >= n) return;
  const int64_t s0 = src0[row];
  const int st = stride[row];
#pragma unroll
  for (int k = 0; k < NR; ++k) U[s0 + (int64_t)k * st] = u[(size_t)row * NR + k];
}

// ----------------------------------------------------------------------------
// host-side merged structures
// ----------------------------------------------------------------------------

struct BCsr {
  int nrows = 0, ncols = 0;
  int64_t nnz = 0;
  int *rp = nullptr, *ci = nullptr;
  double *v64 = nullptr;
  float *v32 = nullptr;
  int lpr = 4;
};

struct SegTable {  // rows [r0, r1) per segment; first block of each segment (prefix, nseg + 1 entries)
  int nseg = 0, nblocks = 0;
  int *r0 = nullptr, *r1 = nullptr, *b0 = nullptr, *c0 = nullptr;
};

struct BLevel {
  int nrows = 0;         // all rows (smoothing meshes, then bottom meshes)
  int nsmooth = 0;       // rows of smoothing meshes (a prefix)
  std::vector<int> mesh; // meshes present; smoothing first
  std::vector<int> off;  // row offset of each present mesh
  std::vector<SegTable> colour;  // colour passes over smoothing meshes (built for the matrix LPR)
  SegTable first;        // mesh segments with colour-0 ends (1 row per thread)
  BCsr A;                // off-diagonal, smoothing rows
  double *dg64 = nullptr, *id64 = nullptr;
  float *dg32 = nullptr, *id32 = nullptr;
  double *x64 = nullptr, *b64 = nullptr, *r64 = nullptr;
  float *x32 = nullptr, *b32 = nullptr, *r32 = nullptr;
  BCsr P, PT;            // P: rows = smoothing rows, cols = rows of level k+1
  // bottom meshes
  int nbottom = 0;
  int *bt_rowpref = nullptr, *bt_nc = nullptr, *bt_voff = nullptr;
  int64_t *bt_moff = nullptr;
  double *inv64 = nullptr;
  float *inv32 = nullptr;
  int bottom_rows = 0;
};

struct BatchDevice {
  int ordinal = 0, nm = 0, d = 2, nu_aux = 2, nu_fine = 1, maxit = 1000, precision = 0;
  std::vector<void *> allocs;
  std::vector<int64_t> n_m;       // unknowns per mesh
  std::vector<int64_t> dof_off;   // prefix of n_m (user vectors, per rhs block)
  // fine level
  BLevel fine;                    // nsmooth = nrows
  SegTable fine_sp, fine_ew;      // per-mesh block tables for SpMV-type / element-wise CG kernels
  BCsr Pi, PiT;
  int *row_stride = nullptr;      // gather/scatter
  int64_t *row_src0[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // per NR (index NR)
  std::vector<BLevel> aux;        // merged level k = 0..K
  // CG
  double *f = nullptr, *u = nullptr, *r = nullptr, *p = nullptr, *q = nullptr;
  double *partials = nullptr;
  BCtl ctl{};
  int *ctl_ints = nullptr;        // backing store of the int arrays
  int *mask = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraphExec_t graph[2][5] = {{nullptr}};
  int last_iters[2][5] = {{0}};
  bool use_graph = true;
  // byte model
  bool count_bytes = false;
  double bytes = 0;
};

template <class T>
static T *balloc(BatchDevice *dv, int64_t n) {
  if (n <= 0) n = 1;
  void *p = nullptr;
  HIPCHECK(hipMalloc(&p, (size_t)n * sizeof(T)));
  dv->allocs.push_back(p);
  return (T *)p;
}

template <class T>
static T *bupload(BatchDevice *dv, const std::vector<T> &v) {
  T *p = balloc<T>(dv, (int64_t)v.size());
  if (!v.empty()) HIPCHECK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return p;
}

struct HMat {  // host CSR in merged numbering
  int nrows = 0, ncols = 0;
  std::vector<int> rp{0}, ci;
  std::vector<double> v;
};

// append rows of A (rows in order rperm, columns mapped by cmap + col_shift) to M
static void append_rows(HMat &M, const Csr &A, const std::vector<int> &rperm, const std::vector<int> *cmap,
                        int col_shift, bool split_diag, std::vector<double> *diag) {
  std::vector<std::pair<int, double>> row;
  for (size_t i = 0; i < rperm.size(); ++i) {
    const int64_t o = rperm[i];
    row.clear();
    double dval = 0;
    for (int64_t p = A.rp[o]; p < A.rp[o + 1]; ++p) {
      if (split_diag && A.ci[p] == o) {
        dval = A.v[p];
        continue;
      }
      const int c = (cmap ? (*cmap)[A.ci[p]] : A.ci[p]) + col_shift;
      row.push_back({c, A.v[p]});
    }
    std::sort(row.begin(), row.end());
    for (auto &e : row) {
      M.ci.push_back(e.first);
      M.v.push_back(e.second);
    }
    M.rp.push_back((int)M.ci.size());
    if (diag) diag->push_back(dval);
  }
  M.nrows += (int)rperm.size();
}

static HMat htranspose(const HMat &A) {
  HMat T;
  T.nrows = A.ncols;
  T.ncols = A.nrows;
  T.rp.assign(T.nrows + 1, 0);
  for (int c : A.ci) T.rp[c + 1]++;
  for (int i = 0; i < T.nrows; ++i) T.rp[i + 1] += T.rp[i];
  T.ci.resize(A.ci.size());
  T.v.resize(A.v.size());
  std::vector<int> pos(T.rp.begin(), T.rp.end() - 1);
  for (int i = 0; i < A.nrows; ++i)
    for (int p = A.rp[i]; p < A.rp[i + 1]; ++p) {
      const int q = pos[A.ci[p]]++;
      T.ci[q] = i;
      T.v[q] = A.v[p];
    }
  return T;
}

static void bupload_csr(BatchDevice *dv, const HMat &H, BCsr &D) {
  D.nrows = H.nrows;
  D.ncols = H.ncols;
  D.nnz = (int64_t)H.ci.size();
  D.rp = bupload(dv, H.rp);
  D.ci = bupload(dv, H.ci);
  D.v64 = bupload(dv, H.v);
  std::vector<float> f(H.v.begin(), H.v.end());
  D.v32 = bupload(dv, f);
  D.lpr = pick_lpr(D.nnz, D.nrows);
}

static SegTable make_segs(BatchDevice *dv, const std::vector<int> &r0, const std::vector<int> &r1,
                          const std::vector<int> *c0, int rows_per_block) {
  SegTable S;
  std::vector<int> a, b, blk, cc;
  int nb = 0;
  for (size_t i = 0; i < r0.size(); ++i) {
    if (r1[i] <= r0[i]) continue;
    a.push_back(r0[i]);
    b.push_back(r1[i]);
    if (c0) cc.push_back((*c0)[i]);
    blk.push_back(nb);
    nb += (r1[i] - r0[i] + rows_per_block - 1) / rows_per_block;
  }
  blk.push_back(nb);
  S.nseg = (int)a.size();
  S.nblocks = nb;
  S.r0 = bupload(dv, a);
  S.r1 = bupload(dv, b);
  S.b0 = bupload(dv, blk);
  if (c0) S.c0 = bupload(dv, cc);
  return S;
}

// per-mesh block tables that keep every mesh's rows in blocks of its own (empty meshes keep
// one block so that per-mesh reductions always have a finishing block)
static SegTable make_mesh_blocks(BatchDevice *dv, const std::vector<int> &r0, const std::vector<int> &r1,
                                 int rows_per_block) {
  SegTable S;
  std::vector<int> blk;
  int nb = 0;
  for (size_t i = 0; i < r0.size(); ++i) {
    blk.push_back(nb);
    nb += std::max(1, (r1[i] - r0[i] + rows_per_block - 1) / rows_per_block);
  }
  blk.push_back(nb);
  S.nseg = (int)r0.size();
  S.nblocks = nb;
  S.r0 = bupload(dv, r0);
  S.r1 = bupload(dv, r1);
  S.b0 = bupload(dv, blk);
  return S;
}

static void colour_perm(const std::vector<int32_t> &col, std::vector<int> &perm, std::vector<int> &iperm,
                        std::vector<int> &coff) {
  const int n = (int)col.size();
  int C = 0;
  for (int c : col) C = std::max(C, c + 1);
  coff.assign(C + 1, 0);
  for (int c : col) coff[c + 1]++;
  for (int c = 0; c < C; ++c) coff[c + 1] += coff[c];
  perm.resize(n);
  std::vector<int> pos(coff.begin(), coff.end() - 1);
  for (int i = 0; i < n; ++i) perm[pos[col[i]]++] = i;
  iperm.resize(n);
  for (int i = 0; i < n; ++i) iperm[perm[i]] = i;
}

static void alloc_level_vectors(BatchDevice *dv, BLevel &L) {
  const int64_t n = (int64_t)L.nrows * 4;  // room for up to 4 right-hand sides
  L.x64 = balloc<double>(dv, n);
  L.b64 = balloc<double>(dv, n);
  L.r64 = balloc<double>(dv, n);
  L.x32 = balloc<float>(dv, n);
  L.b32 = balloc<float>(dv, n);
  L.r32 = balloc<float>(dv, n);
}

static void upload_diag(BatchDevice *dv, BLevel &L, const std::vector<double> &diag) {
  std::vector<double> inv(diag.size());
  std::vector<float> d32(diag.begin(), diag.end()), i32(diag.size());
  for (size_t i = 0; i < diag.size(); ++i) {
    inv[i] = 1.0 / diag[i];
    i32[i] = 1.0f / (float)diag[i];
  }
  L.dg64 = bupload(dv, diag);
  L.id64 = bupload(dv, inv);
  L.dg32 = bupload(dv, d32);
  L.id32 = bupload(dv, i32);
}

BatchDevice *batch_device_create(std::vector<std::unique_ptr<Hierarchy>> &H, int ordinal) {
  int count = 0;
  HIPCHECK(hipGetDeviceCount(&count));
  if (ordinal < 0 || ordinal >= count) throw AsmgError{ASMG_EDEVICE, "no such HIP device"};
  HIPCHECK(hipSetDevice(ordinal));
  BatchDevice *dv = new BatchDevice();
  try {
    const int nm = (int)H.size();
    dv->ordinal = ordinal;
    dv->nm = nm;
    dv->d = H[0]->d;
    dv->nu_aux = H[0]->opt.nu_aux;
    dv->nu_fine = H[0]->opt.nu_fine;
    dv->maxit = H[0]->opt.max_iter;
    dv->precision = H[0]->opt.precision;
    // per-mesh colour-major orderings of every smoothing level
    struct MeshOrd {
      std::vector<int> perm, iperm, coff;
    };
    std::vector<MeshOrd> fine(nm);
    std::vector<std::vector<MeshOrd>> lev(nm);  // index k (aux level J - k), smoothing levels only
    int K = 0;
    dv->n_m.resize(nm);
    dv->dof_off.assign(nm + 1, 0);
    for (int m = 0; m < nm; ++m) {
      Hierarchy &h = *H[m];
      colour_perm(h.colour_fine, fine[m].perm, fine[m].iperm, fine[m].coff);
      const int D = h.J - h.lc;
      K = std::max(K, D);
      lev[m].resize(D);
      for (int k = 0; k < D; ++k)
        colour_perm(h.colour_aux.at(h.J - k), lev[m][k].perm, lev[m][k].iperm, lev[m][k].coff);
      dv->n_m[m] = h.n();
      dv->dof_off[m + 1] = dv->dof_off[m] + h.n();
    }
    if (dv->dof_off[nm] * 4 > INT32_MAX) throw AsmgError{ASMG_EINVAL, "batch too large"};
    // ---- fine level
    {
      BLevel &F = dv->fine;
      HMat A;
      std::vector<double> diag;
      std::vector<int> r0, r1, c0;
      int off = 0;
      int C = 0;
      for (int m = 0; m < nm; ++m) {
        F.mesh.push_back(m);
        F.off.push_back(off);
        append_rows(A, H[m]->A, fine[m].perm, &fine[m].iperm, off, true, &diag);
        C = std::max(C, (int)fine[m].coff.size() - 1);
        r0.push_back(off);
        r1.push_back(off + (int)H[m]->n());
        c0.push_back(off + fine[m].coff[1]);
        off += (int)H[m]->n();
      }
      A.ncols = off;
      F.nrows = F.nsmooth = off;
      bupload_csr(dv, A, F.A);
      upload_diag(dv, F, diag);
      alloc_level_vectors(dv, F);
      for (int c = 0; c < C; ++c) {
        std::vector<int> a, b;
        for (int m = 0; m < nm; ++m) {
          const auto &co = fine[m].coff;
          if (c + 1 < (int)co.size()) {
            a.push_back(F.off[m] + co[c]);
            b.push_back(F.off[m] + co[c + 1]);
          }
        }
        F.colour.push_back(make_segs(dv, a, b, nullptr, BS / F.A.lpr));
      }
      F.first = make_segs(dv, r0, r1, &c0, BS);
      dv->fine_sp = make_mesh_blocks(dv, r0, r1, BS / F.A.lpr);
      dv->fine_ew = make_mesh_blocks(dv, r0, r1, BS);
    }
    // ---- auxiliary levels k = 0..K
    dv->aux.resize(K + 1);
    for (int k = 0; k <= K; ++k) {
      BLevel &L = dv->aux[k];
      std::vector<int> sm, bt;
      for (int m = 0; m < nm; ++m) {
        const int D = H[m]->J - H[m]->lc;
        if (D > k) sm.push_back(m);
        if (D == k) bt.push_back(m);
      }
      int off = 0;
      HMat A;
      std::vector<double> diag;
      std::vector<int> r0, r1, c0;
      int C = 0;
      for (int m : sm) {
        L.mesh.push_back(m);
        L.off.push_back(off);
        const int l = H[m]->J - k;
        append_rows(A, H[m]->Al.at(l), lev[m][k].perm, &lev[m][k].iperm, off, true, &diag);
        C = std::max(C, (int)lev[m][k].coff.size() - 1);
        r0.push_back(off);
        const int nl = (int)H[m]->Al.at(l).nrows;
        r1.push_back(off + nl);
        c0.push_back(off + lev[m][k].coff[1]);
        off += nl;
      }
      L.nsmooth = off;
      A.ncols = off;
      bupload_csr(dv, A, L.A);
      upload_diag(dv, L, diag);
      for (int c = 0; c < C; ++c) {
        std::vector<int> a, b;
        for (size_t i = 0; i < sm.size(); ++i) {
          const auto &co = lev[sm[i]][k].coff;
          if (c + 1 < (int)co.size()) {
            a.push_back(L.off[i] + co[c]);
            b.push_back(L.off[i] + co[c + 1]);
          }
        }
        L.colour.push_back(make_segs(dv, a, b, nullptr, BS / L.A.lpr));
      }
      L.first = make_segs(dv, r0, r1, &c0, BS);
      // bottom meshes
      std::vector<int> pref{0}, ncs, voff;
      std::vector<int64_t> moff;
      std::vector<double> inv;
      for (int m : bt) {
        L.mesh.push_back(m);
        L.off.push_back(off);
        const int nc = (int)H[m]->nc;
        ncs.push_back(nc);
        voff.push_back(off);
        moff.push_back((int64_t)inv.size());
        inv.insert(inv.end(), H[m]->coarse_inv.begin(), H[m]->coarse_inv.end());
        pref.push_back(pref.back() + nc);
        off += nc;
      }
      L.nrows = off;
      L.nbottom = (int)bt.size();
      L.bottom_rows = pref.back();
      L.bt_rowpref = bupload(dv, pref);
      L.bt_nc = bupload(dv, ncs);
      L.bt_voff = bupload(dv, voff);
      L.bt_moff = bupload(dv, moff);
      L.inv64 = bupload(dv, inv);
      std::vector<float> inv32(inv.begin(), inv.end());
      L.inv32 = bupload(dv, inv32);
      alloc_level_vectors(dv, L);
    }
    // ---- prolongations P (level k+1 -> k) for the smoothing meshes of level k
    for (int k = 0; k < K; ++k) {
      BLevel &L = dv->aux[k], &Lc = dv->aux[k + 1];
      HMat P;
      for (size_t i = 0; i < L.mesh.size(); ++i) {
        const int m = L.mesh[i];
        const int D = H[m]->J - H[m]->lc;
        if (D <= k) break;  // bottom meshes follow the smoothing ones
        const int l = H[m]->J - k;
        const size_t j = std::find(Lc.mesh.begin(), Lc.mesh.end(), m) - Lc.mesh.begin();
        const std::vector<int> *cmap = (D > k + 1) ? &lev[m][k + 1].iperm : nullptr;
        append_rows(P, H[m]->P.at(l), lev[m][k].perm, cmap, Lc.off[j], false, nullptr);
      }
      P.ncols = Lc.nrows;
      bupload_csr(dv, P, L.P);
      bupload_csr(dv, htranspose(P), L.PT);
    }
    // ---- Pi (fine rows -> merged level 0 rows)
    {
      HMat Pi;
      BLevel &L0 = dv->aux[0];
      for (int m = 0; m < nm; ++m) {
        const int D = H[m]->J - H[m]->lc;
        const size_t j = std::find(L0.mesh.begin(), L0.mesh.end(), m) - L0.mesh.begin();
        const std::vector<int> *cmap = D > 0 ? &lev[m][0].iperm : nullptr;
        append_rows(Pi, H[m]->Pi, fine[m].perm, cmap, L0.off[j], false, nullptr);
      }
      Pi.ncols = L0.nrows;
      bupload_csr(dv, Pi, dv->Pi);
      bupload_csr(dv, htranspose(Pi), dv->PiT);
    }
    // ---- gather/scatter maps: internal fine row -> user offset of (mesh, rhs 0, dof), stride n_m
    {
      const int n = dv->fine.nrows;
      std::vector<int> stride(n);
      for (int NR = 1; NR <= 4; NR *= 2) {
        std::vector<int64_t> src(n);
        for (int m = 0; m < nm; ++m)
          for (int64_t i = 0; i < dv->n_m[m]; ++i) {
            const int row = dv->fine.off[m] + (int)i;
            src[row] = dv->dof_off[m] * NR + fine[m].perm[i];
            stride[row] = (int)dv->n_m[m];
          }
        dv->row_src0[NR] = bupload(dv, src);
      }
      dv->row_stride = bupload(dv, stride);
    }
    // ---- CG vectors and scalars
    const int64_t nv = (int64_t)dv->fine.nrows * 4;
    dv->f = balloc<double>(dv, nv);
    dv->u = balloc<double>(dv, nv);
    dv->r = balloc<double>(dv, nv);
    dv->p = balloc<double>(dv, nv);
    dv->q = balloc<double>(dv, nv);
    const int ns = nm * 4;
    dv->partials = balloc<double>(dv, (int64_t)std::max(dv->fine_sp.nblocks, dv->fine_ew.nblocks) * 4);
    double *sc = balloc<double>(dv, (int64_t)ns * 9);
    HIPCHECK(hipMemset(sc, 0, (size_t)ns * 9 * sizeof(double)));
    dv->ctl.rho = sc;
    dv->ctl.pq = sc + ns;
    dv->ctl.rr = sc + 2 * ns;
    dv->ctl.alpha = sc + 3 * ns;
    dv->ctl.beta = sc + 4 * ns;
    dv->ctl.fn2 = sc + 5 * ns;
    dv->ctl.tol2 = sc + 6 * ns;
    dv->ctl.rz = sc + 7 * ns;
    dv->ctl.tr = sc + 8 * ns;
    // ints: iter, done, status, first (ns each), tickets (nm), active, gdone, and an always-zero flag
    int *ci = balloc<int>(dv, (int64_t)ns * 4 + nm + 3);
    HIPCHECK(hipMemset(ci, 0, ((size_t)ns * 4 + nm + 3) * sizeof(int)));
    dv->ctl_ints = ci;
    dv->ctl.iter = ci;
    dv->ctl.dn = ci + ns;
    dv->ctl.status = ci + 2 * ns;
    dv->ctl.first = ci + 3 * ns;
    dv->ctl.ticket = (unsigned *)(ci + 4 * ns);
    dv->ctl.active = ci + 4 * ns + nm;
    dv->ctl.gdone = ci + 4 * ns + nm + 1;
    dv->ctl.maxit = dv->maxit;
    dv->mask = balloc<int>(dv, ns);
    HIPCHECK(hipStreamCreateWithFlags(&dv->stream, hipStreamNonBlocking));
    HIPCHECK(hipEventCreateWithFlags(&dv->ev_in, hipEventDisableTiming));
    HIPCHECK(hipEventCreateWithFlags(&dv->ev_out, hipEventDisableTiming));
    HIPCHECK(hipDeviceSynchronize());
  } catch (...) {
    batch_device_destroy(dv);
    throw;
  }
  return dv;
}

void batch_device_destroy(BatchDevice *dv) {
  if (!dv) return;
  (void)hipSetDevice(dv->ordinal);
  if (dv->stream) (void)hipStreamSynchronize(dv->stream);
  for (auto &g : dv->graph)
    for (auto &x : g)
      if (x) (void)hipGraphExecDestroy(x);
  if (dv->ev_in) (void)hipEventDestroy(dv->ev_in);
  if (dv->ev_out) (void)hipEventDestroy(dv->ev_out);
  if (dv->stream) (void)hipStreamDestroy(dv->stream);
  for (void *p : dv->allocs) (void)hipFree(p);
  delete dv;
}

void batch_device_set_precision(BatchDevice *dv, int precision) { dv->precision = precision; }

// ----------------------------------------------------------------------------
// launch sequence
// ----------------------------------------------------------------------------

template <class T>
struct BV;
template <>
struct BV<double> {
  static double *x(BLevel &L) { return L.x64; }
  static double *b(BLevel &L) { return L.b64; }
  static double *r(BLevel &L) { return L.r64; }
  static const double *dg(BLevel &L) { return L.dg64; }
  static const double *id(BLevel &L) { return L.id64; }
  static const double *v(const BCsr &A) { return A.v64; }
  static const double *inv(BLevel &L) { return L.inv64; }
};
template <>
struct BV<float> {
  static float *x(BLevel &L) { return L.x32; }
  static float *b(BLevel &L) { return L.b32; }
  static float *r(BLevel &L) { return L.r32; }
  static const float *dg(BLevel &L) { return L.dg32; }
  static const float *id(BLevel &L) { return L.id32; }
  static const float *v(const BCsr &A) { return A.v32; }
  static const float *inv(BLevel &L) { return L.inv32; }
};

static inline double bcsr_bytes(const BCsr &A, int s) { return (double)A.nnz * (s + 4) + 4.0 * (A.nrows + 1); }

template <int NR, class T>
static void b_sweep(BatchDevice *dv, BLevel &L, const T *b, bool from_zero, bool forward, const int *done,
                    hipStream_t s) {
  if (L.nsmooth == 0) return;
  T *x = BV<T>::x(L);
  const int C = (int)L.colour.size();
  auto pass = [&](int c) {
    const SegTable &S = L.colour[c];
    if (S.nblocks == 0) return;
    with_lpr(L.A.lpr, [&](auto cc) {
      constexpr int LP = decltype(cc)::value;
      hipLaunchKernelGGL((kb_gs<LP, NR, T>), dim3(S.nblocks), dim3(BS), 0, s, S.r0, S.r1, S.b0, S.nseg, L.A.rp,
                         L.A.ci, BV<T>::v(L.A), BV<T>::id(L), b, x, done);
    });
  };
  if (forward) {
    int c = 0;
    if (from_zero) {
      hipLaunchKernelGGL((kb_gs_first<NR, T>), dim3(L.first.nblocks), dim3(BS), 0, s, L.first.r0, L.first.c0,
                         L.first.r1, L.first.b0, L.first.nseg, b, BV<T>::id(L), x, done);
      c = 1;
    }
    for (; c < C; ++c) pass(c);
  } else {
    for (int c = C - 1; c >= 0; --c) pass(c);
  }
  if (dv->count_bytes) dv->bytes += bcsr_bytes(L.A, sizeof(T)) + (double)L.nsmooth * sizeof(T) * (3.0 * NR + 1);
}

template <int NR, class T>
static void b_residual(BatchDevice *dv, BLevel &L, const T *b, const int *done, hipStream_t s) {
  if (L.nsmooth == 0) return;
  with_lpr(L.A.lpr, [&](auto cc) {
    constexpr int LP = decltype(cc)::value;
    hipLaunchKernelGGL((kb_residual<LP, NR, T>), dim3(nblk((int64_t)L.nsmooth * LP)), dim3(BS), 0, s, L.nsmooth,
                       L.A.rp, L.A.ci, BV<T>::v(L.A), BV<T>::dg(L), b, BV<T>::x(L), BV<T>::r(L), done);
  });
  if (dv->count_bytes) dv->bytes += bcsr_bytes(L.A, sizeof(T)) + (double)L.nsmooth * sizeof(T) * (3.0 * NR + 1);
}

template <int NR, int ADD, class T>
static void b_spmv(BatchDevice *dv, const BCsr &A, const T *x, T *y, const int *done, hipStream_t s) {
  if (A.nrows == 0) return;
  with_lpr(A.lpr, [&](auto cc) {
    constexpr int LP = decltype(cc)::value;
    hipLaunchKernelGGL((kb_spmv<LP, NR, ADD, T>), dim3(nblk((int64_t)A.nrows * LP)), dim3(BS), 0, s, A.nrows, A.rp,
                       A.ci, BV<T>::v(A), x, y, done);
  });
  if (dv->count_bytes)
    dv->bytes += bcsr_bytes(A, sizeof(T)) + (double)sizeof(T) * NR * (A.ncols + (1 + ADD) * (double)A.nrows);
}

template <int NR, class T>
static void b_vcycle(BatchDevice *dv, int k, const int *done, hipStream_t s) {
  BLevel &L = dv->aux[k];
  const T *b = BV<T>::b(L);
  if (L.nbottom > 0 && L.bottom_rows > 0) {
    hipLaunchKernelGGL((kb_gemv<NR, T>), dim3(nblk((int64_t)L.bottom_rows * 64)), dim3(BS), 0, s, L.bt_rowpref,
                       L.nbottom, L.bt_nc, L.bt_moff, L.bt_voff, BV<T>::inv(L), b, BV<T>::x(L), done);
  }
  if (L.nsmooth == 0) return;
  for (int it = 0; it < dv->nu_aux; ++it) b_sweep<NR, T>(dv, L, b, it == 0, true, done, s);
  b_residual<NR, T>(dv, L, b, done, s);
  BLevel &Lc = dv->aux[k + 1];
  b_spmv<NR, 0, T>(dv, L.PT, BV<T>::r(L), BV<T>::b(Lc), done, s);
  b_vcycle<NR, T>(dv, k + 1, done, s);
  b_spmv<NR, 1, T>(dv, L.P, BV<T>::x(Lc), BV<T>::x(L), done, s);
  for (int it = 0; it < dv->nu_aux; ++it) b_sweep<NR, T>(dv, L, b, false, false, done, s);
}

// z = B_co r for every system; r (FP64, internal) -> fine.x (precision T)
template <int NR, class T>
static void b_apply(BatchDevice *dv, const double *r, const int *done, hipStream_t s) {
  BLevel &F = dv->fine;
  const T *b;
  if constexpr (sizeof(T) == 8) {
    b = r;
  } else {
    hipLaunchKernelGGL((kb_cvt<NR>), dim3(nblk((int64_t)F.nrows * NR)), dim3(BS), 0, s, F.nrows, r, F.b32, done);
    b = F.b32;
  }
  for (int it = 0; it < dv->nu_fine; ++it) b_sweep<NR, T>(dv, F, b, it == 0, true, done, s);
  b_residual<NR, T>(dv, F, b, done, s);
  b_spmv<NR, 0, T>(dv, dv->PiT, BV<T>::r(F), BV<T>::b(dv->aux[0]), done, s);
  b_vcycle<NR, T>(dv, 0, done, s);
  b_spmv<NR, 1, T>(dv, dv->Pi, BV<T>::x(dv->aux[0]), BV<T>::x(F), done, s);
  for (int it = 0; it < dv->nu_fine; ++it) b_sweep<NR, T>(dv, F, b, false, false, done, s);
}

template <int NR, class T>
static void b_tail(BatchDevice *dv, hipStream_t s) {
  const SegTable &E = dv->fine_ew;
  b_apply<NR, T>(dv, dv->r, dv->ctl.gdone, s);
  const T *z = BV<T>::x(dv->fine);
  hipLaunchKernelGGL((kb_cg_rz<NR, T>), dim3(E.nblocks), dim3(BS), 0, s, E.r0, E.r1, E.b0, E.nseg, dv->r, z, dv->ctl,
                     dv->partials);
  hipLaunchKernelGGL((kb_fin_rz<NR>), dim3(dv->nm), dim3(BS), 0, s, E.b0, dv->partials, dv->ctl);
  hipLaunchKernelGGL((kb_cg_p<NR, T>), dim3(E.nblocks), dim3(BS), 0, s, E.r0, E.r1, E.b0, E.nseg, z, dv->p, dv->ctl);
}

template <int NR, class T>
static void b_iteration(BatchDevice *dv, hipStream_t s) {
  BLevel &F = dv->fine;
  const SegTable &Sp = dv->fine_sp, &E = dv->fine_ew;
  with_lpr(F.A.lpr, [&](auto cc) {
    constexpr int LP = decltype(cc)::value;
    hipLaunchKernelGGL((kb_cg_spmv<LP, NR>), dim3(Sp.nblocks), dim3(BS), 0, s, Sp.r0, Sp.r1, Sp.b0, Sp.nseg, F.A.rp,
                       F.A.ci, F.A.v64, F.dg64, dv->p, dv->q, dv->ctl, dv->partials);
  });
  hipLaunchKernelGGL((kb_fin_spmv<NR>), dim3(dv->nm), dim3(BS), 0, s, Sp.b0, dv->partials, dv->ctl);
  hipLaunchKernelGGL((kb_cg_axpy<NR>), dim3(E.nblocks), dim3(BS), 0, s, E.r0, E.r1, E.b0, E.nseg, dv->u, dv->r, dv->p,
                     dv->q, dv->ctl, dv->partials);
  hipLaunchKernelGGL((kb_fin_axpy<NR>), dim3(dv->nm), dim3(BS), 0, s, E.b0, dv->partials, dv->ctl);
  b_tail<NR, T>(dv, s);
}

template <int NR, class T>
static void b_launch_iterations(BatchDevice *dv, int count, hipStream_t s) {
  const int pi = sizeof(T) == 4 ? 1 : 0;
  if (dv->use_graph && !dv->graph[pi][NR]) {
    hipGraph_t g;
    HIPCHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    b_iteration<NR, T>(dv, s);
    HIPCHECK(hipStreamEndCapture(s, &g));
    HIPCHECK(hipGraphInstantiate(&dv->graph[pi][NR], g, nullptr, nullptr, 0));
    HIPCHECK(hipGraphDestroy(g));
  }
  for (int i = 0; i < count; ++i) {
    if (dv->use_graph)
      HIPCHECK(hipGraphLaunch(dv->graph[pi][NR], s));
    else
      b_iteration<NR, T>(dv, s);
  }
}

template <int NR, class T>
static int b_pcg(BatchDevice *dv, double tol, int *iters, double *true_rel, hipStream_t s) {
  const int pi = sizeof(T) == 4 ? 1 : 0;
  const int nm = dv->nm, ns = nm * NR;
  const SegTable &E = dv->fine_ew, &Sp = dv->fine_sp;
  BLevel &F = dv->fine;
  // per-system ints (4 arrays sized for 4 right-hand sides), mesh tickets, active count, done flag
  HIPCHECK(hipMemsetAsync(dv->ctl_ints, 0, ((size_t)nm * 4 * 4 + nm + 2) * sizeof(int), s));
  hipLaunchKernelGGL((kb_cg_init<NR>), dim3(E.nblocks), dim3(BS), 0, s, E.r0, E.r1, E.b0, E.nseg, dv->f, dv->r, dv->u,
                     dv->p, dv->partials);
  hipLaunchKernelGGL((kb_fin_init<NR>), dim3(nm), dim3(BS), 0, s, E.b0, dv->partials, tol, dv->ctl);
  int hst[2];
  HIPCHECK(hipMemcpyAsync(hst, dv->ctl.active, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  if (hst[0] == 0) HIPCHECK(hipMemcpyAsync(dv->ctl.gdone, &(hst[1] = 1), sizeof(int), hipMemcpyHostToDevice, s));
  b_tail<NR, T>(dv, s);
  const int first = dv->last_iters[pi][NR] > 1 ? dv->last_iters[pi][NR] - 1 : 0;
  if (first > 0) b_launch_iterations<NR, T>(dv, std::min(first, dv->maxit), s);
  const int Kc = dv->last_iters[pi][NR] > 0 ? 1 : 4;
  std::vector<int> mask(ns);
  int restarts = 0;
  std::vector<double> tr(ns), fn2(ns);
  std::vector<int> st(ns), it(ns);
  while (true) {
    int gd = 0;
    HIPCHECK(hipMemcpyAsync(&gd, dv->ctl.gdone, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    if (!gd) {
      b_launch_iterations<NR, T>(dv, Kc, s);
      continue;
    }
    with_lpr(F.A.lpr, [&](auto cc) {
      constexpr int LP = decltype(cc)::value;
      hipLaunchKernelGGL((kb_true_res<LP, NR>), dim3(Sp.nblocks), dim3(BS), 0, s, Sp.r0, Sp.r1, Sp.b0, Sp.nseg,
                         F.A.rp, F.A.ci, F.A.v64, F.dg64, dv->f, dv->u, dv->partials);
    });
    hipLaunchKernelGGL((kb_fin_tr<NR>), dim3(nm), dim3(BS), 0, s, Sp.b0, dv->partials, dv->ctl);
    HIPCHECK(hipMemcpyAsync(tr.data(), dv->ctl.tr, ns * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipMemcpyAsync(fn2.data(), dv->ctl.fn2, ns * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipMemcpyAsync(st.data(), dv->ctl.status, ns * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipMemcpyAsync(it.data(), dv->ctl.iter, ns * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    int nre = 0;
    for (int i = 0; i < ns; ++i) {
      const double rel = fn2[i] > 0 ? std::sqrt(tr[i] / fn2[i]) : 0.0;
      mask[i] = (sizeof(T) == 4 && st[i] == BST_OK && fn2[i] > 0 && rel > tol && it[i] < dv->maxit) ? 1 : 0;
      nre += mask[i];
    }
    if (nre > 0 && restarts < 3) {
      ++restarts;
      HIPCHECK(hipMemcpyAsync(dv->mask, mask.data(), ns * sizeof(int), hipMemcpyHostToDevice, s));
      with_lpr(F.A.lpr, [&](auto cc) {
        constexpr int LP = decltype(cc)::value;
        hipLaunchKernelGGL((kb_restart<LP, NR>), dim3(Sp.nblocks), dim3(BS), 0, s, Sp.r0, Sp.r1, Sp.b0, Sp.nseg,
                           F.A.rp, F.A.ci, F.A.v64, F.dg64, dv->f, dv->u, dv->r, dv->p, dv->mask);
      });
      // reopen the restarted systems: done = 0, first = 1, active = count, gdone = 0
      std::vector<int> dn(ns), fi(ns);
      HIPCHECK(hipMemcpyAsync(dn.data(), dv->ctl.dn, ns * sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHECK(hipMemcpyAsync(fi.data(), dv->ctl.first, ns * sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHECK(hipStreamSynchronize(s));
      for (int i = 0; i < ns; ++i)
        if (mask[i]) {
          dn[i] = 0;
          fi[i] = 1;
        }
      int two[2] = {nre, 0};
      HIPCHECK(hipMemcpyAsync(dv->ctl.dn, dn.data(), ns * sizeof(int), hipMemcpyHostToDevice, s));
      HIPCHECK(hipMemcpyAsync(dv->ctl.first, fi.data(), ns * sizeof(int), hipMemcpyHostToDevice, s));
      HIPCHECK(hipMemcpyAsync(dv->ctl.active, two, 2 * sizeof(int), hipMemcpyHostToDevice, s));
      HIPCHECK(hipStreamSynchronize(s));
      b_tail<NR, T>(dv, s);
      continue;
    }
    int rc = ASMG_OK, maxit = 0;
    for (int i = 0; i < ns; ++i) {
      if (iters) iters[i] = it[i];
      if (true_rel) true_rel[i] = fn2[i] > 0 ? std::sqrt(tr[i] / fn2[i]) : 0.0;
      maxit = std::max(maxit, it[i]);
      if (st[i] == BST_NOTSPD) rc = ASMG_ENOTSPD;
      if (st[i] == BST_NAN && rc == ASMG_OK) rc = ASMG_ENAN;
      if (st[i] == BST_NOCONV && rc == ASMG_OK) rc = ASMG_ENOCONV;
    }
    if (rc == ASMG_OK) dv->last_iters[pi][NR] = maxit;
    return rc;
  }
}

template <int NR>
static int b_solve_nr(BatchDevice *dv, const double *d_F, double tol, double *d_U, int *iters, double *true_rel,
                      hipStream_t cs) {
  hipStream_t s = dv->stream;
  const int n = dv->fine.nrows;
  HIPCHECK(hipEventRecord(dv->ev_in, cs));
  HIPCHECK(hipStreamWaitEvent(s, dv->ev_in, 0));
  hipLaunchKernelGGL((kb_gather<NR>), dim3(nblk(n)), dim3(BS), 0, s, n, dv->row_src0[NR], dv->row_stride, d_F, dv->f);
  const int rc = dv->precision == ASMG_PREC_MIXED ? b_pcg<NR, float>(dv, tol, iters, true_rel, s)
                                                   : b_pcg<NR, double>(dv, tol, iters, true_rel, s);
  hipLaunchKernelGGL((kb_scatter<NR>), dim3(nblk(n)), dim3(BS), 0, s, n, dv->row_src0[NR], dv->row_stride, dv->u, d_U);
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipEventRecord(dv->ev_out, s));
  HIPCHECK(hipStreamWaitEvent(cs, dv->ev_out, 0));
  HIPCHECK(hipStreamSynchronize(s));
  return rc;
}

int batch_device_solve(BatchDevice *dv, int n_rhs, const double *d_F, double tol, double *d_U, int *iters,
                       double *true_rel, void *stream) {
  HIPCHECK(hipSetDevice(dv->ordinal));
  hipStream_t cs = (hipStream_t)stream;
  switch (n_rhs) {
    case 1: return b_solve_nr<1>(dv, d_F, tol, d_U, iters, true_rel, cs);
    case 2: return b_solve_nr<2>(dv, d_F, tol, d_U, iters, true_rel, cs);
    case 4: return b_solve_nr<4>(dv, d_F, tol, d_U, iters, true_rel, cs);
    default: throw AsmgError{ASMG_EINVAL, "n_rhs must be 1, 2 or 4"};
  }
}

int batch_device_time(BatchDevice *dv, int n_rhs, int reps, int precision, void *stream, double *ms, double *bytes) {
  HIPCHECK(hipSetDevice(dv->ordinal));
  hipStream_t s = (hipStream_t)stream;
  auto one = [&]() {
    const bool mixed = precision == ASMG_PREC_MIXED;
    switch (n_rhs) {
      case 1: mixed ? b_apply<1, float>(dv, dv->f, dv->ctl.gdone + 1, s) : b_apply<1, double>(dv, dv->f, dv->ctl.gdone + 1, s); break;
      case 2: mixed ? b_apply<2, float>(dv, dv->f, dv->ctl.gdone + 1, s) : b_apply<2, double>(dv, dv->f, dv->ctl.gdone + 1, s); break;
      default: mixed ? b_apply<4, float>(dv, dv->f, dv->ctl.gdone + 1, s) : b_apply<4, double>(dv, dv->f, dv->ctl.gdone + 1, s); break;
    }
  };
  HIPCHECK(hipMemsetAsync(dv->f, 0, (size_t)dv->fine.nrows * 4 * sizeof(double), s));
  dv->count_bytes = true;
  dv->bytes = 0;
  one();
  dv->count_bytes = false;
  *bytes = dv->bytes;
  hipEvent_t e0, e1;
  HIPCHECK(hipEventCreate(&e0));
  HIPCHECK(hipEventCreate(&e1));
  HIPCHECK(hipEventRecord(e0, s));
  for (int k = 0; k < reps; ++k) one();
  HIPCHECK(hipEventRecord(e1, s));
  HIPCHECK(hipEventSynchronize(e1));
  float t = 0;
  HIPCHECK(hipEventElapsedTime(&t, e0, e1));
  *ms = (double)t / reps;
  HIPCHECK(hipEventDestroy(e0));
  HIPCHECK(hipEventDestroy(e1));
  return ASMG_OK;
}

int64_t batch_n_total(BatchDevice *dv) { return dv->dof_off.back(); }

}  // namespace asmg
