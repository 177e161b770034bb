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
#include <climits>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>
#include <thread>
#include <vector>

#include "batch.hpp"
#include "common.hpp"
#include "host_parallel.hpp"
#include "trace.hpp"

namespace asmg {

#ifndef LOWER_FIRST_SWEEP
#define LOWER_FIRST_SWEEP 1
#endif
#ifndef UPPER_RESIDUAL
#define UPPER_RESIDUAL 1
#endif

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

// ----------------------------------------------------------------------------
// sliced ELL over NR interleaved right-hand sides
//
// Layout as in the single-mesh engine: 64 rows per slice (one wave, one row per lane), entry k
// of slice s and lane j at soff[s] + 64 k + j, padding entries repeat a column of the lane's
// row with value 0, srow = -1 marks empty lanes. A wave's slice width w is uniform, so each
// width has straight-line code that issues every column and value load of the row, then the
// row's own loads (`pre`), then the NR-wide gathers of x, then calls `post` with the NR sums.
// ----------------------------------------------------------------------------

template <class T>
__device__ __forceinline__ void bpin(T &v) {
  asm volatile("" : "+v"(v));
}

// MASK 1: only the entries with a column above `urow` (the row's later colours) are gathered and
// added; MASK 2: only those with a column below it (its earlier colours); MASK 0: every entry
template <int W, int NR, int MASK = 0, class T, class Pre, class Post>
__device__ __forceinline__ void bsell_row_w(const int *__restrict__ cp, const T *__restrict__ vp,
                                            const T *__restrict__ x, Pre &pre, Post &post, int urow = 0) {
  const VecR<NR, T> *X = reinterpret_cast<const VecR<NR, T> *>(x);
  int c[W];
  T v[W];
  if constexpr (std::is_same<T, float>::value) {
    // FP32: nontemporal matrix loads, as in the single-mesh row products (batched mixed solve
    // 185 -> 183 ms; FP64 unchanged, so it keeps plain loads)
#pragma unroll
    for (int k = 0; k < W; ++k) c[k] = __builtin_nontemporal_load(cp + k * 64);
#pragma unroll
    for (int k = 0; k < W; ++k) v[k] = __builtin_nontemporal_load(vp + k * 64);
  } else {
#pragma unroll
    for (int k = 0; k < W; ++k) c[k] = cp[k * 64];
#pragma unroll
    for (int k = 0; k < W; ++k) v[k] = vp[k * 64];
  }
  pre();
  T a0[NR], a1[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) a0[r] = a1[r] = 0;
#pragma unroll
  for (int k = 0; k < W; ++k) {
    if ((MASK == 1 && c[k] <= urow) || (MASK == 2 && c[k] >= urow)) continue;
    const VecR<NR, T> xv = X[c[k]];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (k & 1)
        a1[r] += v[k] * xv.v[r];
      else
        a0[r] += v[k] * xv.v[r];
    }
  }
  T acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    acc[r] = a0[r] + a1[r];
    bpin(acc[r]);
  }
  post(acc);
}

template <int NR, int MASK, class T>
__device__ __forceinline__ void bsell_chunk(const int *__restrict__ cp, const T *__restrict__ vp,
                                            const T *__restrict__ x, T acc[NR], int urow) {
  auto pre = [] {};
  auto post = [&](T a[NR]) {
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] += a[r];
  };
  bsell_row_w<8, NR, MASK>(cp, vp, x, pre, post, urow);
}

template <int NR, class T, int MASK = 0, class Pre, class Post>
__device__ __forceinline__ void bsell_row(int w, const int *__restrict__ cp, const T *__restrict__ vp,
                                          const T *__restrict__ x, Pre &pre, Post &post, int urow = 0) {
  switch (w) {
    case 0: {
      pre();
      T z[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) z[r] = 0;
      post(z);
      break;
    }
    case 1: bsell_row_w<1, NR, MASK>(cp, vp, x, pre, post, urow); break;
    case 2: bsell_row_w<2, NR, MASK>(cp, vp, x, pre, post, urow); break;
    case 3: bsell_row_w<3, NR, MASK>(cp, vp, x, pre, post, urow); break;
    case 4: bsell_row_w<4, NR, MASK>(cp, vp, x, pre, post, urow); break;
    case 5: bsell_row_w<5, NR, MASK>(cp, vp, x, pre, post, urow); break;
    case 6: bsell_row_w<6, NR, MASK>(cp, vp, x, pre, post, urow); break;
    case 7: bsell_row_w<7, NR, MASK>(cp, vp, x, pre, post, urow); break;
    case 8: bsell_row_w<8, NR, MASK>(cp, vp, x, pre, post, urow); break;
    case 9: bsell_row_w<9, NR, MASK>(cp, vp, x, pre, post, urow); break;
    case 10: bsell_row_w<10, NR, MASK>(cp, vp, x, pre, post, urow); break;
    case 11: bsell_row_w<11, NR, MASK>(cp, vp, x, pre, post, urow); break;
    case 12: bsell_row_w<12, NR, MASK>(cp, vp, x, pre, post, urow); break;
    default: {
      // long rows: chunks of 8 entries, each with its loads issued together
      pre();
      const VecR<NR, T> *X = reinterpret_cast<const VecR<NR, T> *>(x);
      T acc[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) acc[r] = 0;
      int k = 0;
      for (; k + 8 <= w; k += 8) bsell_chunk<NR, MASK>(cp + k * 64, vp + k * 64, x, acc, urow);
      for (; k < w; ++k) {
        const int ck = cp[k * 64];
        if ((MASK == 1 && ck <= urow) || (MASK == 2 && ck >= urow)) continue;
        const T a = vp[k * 64];
        const VecR<NR, T> xv = X[ck];
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[r] += a * xv.v[r];
      }
      post(acc);
    }
  }
}

__device__ __forceinline__ int bwave_slice(int first) {
  return first + xcd_block() * (BS / 64) + __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
}

// MODE 0: Gauss-Seidel colour pass x_i = (b_i - sum_{j != i} a_ij x_j) / a_ii (dv_ = 1/a_ii)
// MODE 1: residual r_i = b_i - a_ii x_i - sum_{j != i} a_ij x_j (dv_ = a_ii)
// MODE 2: residual right after a single forward sweep from x = 0, r_i = -sum_{j > i} a_ij x_j:
// when row i's colour was solved its later colours were zero and its earlier ones final, so only
// the later colours' terms remain (each mesh numbers its rows colour by colour). Slice s starts
// at shi[s] (passed as soff); b, dv_ and x at the row are not read.
// MODE 3: the Gauss-Seidel pass of MODE 0 in a sweep from x = 0, reading only each row's earlier
// colours (columns below the row; slices end at slo[s], passed as send). The later colours are
// zero at that point in exact terms but are not read, so x need not be cleared beforehand.
// over slices [s0, s1), every right-hand side of a row at once
template <int MODE, int NR, class T, int VAR = 0>
__global__ __launch_bounds__(BS_MAX) void kb_sell(int s0, int s1, const int *__restrict__ srow,
                                                  const int *__restrict__ soff, const int *__restrict__ send,
                                                  const int *__restrict__ scol,
                                                  const T *__restrict__ sv, const T *__restrict__ dv_,
                                                  const T *__restrict__ b, T *__restrict__ x, T *__restrict__ r,
                                                  int shape) {
  const int lane = threadIdx.x & 63;
  for_slices<VAR>(s0, s1, shape, srow, soff, send, [&](int row, int o0, int w) {
    VecR<NR, T> bv, xv;
    T di = 0;
    auto pre = [&] {
      if (MODE == 2) return;
      const int rr = row < 0 ? 0 : row;
      bv = reinterpret_cast<const VecR<NR, T> *>(b)[rr];
      di = dv_[rr];
      if (MODE == 1) xv = reinterpret_cast<const VecR<NR, T> *>(x)[rr];
    };
    auto post = [&](T acc[NR]) {
      if (MODE != 2) {
#pragma unroll
        for (int q = 0; q < NR; ++q) bpin(bv.v[q]);
        bpin(di);
      }
      if (row < 0) return;
      VecR<NR, T> o;
#pragma unroll
      for (int q = 0; q < NR; ++q)
        o.v[q] = MODE == 0 || MODE == 3 ? (bv.v[q] - acc[q]) * di
                 : MODE == 1           ? bv.v[q] - di * xv.v[q] - acc[q]
                                       : -acc[q];
      reinterpret_cast<VecR<NR, T> *>(MODE == 0 || MODE == 3 ? x : r)[row] = o;
    };
    bsell_row<NR, T, MODE == 2 ? 1 : MODE == 3 ? 2 : 0>(w, scol + o0 + lane, sv + o0 + lane, x, pre, post, row);
  });
}

// transfer product y = A x (ADD 0) or y += A x (ADD 1). FIRST (ADD 0): y is the right-hand side
// of a level whose smoothing starts from zero; the kernel also runs its first colour pass,
// xs_i = y_i * id0_i on the colour-0 rows of their mesh (id0_i = 1/a_ii there, 0 elsewhere).
// The other rows of xs are left as they are: the sweep's later passes read only earlier colours
// (kb_sell MODE 3), and each of them writes its own rows.
template <int ADD, int FIRST, int NR, class T, int VAR = 0>
__global__ __launch_bounds__(BS_MAX) void kb_sell_spmv(int ns, const int *__restrict__ srow,
                                                       const int *__restrict__ soff, const int *__restrict__ scol,
                                                       const T *__restrict__ sv, const T *__restrict__ x,
                                                       T *__restrict__ y, const T *__restrict__ id0,
                                                       T *__restrict__ xs, int shape) {
  const int lane = threadIdx.x & 63;
  for_slices<VAR>(0, ns, shape, srow, soff, soff + 1, [&](int row, int o0, int w) {
    VecR<NR, T> yv;
    T di = 0;
    auto pre = [&] {
      const int rr = row < 0 ? 0 : row;
      if (ADD) yv = reinterpret_cast<const VecR<NR, T> *>(y)[rr];
      if (FIRST) di = id0[rr];
    };
    auto post = [&](T acc[NR]) {
      if (ADD)
#pragma unroll
        for (int q = 0; q < NR; ++q) bpin(yv.v[q]);
      if (FIRST) bpin(di);
      if (row < 0) return;
      VecR<NR, T> o, f;
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        o.v[q] = ADD ? yv.v[q] + acc[q] : acc[q];
        f.v[q] = acc[q] * di;
      }
      reinterpret_cast<VecR<NR, T> *>(y)[row] = o;
      if (FIRST && di != T(0)) reinterpret_cast<VecR<NR, T> *>(xs)[row] = f;
    };
    bsell_row<NR, T>(w, scol + o0 + lane, sv + o0 + lane, x, pre, post);
  });
}

// first colour pass of a sweep from zero on its own: x_i = b_i * id0_i on colour 0 (other rows
// are written by the later passes, which do not read them before)
template <int NR, class T>
__global__ __launch_bounds__(BS) void kb_first(int n, const T *__restrict__ b, const T *__restrict__ id0,
                                               T *__restrict__ x) {
  const int i = blockIdx.x * BS + threadIdx.x;
  if (i >= n) return;
  const T d = id0[i];
  if (d == T(0)) return;
  const VecR<NR, T> bv = reinterpret_cast<const VecR<NR, T> *>(b)[i];
  VecR<NR, T> o;
#pragma unroll
  for (int q = 0; q < NR; ++q) o.v[q] = bv.v[q] * d;
  reinterpret_cast<VecR<NR, T> *>(x)[i] = o;
}

// mixed precision: the same pass on the original grid, which also rounds the FP64 residual to FP32
template <int NR>
__global__ __launch_bounds__(BS) void kb_first_cvt(int n, const double *__restrict__ r, const float *__restrict__ id0,
                                                   float *__restrict__ b32, float *__restrict__ x) {
  const int i = blockIdx.x * BS + threadIdx.x;
  if (i >= n) return;
  const float d = id0[i];
  VecR<NR, float> bo, o;
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    bo.v[q] = (float)r[(size_t)i * NR + q];
    o.v[q] = bo.v[q] * d;
  }
  reinterpret_cast<VecR<NR, float> *>(b32)[i] = bo;
  if (d != 0.0f) reinterpret_cast<VecR<NR, float> *>(x)[i] = o;
}

// bottom solves of the meshes whose V-cycle ends on this level: y = M_m g. A wave computes
// kGemvRows consecutive rows of one mesh, so that each gathered g entry (NR values) serves all of
// them: per row the wave streams n entries of M from HBM and n / kGemvRows entries of g from L2
// (one row per wave read g once per row, four times the bytes of M with four right-hand sides).
constexpr int kGemvRows = 4;

template <int NR, class T>
__global__ __launch_bounds__(BS) void kb_gemv(const int *__restrict__ wavepref, int nb, const int *__restrict__ nc,
                                              const int64_t *__restrict__ moff, const int *__restrict__ voff,
                                              const T *__restrict__ M, const T *__restrict__ g, T *__restrict__ y) {
  const int w = blockIdx.x * (BS / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (w >= wavepref[nb]) return;  // whole wave leaves together
  const int s = find_seg(wavepref, nb, w);
  const int n = nc[s];
  const int i0 = (w - wavepref[s]) * kGemvRows;
  const int nr = min(kGemvRows, n - i0);
  const T *m = M + moff[s] + (int64_t)i0 * n;
  const VecR<NR, T> *G = reinterpret_cast<const VecR<NR, T> *>(g) + voff[s];
  T acc[kGemvRows][NR];
#pragma unroll
  for (int k = 0; k < kGemvRows; ++k)
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[k][r] = 0;
  for (int j = lane; j < n; j += 64) {
    const VecR<NR, T> gv = G[j];
#pragma unroll
    for (int k = 0; k < kGemvRows; ++k) {
      const T a = k < nr ? m[(int64_t)k * n + j] : T(0);
#pragma unroll
      for (int r = 0; r < NR; ++r) acc[k][r] += a * gv.v[r];
    }
  }
#pragma unroll
  for (int k = 0; k < kGemvRows; ++k)
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[k][r] = group_sum<64>(acc[k][r]);
  if (lane < nr) {
    VecR<NR, T> o;
#pragma unroll
    for (int k = 0; k < kGemvRows; ++k)
      if (k == lane)
#pragma unroll
        for (int r = 0; r < NR; ++r) o.v[r] = acc[k][r];
    reinterpret_cast<VecR<NR, T> *>(y)[voff[s] + i0 + lane] = o;
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

// block sums of the NR values into partials[blk] (blk = the block's logical index)
template <int NR>
__device__ __forceinline__ void bwrite(double v[NR], double *partials, int blk) {
  block_sum_n<NR>(v);
  if (threadIdx.x == 0)
#pragma unroll
    for (int r = 0; r < NR; ++r) partials[(size_t)blk * NR + r] = v[r];
}

template <int NR>
__device__ __forceinline__ void bwrite(double v[NR], double *partials) {
  bwrite<NR>(v, partials, (int)blockIdx.x);
}

template <int NR>
__device__ __forceinline__ void breduce(const double *partials, int b0, int b1, double out[NR]) {
  double s[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) s[r] = 0;
  for (int b = b0 + (int)threadIdx.x; b < b1; b += BS)
#pragma unroll
    for (int r = 0; r < NR; ++r) s[r] += partials[(size_t)b * NR + r];
  block_sum_n<NR>(s);
#pragma unroll
  for (int r = 0; r < NR; ++r) out[r] = s[r];
}

__device__ __forceinline__ void bretire(BCtl c, int sys, int status) {
  c.dn[sys] = 1;
  c.status[sys] = status;
  const int prev = atomicSub(c.active, 1);
  if (prev == 1) *c.gdone = 1;
}

// Element-wise CG kernels run one block per (mesh, 256-row chunk): block b covers rows
// [ew_r0[b], ew_r1[b]) of mesh ew_m[b], and the blocks of a mesh are contiguous.
template <int NR>
__global__ __launch_bounds__(BS) void kb_cg_init(const int *__restrict__ ew_r0, const int *__restrict__ ew_r1,
                                                 const double *__restrict__ f, double *__restrict__ r,
                                                 double *__restrict__ u, double *__restrict__ p, double *partials) {
  using V = VecR<NR, double>;
  const int row = ew_r0[blockIdx.x] + threadIdx.x;
  double v[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) v[q] = 0;
  if (row < ew_r1[blockIdx.x]) {
    const V fv = reinterpret_cast<const V *>(f)[row];
    V z;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      z.v[q] = 0.0;
      v[q] = fv.v[q] * fv.v[q];
    }
    reinterpret_cast<V *>(r)[row] = fv;
    reinterpret_cast<V *>(u)[row] = z;
    reinterpret_cast<V *>(p)[row] = z;
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

// q = A p over the mesh-major sliced ELL of the original grids (each mesh padded to whole
// blocks of 4 slices, so no block straddles two meshes); partials of p.q per block
template <int NR>
__global__ __launch_bounds__(BS) void kb_cg_spmv(const int *__restrict__ srow, const int *__restrict__ soff,
                                                 const int *__restrict__ scol, const double *__restrict__ sv,
                                                 const double *__restrict__ dg, const double *__restrict__ p,
                                                 double *__restrict__ q, BCtl c, double *partials) {
  if (*c.gdone) return;
  const int s = bwave_slice(0);
  const int lane = threadIdx.x & 63;
  const int row = srow[(size_t)s * 64 + lane];
  const int o0 = soff[s];
  const int w = (soff[s + 1] - o0) >> 6;
  double v[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) v[k] = 0;
  VecR<NR, double> pv;
  double di = 0;
  auto pre = [&] {
    const int rr = row < 0 ? 0 : row;
    pv = reinterpret_cast<const VecR<NR, double> *>(p)[rr];
    di = dg[rr];
  };
  auto post = [&](double acc[NR]) {
#pragma unroll
    for (int k = 0; k < NR; ++k) bpin(pv.v[k]);
    bpin(di);
    if (row < 0) return;
    VecR<NR, double> o;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      o.v[k] = di * pv.v[k] + acc[k];
      v[k] = pv.v[k] * o.v[k];
    }
    reinterpret_cast<VecR<NR, double> *>(q)[row] = o;
  };
  bsell_row<NR, double>(w, scol + o0 + lane, sv + o0 + lane, p, pre, post);
  bwrite<NR>(v, partials, xcd_block());  // the logical block of this block's slices
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

// u += alpha p, r -= alpha q per system; partials of ||r||^2. The same pass runs the first
// colour pass of the next B_co on the new r in precision T: xf = r * id0 on colour 0 (the other
// rows of xf are written by the sweep's later passes), and in FP32 also bf = (float) r.
template <int NR, class T>
__global__ __launch_bounds__(BS) void kb_cg_axpy(const int *__restrict__ ew_m, const int *__restrict__ ew_r0,
                                                 const int *__restrict__ ew_r1, double *__restrict__ u,
                                                 double *__restrict__ r, const double *__restrict__ p,
                                                 const double *__restrict__ q, BCtl c, double *partials,
                                                 const T *__restrict__ id0, T *__restrict__ bf, T *__restrict__ xf) {
  if (*c.gdone) return;
  using V = VecR<NR, double>;
  const int m = ew_m[blockIdx.x];
  const int row = ew_r0[blockIdx.x] + threadIdx.x;
  const bool act = row < ew_r1[blockIdx.x];
  double v[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) v[k] = 0;
  if (act) {
    const V al = reinterpret_cast<const V *>(c.alpha)[m];
    const VecR<NR, int> dn = reinterpret_cast<const VecR<NR, int> *>(c.dn)[m];
    const T d = id0[row];
    V uv = reinterpret_cast<const V *>(u)[row];
    V rv = reinterpret_cast<const V *>(r)[row];
    const V pv = reinterpret_cast<const V *>(p)[row];
    const V qv = reinterpret_cast<const V *>(q)[row];
    VecR<NR, T> bo, xo;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      if (!dn.v[k]) {
        uv.v[k] += al.v[k] * pv.v[k];
        rv.v[k] = rv.v[k] - al.v[k] * qv.v[k];
        v[k] = rv.v[k] * rv.v[k];
      }
      bo.v[k] = (T)rv.v[k];
      xo.v[k] = bo.v[k] * d;
    }
    reinterpret_cast<V *>(u)[row] = uv;
    reinterpret_cast<V *>(r)[row] = rv;
    if constexpr (sizeof(T) == 4) reinterpret_cast<VecR<NR, T> *>(bf)[row] = bo;
    if (d != T(0)) reinterpret_cast<VecR<NR, T> *>(xf)[row] = xo;  // colour 0 only, as kb_first
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
__global__ __launch_bounds__(BS) void kb_cg_rz(const int *__restrict__ ew_r0, const int *__restrict__ ew_r1,
                                               const double *__restrict__ r, const T *__restrict__ z, BCtl c,
                                               double *partials) {
  if (*c.gdone) return;
  const int row = ew_r0[blockIdx.x] + threadIdx.x;
  double v[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) v[k] = 0;
  if (row < ew_r1[blockIdx.x]) {
    const VecR<NR, double> rv = reinterpret_cast<const VecR<NR, double> *>(r)[row];
    const VecR<NR, T> zv = reinterpret_cast<const VecR<NR, T> *>(z)[row];
#pragma unroll
    for (int k = 0; k < NR; ++k) v[k] = rv.v[k] * (double)zv.v[k];
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
__global__ __launch_bounds__(BS) void kb_cg_p(const int *__restrict__ ew_m, const int *__restrict__ ew_r0,
                                              const int *__restrict__ ew_r1, const T *__restrict__ z,
                                              double *__restrict__ p, BCtl c) {
  if (*c.gdone) return;
  using V = VecR<NR, double>;
  const int m = ew_m[blockIdx.x];
  const int row = ew_r0[blockIdx.x] + threadIdx.x;
  if (row >= ew_r1[blockIdx.x]) return;
  const V be = reinterpret_cast<const V *>(c.beta)[m];
  const VecR<NR, int> dn = reinterpret_cast<const VecR<NR, int> *>(c.dn)[m];
  const VecR<NR, T> zv = reinterpret_cast<const VecR<NR, T> *>(z)[row];
  V pv = reinterpret_cast<const V *>(p)[row];
#pragma unroll
  for (int k = 0; k < NR; ++k)
    if (!dn.v[k]) pv.v[k] = (double)zv.v[k] + be.v[k] * pv.v[k];
  reinterpret_cast<V *>(p)[row] = pv;
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

// sliced ELL of a merged matrix; slice groups (colour classes, or meshes) in cslice
struct BSell {
  int nrows = 0, ncols = 0, nslices = 0;
  int64_t nnz = 0, entries = 0;
  std::vector<int> cslice{0};
  int *srow = nullptr, *soff = nullptr, *scol = nullptr;
  int *slo = nullptr;    // per slice: end of its entries before each row's own colour range
  int *shi = nullptr;    // per slice: end of the narrowest such prefix over its rows
  double *sv64 = nullptr;
  float *sv32 = nullptr;
};

struct BLevel {
  int nrows = 0;         // all rows (smoothing meshes, then bottom meshes)
  int nsmooth = 0;       // rows of smoothing meshes (a prefix)
  std::vector<int> mesh; // meshes present; smoothing first
  std::vector<int> off;  // row offset of each present mesh
  BSell sell;            // off-diagonal part of the smoothing rows; group c = colour c of every mesh
  std::vector<int64_t> cnnz, crows, ucols;  // per colour group: nonzeros, rows, distinct columns gathered
  std::vector<int64_t> cnnz_lo, ucols_lo;   // the same over the columns of earlier colours
  std::vector<int64_t> cnnz_up, ucols_up;   // the same over the columns of later colours
  double *dg64 = nullptr, *id64 = nullptr, *id0_64 = nullptr;  // a_ii, 1/a_ii, 1/a_ii on colour 0 else 0
  float *dg32 = nullptr, *id32 = nullptr, *id0_32 = nullptr;
  double *x64 = nullptr, *b64 = nullptr, *r64 = nullptr;
  float *x32 = nullptr, *b32 = nullptr, *r32 = nullptr;
  BSell P, PT;           // P: rows = smoothing rows, cols = rows of level k+1 (as used in B_co:
                         // P without each mesh's last colour rows, P^T without the zero-residual
                         // columns of the last colour group)
  // bottom meshes
  int nbottom = 0;
  int *bt_wavepref = nullptr, *bt_nc = nullptr, *bt_voff = nullptr;  // waves of kb_gemv per mesh (prefix)
  int64_t *bt_moff = nullptr;
  double *inv64 = nullptr;
  float *inv32 = nullptr;
  int bottom_waves = 0;
  double bt_entries = 0, bt_rows = 0;  // byte model: inverse entries, rows of the bottom meshes
};

struct BatchDevice {
  int ordinal = 0, nm = 0, d = 2, nu_aux = 2, nu_fine = 1, maxit = 1000, precision = 0;
  std::vector<void *> allocs;
  std::vector<int64_t> n_m;       // unknowns per mesh
  std::vector<int64_t> dof_off;   // prefix of n_m (user vectors, per rhs block)
  // fine level
  BLevel fine;                    // nsmooth = nrows
  BCsr fineA;                     // CSR of the original grids (true residual, restart)
  SegTable fine_sp;               // per-mesh row-group blocks for the CSR kernels
  BSell cg_sell;                  // mesh-major sliced ELL (whole 4-slice blocks per mesh) for q = A p
  BSell fine_up;                  // the later colours' entries of every row, negated (r = U x after
                                  // a single fine sweep from zero), rows that have any
  int *cg_b0 = nullptr;           // first block of each mesh in cg_sell (nm + 1)
  int ew_blocks = 0;              // element-wise blocks: (mesh, 256-row chunk)
  int *ew_m = nullptr, *ew_r0 = nullptr, *ew_r1 = nullptr, *ew_b0 = nullptr;
  BSell Pi, PiT;
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
  // launch shapes of the V-cycle slice kernels, per (precision, NR) and launch site (the k-th
  // slice-kernel launch of one B_co application), chosen by `tune`
  std::vector<Shape> shape[2][5];  // (threads per block, xcd order, kernel variant)
  std::vector<std::vector<float>> tune_times[2][5];  // autotuner: best ms per site and candidate
  bool tuned[2][5] = {{false}};
  bool tuning = false;
  int site = 0;
  int shape_pi = 0, shape_nr = 1;
  int autotune = 1;
  int r_nr = 0;                        // NR of the last residuals written (0: r all zero)
  int tune_k = 0, tune_live = 0;       // autotuner: candidate under trial, sites seen
  std::vector<hipEvent_t> tune_ev;     // two events per launch site
  std::vector<uint8_t> tune_has;       // site launched something
  // per-launch timing of the Gauss-Seidel colour passes (batch_device_time_kernel)
  bool probe = false;
  std::vector<hipEvent_t> probe_ev;    // pairs (start, stop)
  std::vector<double> probe_bytes;
  size_t probe_used = 0;
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

// Sliced ELL of H over row-range groups: inside a range, windows of 256 rows sorted by length
// (longest first, stable), 64 rows per slice. With `order`, range positions map to rows
// through it (transfer products visit their rows in a spatially coherent order). pad_blocks: every group ends on a whole block of
// 4 slices (at least one block), so blocks never straddle groups; block0 gets the first block
// of each group.
using Groups = std::vector<std::vector<std::pair<int, int>>>;

// host image of a BSell (built on host threads, uploaded afterwards)
struct BSellHost {
  int nrows = 0, ncols = 0;
  int64_t nnz = 0;
  // slo[s]: end of the entries of slice s before each row's own range (the widest such prefix
  // over the lanes; rows store their columns in ascending order); shi[s]: the narrowest one
  std::vector<int> srow, soff{0}, scol, cslice{0}, block0{0}, slo, shi;
  std::vector<double> sv;
  std::vector<float> sv32;
};

static void bsell_host(const HMat &H, const Groups &groups, bool pad_blocks, BSellHost &X,
                       const std::vector<int> *order = nullptr) {
  std::vector<int> &srow = X.srow, &soff = X.soff, &scol = X.scol;
  std::vector<int> idx;
  std::vector<double> &sv = X.sv;
  std::vector<int> *block0 = &X.block0;
  auto len = [&](int r) { return H.rp[r + 1] - H.rp[r]; };
  auto empty_slice = [&]() {
    for (int j = 0; j < 64; ++j) srow.push_back(-1);
    X.slo.push_back(soff.back());
    X.shi.push_back(soff.back());
    soff.push_back(soff.back());
  };
  for (const auto &g : groups) {
    const size_t first = srow.size() / 64;
    for (const auto &rg : g) {
      for (int w0 = rg.first; w0 < rg.second; w0 += 256) {
        const int w1 = std::min(w0 + 256, rg.second);
        idx.resize(w1 - w0);
        std::iota(idx.begin(), idx.end(), w0);
        if (order)
          for (int &i : idx) i = (*order)[i];  // position i of the range holds row order[i]
        std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return len(x) > len(y); });
        for (size_t a = 0; a < idx.size(); a += 64) {
          const size_t e = std::min(a + 64, idx.size());
          int wmax = 0, wlo = 0, whi = INT_MAX;
          for (size_t i = a; i < e; ++i) {
            const int r = idx[i];
            wmax = std::max(wmax, len(r));
            int lo = 0;
            while (lo < len(r) && H.ci[H.rp[r] + lo] < rg.first) ++lo;
            wlo = std::max(wlo, lo);
            whi = std::min(whi, lo);
          }
          const int base = soff.back();
          scol.resize(base + 64 * wmax);
          sv.resize(base + 64 * wmax);
          for (int lane = 0; lane < 64; ++lane) {
            const int row = a + lane < e ? idx[a + lane] : -1;
            srow.push_back(row);
            for (int k = 0; k < wmax; ++k) {
              int cc = 0;  // padding: a valid column with value 0
              double v = 0.0;
              if (row >= 0 && k < len(row)) {
                cc = H.ci[H.rp[row] + k];
                v = H.v[H.rp[row] + k];
              } else if (row >= 0 && len(row) > 0) {
                cc = H.ci[H.rp[row]];
              } else if (a < e && len(idx[a]) > 0) {
                cc = H.ci[H.rp[idx[a]]];  // empty lane: a column of the slice's first row
              }
              scol[base + 64 * k + lane] = cc;
              sv[base + 64 * k + lane] = v;
            }
          }
          soff.push_back(base + 64 * wmax);
          X.slo.push_back(base + 64 * wlo);
          X.shi.push_back(base + 64 * std::min(whi, wmax));
        }
      }
    }
    if (pad_blocks) {
      size_t ns = srow.size() / 64 - first;
      if (ns == 0) {
        empty_slice();
        ns = 1;
      }
      while (ns % (BS / 64)) {
        empty_slice();
        ++ns;
      }
      block0->push_back((int)(srow.size() / 64 / (BS / 64)));
    }
    X.cslice.push_back((int)(srow.size() / 64));
  }
  X.nrows = H.nrows;
  X.ncols = H.ncols;
  X.nnz = (int64_t)H.ci.size();
  X.sv32.assign(sv.begin(), sv.end());
}

static void bsell_upload(BatchDevice *dv, const BSellHost &X, BSell &S) {
  S.cslice = X.cslice;
  S.nrows = X.nrows;
  S.ncols = X.ncols;
  S.nnz = X.nnz;
  S.nslices = (int)(X.srow.size() / 64);
  S.entries = (int64_t)X.sv.size();
  S.srow = bupload(dv, X.srow);
  S.soff = bupload(dv, X.soff);
  S.slo = bupload(dv, X.slo);
  S.shi = bupload(dv, X.shi);
  S.scol = bupload(dv, X.scol);
  S.sv64 = bupload(dv, X.sv);
  S.sv32 = bupload(dv, X.sv32);
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

// colour-major numbering; inside a colour ascending `rank` (the unknown id when rank is null)
static void colour_perm(const std::vector<int32_t> &col, std::vector<int> &perm, std::vector<int> &iperm,
                        std::vector<int> &coff, const std::vector<int> *rank = nullptr) {
  const int n = (int)col.size();
  int C = 0;
  for (int c : col) C = std::max(C, c + 1);
  coff.assign(C + 1, 0);
  for (int c : col) coff[c + 1]++;
  for (int c = 0; c < C; ++c) coff[c + 1] += coff[c];
  perm.resize(n);
  std::vector<int> pos(coff.begin(), coff.end() - 1);
  if (rank) {
    std::vector<int> byrank(n);
    for (int i = 0; i < n; ++i) byrank[(*rank)[i]] = i;
    for (int i : byrank) perm[pos[col[i]]++] = i;
  } else {
    for (int i = 0; i < n; ++i) perm[pos[col[i]]++] = i;
  }
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
  // the residual kernel never writes the rows of the last colour group (zero after a sweep)
  HIPCHECK(hipMemset(L.r64, 0, (size_t)std::max<int64_t>(n, 1) * 8));
  HIPCHECK(hipMemset(L.r32, 0, (size_t)std::max<int64_t>(n, 1) * 4));
}

// a_ii, 1/a_ii and the first-pass scale id0 (1/a_ii on colour-0 rows, 0 elsewhere and on the
// rows of bottom meshes, which have no diagonal entry here) for all nrows rows
static void upload_diag(BatchDevice *dv, BLevel &L, const std::vector<double> &diag,
                        const std::vector<uint8_t> &colour0) {
  const size_t n = std::max<size_t>(L.nrows, diag.size());
  std::vector<double> d(n, 1.0), inv(n, 1.0), i0(n, 0.0);
  for (size_t i = 0; i < diag.size(); ++i) {
    d[i] = diag[i];
    inv[i] = 1.0 / diag[i];
    if (colour0[i]) i0[i] = inv[i];
  }
  std::vector<float> d32(n), i32(n), i032(n, 0.0f);
  for (size_t i = 0; i < n; ++i) {
    d32[i] = (float)d[i];
    i32[i] = i < diag.size() ? 1.0f / (float)diag[i] : 1.0f;
    if (i < diag.size() && colour0[i]) i032[i] = i32[i];
  }
  L.dg64 = bupload(dv, d);
  L.id64 = bupload(dv, inv);
  L.id0_64 = bupload(dv, i0);
  L.dg32 = bupload(dv, d32);
  L.id32 = bupload(dv, i32);
  L.id0_32 = bupload(dv, i032);
}

// Transfers inside B_co. The prolongation x += P e need not write the rows of each mesh's last
// colour: the first backward Gauss-Seidel pass overwrites them without reading them. The
// restriction P^T r need not read the columns where the residual is zero: the last colour group,
// whose rows the residual kernel leaves at zero after a forward sweep.
static std::vector<int> keep_rows(const std::vector<int> &order, const std::vector<uint8_t> &drop) {
  std::vector<int> out;
  out.reserve(order.size());
  for (int i : order) {
    if (i < 0 || i >= (int)drop.size()) throw AsmgError{ASMG_EINVAL, "transfer row outside its matrix"};
    if (!drop[i]) out.push_back(i);
  }
  return out;
}

static HMat drop_cols(const HMat &H, const std::vector<uint8_t> &drop) {
  HMat R;
  R.nrows = H.nrows;
  R.ncols = H.ncols;
  R.rp.assign(H.nrows + 1, 0);
  for (int i = 0; i < H.nrows; ++i) {
    for (int p = H.rp[i]; p < H.rp[i + 1]; ++p)
      if (!drop[H.ci[p]]) {
        R.ci.push_back(H.ci[p]);
        R.v.push_back(H.v[p]);
      }
    R.rp[i + 1] = (int)R.ci.size();
  }
  return R;
}

// byte-model counts of a transfer image: the rows it holds, their nonzeros, the distinct columns
static void transfer_stats(const HMat &H, const std::vector<int> &rows, BSellHost &X) {
  std::vector<uint8_t> seen(std::max(H.ncols, 1), 0);
  int64_t nnz = 0;
  int cols = 0;
  for (int i : rows)
    for (int p = H.rp[i]; p < H.rp[i + 1]; ++p) {
      ++nnz;
      if (!seen[H.ci[p]]) {
        seen[H.ci[p]] = 1;
        ++cols;
      }
    }
  X.nrows = (int)rows.size();
  X.ncols = cols;
  X.nnz = nnz;
}

// byte-model counts of each row-range group of H: nonzeros, rows, and the distinct columns the
// group's rows gather (each x entry read once per colour pass)
struct GroupCounts {
  std::vector<int64_t> cnnz, crows, ucols, cnnz_lo, ucols_lo, cnnz_up, ucols_up;
};

static void group_counts(const HMat &H, const Groups &groups, GroupCounts &K) {
  const int G = (int)groups.size();
  for (auto *v : {&K.cnnz, &K.crows, &K.ucols, &K.cnnz_lo, &K.ucols_lo, &K.cnnz_up, &K.ucols_up}) v->assign(G, 0);
  std::vector<int> seen(std::max(H.ncols, 1), -1);
  for (int g = 0; g < G; ++g)
    for (const auto &rg : groups[g])
      for (int i = rg.first; i < rg.second; ++i) {
        ++K.crows[g];
        for (int p = H.rp[i]; p < H.rp[i + 1]; ++p) {
          // a column of an earlier / a later colour of the row's mesh
          const bool lo = H.ci[p] < rg.first, up = H.ci[p] >= rg.second;
          ++K.cnnz[g];
          K.cnnz_lo[g] += lo;
          K.cnnz_up[g] += up;
          if (seen[H.ci[p]] != g) {
            seen[H.ci[p]] = g;
            ++K.ucols[g];
            K.ucols_lo[g] += lo;
            K.ucols_up[g] += up;
          }
        }
      }
}

static void set_counts(BLevel &L, GroupCounts &&K) {
  L.cnnz = std::move(K.cnnz);
  L.crows = std::move(K.crows);
  L.ucols = std::move(K.ucols);
  L.cnnz_lo = std::move(K.cnnz_lo);
  L.ucols_lo = std::move(K.ucols_lo);
  L.cnnz_up = std::move(K.cnnz_up);
  L.ucols_up = std::move(K.ucols_up);
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
    dv->autotune = H[0]->opt.autotune;
    // per-mesh colour-major orderings of every smoothing level
    struct MeshOrd {
      std::vector<int> perm, iperm, coff;
      std::vector<int> morton;  // original grid: internal rows in Morton order of their vertices
    };
    std::vector<MeshOrd> fine(nm);
    std::vector<std::vector<MeshOrd>> lev(nm);  // index k (aux level J - k), smoothing levels only
    int K = 0;
    dv->n_m.resize(nm);
    dv->dof_off.assign(nm + 1, 0);
    for (int m = 0; m < nm; ++m) {
      Hierarchy &h = *H[m];
      const std::vector<int> mrank = morton_rank(h);
      colour_perm(h.colour_fine, fine[m].perm, fine[m].iperm, fine[m].coff, &mrank);
      fine[m].morton.resize(mrank.size());
      for (size_t i = 0; i < mrank.size(); ++i) fine[m].morton[mrank[i]] = fine[m].iperm[i];
      const int D = h.J - h.lc;
      K = std::max(K, D);
      lev[m].resize(D);
      for (int k = 0; k < D; ++k)
        colour_perm(h.colour_aux.at(h.J - k), lev[m][k].perm, lev[m][k].iperm, lev[m][k].coff);
      dv->n_m[m] = h.n();
      dv->dof_off[m + 1] = dv->dof_off[m] + h.n();
    }
    if (dv->dof_off[nm] * 4 > INT32_MAX) throw AsmgError{ASMG_EINVAL, "batch too large"};
    // ---- row layout of every merged level (sequential, cheap): the fine level is mesh-major;
    // auxiliary level k holds its smoothing meshes, then the meshes whose bottom level it is
    BLevel &F = dv->fine;
    {
      int off = 0;
      for (int m = 0; m < nm; ++m) {
        F.mesh.push_back(m);
        F.off.push_back(off);
        off += (int)H[m]->n();
      }
      F.nrows = F.nsmooth = off;
    }
    dv->aux.resize(K + 1);
    std::vector<std::vector<int>> smooth_m(K + 1), bottom_m(K + 1);
    for (int k = 0; k <= K; ++k) {
      BLevel &L = dv->aux[k];
      for (int m = 0; m < nm; ++m) {
        const int D = H[m]->J - H[m]->lc;
        if (D > k) smooth_m[k].push_back(m);
        if (D == k) bottom_m[k].push_back(m);
      }
      int off = 0;
      for (int m : smooth_m[k]) {
        L.mesh.push_back(m);
        L.off.push_back(off);
        off += (int)H[m]->Al.at(H[m]->J - k).nrows;
      }
      L.nsmooth = off;
      for (int m : bottom_m[k]) {
        L.mesh.push_back(m);
        L.off.push_back(off);
        off += (int)H[m]->nc;
      }
      L.nrows = off;
      L.nbottom = (int)bottom_m[k].size();
    }
    // rows of merged level k in each mesh's own (Morton) numbering: smoothing meshes through their
    // colour permutation, bottom meshes as they are
    auto natural_rows = [&](const BLevel &L, int k) {
      std::vector<int> o;
      o.reserve(L.nrows);
      for (size_t i = 0; i < L.mesh.size(); ++i) {
        const int m = L.mesh[i];
        const int end = i + 1 < L.mesh.size() ? L.off[i + 1] : L.nrows;
        if (H[m]->J - H[m]->lc > k)
          for (int r : lev[m][k].iperm) o.push_back(L.off[i] + r);
        else
          for (int r = L.off[i]; r < end; ++r) o.push_back(r);
      }
      return o;
    };
    // ---- host images of every merged matrix, built on host threads (each task writes only its
    // own stage), then uploaded in a fixed order
    struct LevelImage {
      HMat A;
      std::vector<double> diag;
      std::vector<uint8_t> c0flag;
      BSellHost gs, cg, up;
      GroupCounts counts;  // byte-model counts of every colour group
      // bottom meshes
      std::vector<int> pref{0}, ncs, voff;
      double bt_entries = 0, bt_rows = 0;
      std::vector<int64_t> moff;
      std::vector<double> inv;
      std::vector<float> inv32;
    };
    LevelImage fine_img;
    std::vector<LevelImage> aux_img(K + 1);
    std::vector<BSellHost> p_img(K), pt_img(K);
    BSellHost pi_img, pit_img;
    std::vector<int> r0, r1;
    for (int m = 0; m < nm; ++m) {
      r0.push_back(F.off[m]);
      r1.push_back(F.off[m] + (int)H[m]->n());
    }
    // ---- the merged original-grid matrix and Pi (inputs of several images below)
    HMat Pi;
    BLevel &L0 = dv->aux[0];
    int Cf = 0;  // colours of the original grids (most over the meshes)
    host_parallel(0, 2, [&](int t) {
      if (t == 0) {
        LevelImage &X = fine_img;
        for (int m = 0; m < nm; ++m) {
          append_rows(X.A, H[m]->A, fine[m].perm, &fine[m].iperm, F.off[m], true, &X.diag);
          for (int64_t i = 0; i < H[m]->n(); ++i) X.c0flag.push_back(i < fine[m].coff[1]);
        }
        X.A.ncols = F.nrows;
      } else {
        // Pi (fine rows -> merged level 0 rows)
        for (int m = 0; m < nm; ++m) {
          const int D = H[m]->J - H[m]->lc;
          const size_t j = std::find(L0.mesh.begin(), L0.mesh.end(), m) - L0.mesh.begin();
          const std::vector<int> *cmap = D > 0 ? &lev[m][0].iperm : nullptr;
          append_rows(Pi, H[m]->Pi, fine[m].perm, cmap, L0.off[j], false, nullptr);
        }
        Pi.ncols = L0.nrows;
      }
    });
    for (int m = 0; m < nm; ++m) Cf = std::max(Cf, (int)fine[m].coff.size() - 1);
    // each mesh's original-grid rows in Morton order of their vertices
    std::vector<int> mo;
    mo.reserve(F.nrows);
    for (int m = 0; m < nm; ++m)
      for (int r : fine[m].morton) mo.push_back(F.off[m] + r);
    // the rows of each mesh's last colour, and of the last colour group (meshes with the most
    // colours), on the original grids
    std::vector<uint8_t> last(F.nrows, 0), zero(F.nrows, 0);
    for (int m = 0; m < nm; ++m) {
      const auto &co = fine[m].coff;
      const int Cm = (int)co.size() - 1;
      if (Cm < 1) continue;
      for (int r = F.off[m] + co[Cm - 1]; r < F.off[m] + co[Cm]; ++r) {
        last[r] = 1;
        if (Cm == Cf) zero[r] = 1;
      }
    }
    // tasks: 0-2 the original grids' smoothing, product and residual images, 3-4 Pi and Pi^T,
    // 5..K+5 the auxiliary levels, then the prolongations
    host_parallel(0, 2 * K + 6, [&](int t) {
      if (t == 0) {
        LevelImage &X = fine_img;
        // Gauss-Seidel passes: group c = colour c of every mesh
        Groups groups(Cf);
        for (int c = 0; c < Cf; ++c)
          for (int m = 0; m < nm; ++m) {
            const auto &co = fine[m].coff;
            if (c + 1 < (int)co.size()) groups[c].push_back({F.off[m] + co[c], F.off[m] + co[c + 1]});
          }
        bsell_host(X.A, groups, false, X.gs);
        group_counts(X.A, groups, X.counts);
      } else if (t == 1) {
        // CG products: group m = mesh m, whole blocks per mesh, each mesh's rows in Morton order of
        // their vertices: a slice's rows of every colour gather neighbouring lines of p, so each line
        // is fetched about once per product (in colour order, once per colour that gathers it)
        LevelImage &X = fine_img;
        Groups mg(nm);
        for (int m = 0; m < nm; ++m) mg[m].push_back({r0[m], r1[m]});
        bsell_host(X.A, mg, true, X.cg, &mo);
      } else if (t == 2) {
        // residual after a single forward sweep from zero: r = U x with U the later colours' entries
        // of each row (columns above the row: each mesh numbers its rows colour by colour), negated;
        // the rows that have such entries, in Morton order. The other rows' r stays zero.
        LevelImage &X = fine_img;
        HMat U;
        U.nrows = X.A.nrows;
        U.ncols = X.A.ncols;
        U.rp.assign((size_t)X.A.nrows + 1, 0);
        std::vector<uint8_t> used(std::max(X.A.ncols, 1), 0);
        int ucols = 0;
        for (int i = 0; i < X.A.nrows; ++i) {
          for (int q = X.A.rp[i]; q < X.A.rp[i + 1]; ++q)
            if (X.A.ci[q] > i) {
              U.ci.push_back(X.A.ci[q]);
              U.v.push_back(-X.A.v[q]);
              ucols += !used[X.A.ci[q]];
              used[X.A.ci[q]] = 1;
            }
          U.rp[i + 1] = (int)U.ci.size();
        }
        std::vector<int> uo;
        for (int r : mo)
          if (U.rp[r + 1] > U.rp[r]) uo.push_back(r);
        bsell_host(U, {{{0, (int)uo.size()}}}, false, X.up, &uo);
        X.up.nrows = (int)uo.size();  // byte model: rows written, distinct x entries gathered
        X.up.ncols = ucols;
      } else if (t == 3) {
        const std::vector<int> oPi = keep_rows(mo, last);
        bsell_host(Pi, {{{0, (int)oPi.size()}}}, false, pi_img, &oPi);
        transfer_stats(Pi, oPi, pi_img);
      } else if (t == 4) {
        const HMat PiT = drop_cols(htranspose(Pi), zero);
        const std::vector<int> oPiT = natural_rows(L0, 0);
        bsell_host(PiT, {{{0, PiT.nrows}}}, false, pit_img, &oPiT);
        transfer_stats(PiT, oPiT, pit_img);
      } else if (t < K + 6) {
        const int k = t - 5;
        BLevel &L = dv->aux[k];
        LevelImage &X = aux_img[k];
        int C = 0;
        for (size_t i = 0; i < smooth_m[k].size(); ++i) {
          const int m = smooth_m[k][i];
          const int l = H[m]->J - k;
          append_rows(X.A, H[m]->Al.at(l), lev[m][k].perm, &lev[m][k].iperm, L.off[i], true, &X.diag);
          C = std::max(C, (int)lev[m][k].coff.size() - 1);
          const int nl = (int)H[m]->Al.at(l).nrows;
          for (int r = 0; r < nl; ++r) X.c0flag.push_back(r < lev[m][k].coff[1]);
        }
        X.A.ncols = L.nsmooth;
        Groups groups(C);
        for (int c = 0; c < C; ++c)
          for (size_t i = 0; i < smooth_m[k].size(); ++i) {
            const auto &co = lev[smooth_m[k][i]][k].coff;
            if (c + 1 < (int)co.size()) groups[c].push_back({L.off[i] + co[c], L.off[i] + co[c + 1]});
          }
        bsell_host(X.A, groups, false, X.gs);
        group_counts(X.A, groups, X.counts);
        for (size_t i = 0; i < bottom_m[k].size(); ++i) {
          const int m = bottom_m[k][i];
          const int nc = (int)H[m]->nc;
          X.ncs.push_back(nc);
          X.voff.push_back(L.off[smooth_m[k].size() + i]);
          X.moff.push_back((int64_t)X.inv.size());
          X.inv.insert(X.inv.end(), H[m]->coarse_inv.begin(), H[m]->coarse_inv.end());
          X.pref.push_back(X.pref.back() + (nc + kGemvRows - 1) / kGemvRows);  // waves of kb_gemv
          X.bt_entries += (double)nc * nc;
          X.bt_rows += nc;
        }
        X.inv32.assign(X.inv.begin(), X.inv.end());
      } else {
        // prolongation P (level k+1 -> k) for the smoothing meshes of level k
        const int k = t - (K + 6);
        BLevel &L = dv->aux[k], &Lc = dv->aux[k + 1];
        HMat P;
        for (int m : smooth_m[k]) {
          const int D = H[m]->J - H[m]->lc;
          const int l = H[m]->J - k;
          const size_t j = std::find(Lc.mesh.begin(), Lc.mesh.end(), m) - Lc.mesh.begin();
          const std::vector<int> *cmap = (D > k + 1) ? &lev[m][k + 1].iperm : nullptr;
          append_rows(P, H[m]->P.at(l), lev[m][k].perm, cmap, Lc.off[j], false, nullptr);
        }
        P.ncols = Lc.nrows;
        std::vector<uint8_t> last(P.nrows, 0), zero(P.nrows, 0);
        int C = 0;
        for (int m : smooth_m[k]) C = std::max(C, (int)lev[m][k].coff.size() - 1);
        for (size_t i = 0; i < smooth_m[k].size(); ++i) {
          const auto &co = lev[smooth_m[k][i]][k].coff;
          const int Cm = (int)co.size() - 1;
          if (Cm < 1) continue;
          for (int r = L.off[i] + co[Cm - 1]; r < L.off[i] + co[Cm]; ++r) {
            last[r] = 1;
            if (Cm == C) zero[r] = 1;
          }
        }
        // the level's rows in each mesh's own numbering; P has the smoothing meshes' rows only
        // (the first P.nrows of the merged level), not those of meshes whose bottom it is
        std::vector<int> nat = natural_rows(L, k);
        nat.erase(std::remove_if(nat.begin(), nat.end(), [&](int r) { return r >= P.nrows; }), nat.end());
        const std::vector<int> oP = keep_rows(nat, last), oPT = natural_rows(Lc, k + 1);
        bsell_host(P, {{{0, (int)oP.size()}}}, false, p_img[k], &oP);
        transfer_stats(P, oP, p_img[k]);
        const HMat PT = drop_cols(htranspose(P), zero);
        bsell_host(PT, {{{0, PT.nrows}}}, false, pt_img[k], &oPT);
        transfer_stats(PT, oPT, pt_img[k]);
      }
    });
    // ---- uploads
    {
      LevelImage &X = fine_img;
      bupload_csr(dv, X.A, dv->fineA);
      upload_diag(dv, F, X.diag, X.c0flag);
      alloc_level_vectors(dv, F);
      bsell_upload(dv, X.gs, F.sell);
      set_counts(F, std::move(X.counts));
      bsell_upload(dv, X.cg, dv->cg_sell);
      bsell_upload(dv, X.up, dv->fine_up);
      dv->cg_b0 = bupload(dv, X.cg.block0);
      dv->fine_sp = make_mesh_blocks(dv, r0, r1, BS / dv->fineA.lpr);
      X = LevelImage();
      // element-wise blocks: 256-row chunks of each mesh (one block for an empty mesh)
      std::vector<int> em, e0, e1, eb{0};
      for (int m = 0; m < nm; ++m) {
        int r = r0[m];
        do {
          em.push_back(m);
          e0.push_back(r);
          e1.push_back(std::min(r + BS, r1[m]));
          r += BS;
        } while (r < r1[m]);
        eb.push_back((int)em.size());
      }
      dv->ew_blocks = (int)em.size();
      dv->ew_m = bupload(dv, em);
      dv->ew_r0 = bupload(dv, e0);
      dv->ew_r1 = bupload(dv, e1);
      dv->ew_b0 = bupload(dv, eb);
    }
    for (int k = 0; k <= K; ++k) {
      BLevel &L = dv->aux[k];
      LevelImage &X = aux_img[k];
      bsell_upload(dv, X.gs, L.sell);
      set_counts(L, std::move(X.counts));
      upload_diag(dv, L, X.diag, X.c0flag);
      L.bottom_waves = X.pref.back();
      L.bt_entries = X.bt_entries;
      L.bt_rows = X.bt_rows;
      L.bt_wavepref = bupload(dv, X.pref);
      L.bt_nc = bupload(dv, X.ncs);
      L.bt_voff = bupload(dv, X.voff);
      L.bt_moff = bupload(dv, X.moff);
      L.inv64 = bupload(dv, X.inv);
      L.inv32 = bupload(dv, X.inv32);
      alloc_level_vectors(dv, L);
      X = LevelImage();
    }
    for (int k = 0; k < K; ++k) {
      bsell_upload(dv, p_img[k], dv->aux[k].P);
      bsell_upload(dv, pt_img[k], dv->aux[k].PT);
    }
    bsell_upload(dv, pi_img, dv->Pi);
    bsell_upload(dv, pit_img, dv->PiT);
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
    const int64_t nblocks_max = std::max<int64_t>({(int64_t)dv->fine_sp.nblocks, (int64_t)dv->ew_blocks,
                                                   (int64_t)dv->cg_sell.nslices / (BS / 64)});
    dv->partials = balloc<double>(dv, nblocks_max * 4);
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
  for (hipEvent_t e : dv->tune_ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : dv->probe_ev) (void)hipEventDestroy(e);
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

static inline double bsell_bytes(const BSell &A, int s) { return (double)A.nnz * (s + 4) + 4.0 * (A.nrows + 1); }

template <class T>
static const T *bsv(const BSell &S);
template <>
const double *bsv<double>(const BSell &S) { return S.sv64; }
template <>
const float *bsv<float>(const BSell &S) { return S.sv32; }

template <class T>
static const T *bid0(const BLevel &L);
template <>
const double *bid0<double>(const BLevel &L) { return L.id0_64; }
template <>
const float *bid0<float>(const BLevel &L) { return L.id0_32; }

// One slice-kernel launch site of B_co: launch(threads, xcd, e0, e1) enqueues the kernel over
// `nslices` slices (launch_timed: with events, they are stamped with the kernel's own start and
// end). While tuning, the site runs the candidate shape under trial with its pair of events, so
// that its time is measured inside a whole B_co application (caches as in a solve); otherwise
// it runs the shape stored for the site (or the default). The tuned kernels have no
// reductions, so the shape does not change any result.
// With probe_bytes >= 0 and per-launch timing on, the launch is stamped with the next pair of
// probe events and counted with that many algorithmic bytes.
template <class F>
static void slice_launch(BatchDevice *dv, int nslices, hipStream_t s, F &&launch, double probe_bytes = -1.0) {
  auto &tab = dv->shape[dv->shape_pi][dv->shape_nr];
  const int site = dv->site++;
  if (nslices <= 0) return;
  auto sh = site < (int)tab.size() ? tab[site] : kShapes[0];
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (dv->probe && probe_bytes >= 0.0) {
    if (dv->probe_used + 2 > dv->probe_ev.size()) {
      hipEvent_t p0, p1;
      HIPCHECK(hipEventCreate(&p0));
      HIPCHECK(hipEventCreate(&p1));
      dv->probe_ev.push_back(p0);
      dv->probe_ev.push_back(p1);
    }
    e0 = dv->probe_ev[dv->probe_used];
    e1 = dv->probe_ev[dv->probe_used + 1];
    dv->probe_used += 2;
    dv->probe_bytes.push_back(probe_bytes);
  } else if (dv->tuning) {
    while ((int)dv->tune_ev.size() < 2 * (site + 1)) {
      hipEvent_t e;
      HIPCHECK(hipEventCreate(&e));
      dv->tune_ev.push_back(e);
    }
    sh = kShapes[dv->tune_k];
    e0 = dv->tune_ev[2 * site];
    e1 = dv->tune_ev[2 * site + 1];
    dv->tune_live = std::max(dv->tune_live, site + 1);
    dv->tune_has.resize(std::max<size_t>(dv->tune_has.size(), site + 1), 0);
    dv->tune_has[site] = 1;
  }
  launch(sh.threads, sh.xcd, sh.var, e0, e1);
}


// Gauss-Seidel sweep over the colour groups of L. `first_done`: the sweep starts from zero and
// its colour-0 pass was run by the kernel that produced b.
template <int NR, class T>
static void b_sweep(BatchDevice *dv, BLevel &L, const T *b, bool from_zero, bool first_done, bool forward,
                    hipStream_t s) {
  if (L.nsmooth == 0) return;
  T *x = BV<T>::x(L);
  const BSell &S = L.sell;
  const int C = (int)S.cslice.size() - 1;
  // `from0`: the pass belongs to a sweep from zero, where every neighbour of a later colour is
  // still zero in exact terms but may hold anything in memory: it adds only the earlier colours'
  // entries (kb_sell MODE 3) and, with LOWER_FIRST_SWEEP, reads only the prefix of each slice's
  // entries that holds them (`lower`)
  auto pass = [&](int c, bool from0) {
    const bool lower = LOWER_FIRST_SWEEP && from0;
    const int s0 = S.cslice[c], s1 = S.cslice[c + 1];
    // algorithmic bytes of the pass: the colour's matrix rows (values, columns, one row index),
    // b, 1/diag and the x write of its rows, each distinct gathered x entry once
    const double sz = sizeof(T), rows = (double)L.crows[c];
    const double nz = (double)(lower ? L.cnnz_lo[c] : L.cnnz[c]), uc = (double)(lower ? L.ucols_lo[c] : L.ucols[c]);
    const double by = nz * (sz + 4) + 4.0 * (rows + 1) + sz * rows * (2.0 * NR + 1) + sz * NR * uc;
    slice_launch(
        dv, s1 - s0, s,
        [&](int th, int xcd, int var, hipEvent_t e0, hipEvent_t e1) {
          with_var(var, [&](auto vc) {
            constexpr int V = decltype(vc)::value;
            if (from0)
              launch_timed((kb_sell<3, NR, T, V>), slice_blocks(s1 - s0, th, var), th, s, e0, e1, s0, s1, S.srow,
                           S.soff, lower ? S.slo : S.soff + 1, S.scol, bsv<T>(S), BV<T>::id(L), b, x, (T *)nullptr,
                           shape_arg(th, xcd));
            else
              launch_timed((kb_sell<0, NR, T, V>), slice_blocks(s1 - s0, th, var), th, s, e0, e1, s0, s1, S.srow,
                           S.soff, S.soff + 1, S.scol, bsv<T>(S), BV<T>::id(L), b, x, (T *)nullptr,
                           shape_arg(th, xcd));
          });
        },
        by);
  };
  const bool lower = LOWER_FIRST_SWEEP && forward && from_zero;
  if (forward) {
    int c = 0;
    if (from_zero) {
      if (!first_done)
        hipLaunchKernelGGL((kb_first<NR, T>), dim3(nblk(L.nsmooth)), dim3(BS), 0, s, L.nsmooth, b, bid0<T>(L), x);
      c = 1;
    }
    for (; c < C; ++c) pass(c, from_zero);
  } else {
    for (int c = C - 1; c >= 0; --c) pass(c, false);
  }
  if (dv->count_bytes) {
    double by = bsell_bytes(S, sizeof(T)) + (double)L.nsmooth * sizeof(T) * (3.0 * NR + 1);
    if (lower)  // the passes of colours >= 1 read only the earlier colours' entries
      for (int c = 1; c < C; ++c) by -= (double)(L.cnnz[c] - L.cnnz_lo[c]) * (sizeof(T) + 4);
    dv->bytes += by;
  }
}

// r = b - A x right after a forward sweep. Slice group C-1 holds only rows of the last colour of
// their mesh, which that sweep's last pass solved with every neighbour final: their residual is
// zero in exact arithmetic, so the kernel skips the group (r was zeroed at setup there and
// nothing else writes it). Meshes with fewer colours have their last colour in earlier groups,
// which are computed.
// `upper`: x is the result of a single forward sweep from zero, and the kernel computes each row's
// residual from its later colours' terms alone (kb_sell MODE 2).
template <int NR, class T>
static void b_residual(BatchDevice *dv, BLevel &L, const T *b, hipStream_t s, bool upper) {
  if (L.nsmooth == 0) return;
  const BSell &S = L.sell;
  const int C = (int)S.cslice.size() - 1;
  const int s1 = C >= 1 ? S.cslice[C - 1] : S.nslices;
  slice_launch(dv, s1, s, [&](int th, int xcd, int var, hipEvent_t e0, hipEvent_t e1) {
    with_var(var, [&](auto vc) {
      if (upper)
        launch_timed((kb_sell<2, NR, T, decltype(vc)::value>), slice_blocks(s1, th, var), th, s, e0, e1, 0, s1, S.srow,
                     S.shi, S.soff + 1, S.scol, bsv<T>(S), (const T *)nullptr, (const T *)nullptr, BV<T>::x(L),
                     BV<T>::r(L), shape_arg(th, xcd));
      else
        launch_timed((kb_sell<1, NR, T, decltype(vc)::value>), slice_blocks(s1, th, var), th, s, e0, e1, 0, s1, S.srow,
                     S.soff, S.soff + 1, S.scol, bsv<T>(S), BV<T>::dg(L), b, BV<T>::x(L), BV<T>::r(L),
                     shape_arg(th, xcd));
    });
  });
  if (dv->count_bytes && S.nslices > 0) {
    if (upper) {
      // the later colours' entries, the row indices, r written, each gathered x entry once
      const double sz = sizeof(T);
      for (int c = 0; c + 1 < C; ++c)
        dv->bytes += (double)L.cnnz_up[c] * (sz + 4) + 4.0 * (double)L.crows[c] +
                     sz * NR * (double)(L.crows[c] + L.ucols_up[c]);
    } else {
      dv->bytes += (bsell_bytes(S, sizeof(T)) + (double)L.nsmooth * sizeof(T) * (3.0 * NR + 1)) * s1 / S.nslices;
    }
  }
}

// y = A x (ADD 0) or y += A x (ADD 1); FIRST: y is level Lt's right-hand side and the first colour
// pass on Lt runs in the same kernel
template <int NR, int ADD, int FIRST, class T>
static void b_spmv(BatchDevice *dv, const BSell &A, const T *x, T *y, BLevel *Lt, hipStream_t s) {
  if (A.nrows == 0) return;
  slice_launch(dv, A.nslices, s, [&](int th, int xcd, int var, hipEvent_t e0, hipEvent_t e1) {
    with_var(var, [&](auto vc) {
      launch_timed((kb_sell_spmv<ADD, FIRST, NR, T, decltype(vc)::value>), slice_blocks(A.nslices, th, var), th, s, e0, e1,
                   A.nslices, A.srow, A.soff, A.scol, bsv<T>(A), x, y, FIRST ? bid0<T>(*Lt) : (const T *)nullptr,
                   FIRST ? BV<T>::x(*Lt) : (T *)nullptr, shape_arg(th, xcd));
    });
  });
  if (dv->count_bytes) {
    // matrix, x gathered, y written (and read with ADD); FIRST: 1/a_ii read on every row, the
    // first pass's x written on the colour-0 rows
    const double c0 = FIRST && Lt && !Lt->crows.empty() ? (double)Lt->crows[0] : 0.0;
    dv->bytes += bsell_bytes(A, sizeof(T)) + (double)sizeof(T) * NR * (A.ncols + (1 + ADD) * (double)A.nrows + c0) +
                 (FIRST ? (double)sizeof(T) * A.nrows : 0.0);
  }
}

template <int NR, class T>
static void b_vcycle(BatchDevice *dv, int k, hipStream_t s) {
  BLevel &L = dv->aux[k];
  const T *b = BV<T>::b(L);
  if (L.nbottom > 0 && L.bottom_waves > 0) {
    hipLaunchKernelGGL((kb_gemv<NR, T>), dim3(nblk((int64_t)L.bottom_waves * 64)), dim3(BS), 0, s, L.bt_wavepref,
                       L.nbottom, L.bt_nc, L.bt_moff, L.bt_voff, BV<T>::inv(L), b, BV<T>::x(L));
    // the bottom inverses, g read and y written
    if (dv->count_bytes) dv->bytes += L.bt_entries * sizeof(T) + 2.0 * NR * sizeof(T) * L.bt_rows;
  }
  if (L.nsmooth == 0) return;
  for (int it = 0; it < dv->nu_aux; ++it) b_sweep<NR, T>(dv, L, b, it == 0, true, true, s);
  b_residual<NR, T>(dv, L, b, s, UPPER_RESIDUAL && dv->nu_aux == 1);
  BLevel &Lc = dv->aux[k + 1];
  b_spmv<NR, 0, 1, T>(dv, L.PT, BV<T>::r(L), BV<T>::b(Lc), &Lc, s);
  b_vcycle<NR, T>(dv, k + 1, s);
  b_spmv<NR, 1, 0, T>(dv, L.P, BV<T>::x(Lc), BV<T>::x(L), nullptr, s);
  for (int it = 0; it < dv->nu_aux; ++it) b_sweep<NR, T>(dv, L, b, false, false, false, s);
}

// z = B_co r for every system; r (FP64, internal) -> fine.x (precision T). `first_done`: the CG
// update already ran the first colour pass on the original grids (and the FP32 rounding of r).
template <int NR, class T>
static void b_apply(BatchDevice *dv, const double *r, bool first_done, hipStream_t s) {
  BLevel &F = dv->fine;
  dv->site = 0;
  dv->shape_pi = sizeof(T) == 4 ? 1 : 0;
  dv->shape_nr = NR;
  const T *b;
  if constexpr (sizeof(T) == 8) {
    b = r;
  } else {
    if (!first_done) {
      hipLaunchKernelGGL((kb_first_cvt<NR>), dim3(nblk(F.nrows)), dim3(BS), 0, s, F.nrows, r, F.id0_32, F.b32, F.x32);
      first_done = true;
    }
    b = F.b32;
  }
  for (int it = 0; it < dv->nu_fine; ++it) b_sweep<NR, T>(dv, F, b, it == 0, first_done, true, s);
  if (UPPER_RESIDUAL && dv->nu_fine == 1)
    b_spmv<NR, 0, 0, T>(dv, dv->fine_up, BV<T>::x(F), BV<T>::r(F), nullptr, s);  // r = U x (U negated)
  else
    b_residual<NR, T>(dv, F, b, s, false);
  b_spmv<NR, 0, 1, T>(dv, dv->PiT, BV<T>::r(F), BV<T>::b(dv->aux[0]), &dv->aux[0], s);
  b_vcycle<NR, T>(dv, 0, s);
  b_spmv<NR, 1, 0, T>(dv, dv->Pi, BV<T>::x(dv->aux[0]), BV<T>::x(F), nullptr, s);
  for (int it = 0; it < dv->nu_fine; ++it) b_sweep<NR, T>(dv, F, b, false, false, false, s);
}

template <int NR, class T>
static void b_tail(BatchDevice *dv, hipStream_t s, bool first_done) {
  b_apply<NR, T>(dv, dv->r, first_done, s);
  const T *z = BV<T>::x(dv->fine);
  hipLaunchKernelGGL((kb_cg_rz<NR, T>), dim3(dv->ew_blocks), dim3(BS), 0, s, dv->ew_r0, dv->ew_r1, dv->r, z, dv->ctl,
                     dv->partials);
  hipLaunchKernelGGL((kb_fin_rz<NR>), dim3(dv->nm), dim3(BS), 0, s, dv->ew_b0, dv->partials, dv->ctl);
  hipLaunchKernelGGL((kb_cg_p<NR, T>), dim3(dv->ew_blocks), dim3(BS), 0, s, dv->ew_m, dv->ew_r0, dv->ew_r1, z, dv->p,
                     dv->ctl);
}

template <int NR, class T>
static void b_iteration(BatchDevice *dv, hipStream_t s) {
  BLevel &F = dv->fine;
  const BSell &Q = dv->cg_sell;
  hipLaunchKernelGGL((kb_cg_spmv<NR>), dim3(Q.nslices / (BS / 64)), dim3(BS), 0, s, Q.srow, Q.soff, Q.scol, Q.sv64,
                     F.dg64, dv->p, dv->q, dv->ctl, dv->partials);
  hipLaunchKernelGGL((kb_fin_spmv<NR>), dim3(dv->nm), dim3(BS), 0, s, dv->cg_b0, dv->partials, dv->ctl);
  hipLaunchKernelGGL((kb_cg_axpy<NR, T>), dim3(dv->ew_blocks), dim3(BS), 0, s, dv->ew_m, dv->ew_r0, dv->ew_r1, dv->u,
                     dv->r, dv->p, dv->q, dv->ctl, dv->partials, bid0<T>(F), BV<T>::b(F), BV<T>::x(F));
  hipLaunchKernelGGL((kb_fin_axpy<NR>), dim3(dv->nm), dim3(BS), 0, s, dv->ew_b0, dv->partials, dv->ctl);
  b_tail<NR, T>(dv, s, true);
}

// Autotuner: for every candidate shape (twice), one eager B_co application on the current r with
// all slice sites in that shape and HIP events around each; every site then keeps the shape of
// its shortest time if that beats the default clearly (pick_shape). The solve that follows starts
// B_co from scratch.
template <int NR, class T>
static void b_tune(BatchDevice *dv, hipStream_t s) {
  const int pi = sizeof(T) == 4 ? 1 : 0;
  if (dv->tuned[pi][NR] || !dv->autotune) return;
  TraceRange tr_tune("asmg::batch_autotune");
  const int K = kNumShapes;
  std::vector<std::vector<float>> t;
  dv->tuning = true;
  try {
    for (int round = 0; round < kTuneRounds; ++round)
      for (int k = 0; k < K; ++k) {
        dv->tune_k = k;
        dv->tune_live = 0;
        b_apply<NR, T>(dv, dv->r, false, s);
        HIPCHECK(hipStreamSynchronize(s));
        if ((int)t.size() < dv->tune_live) t.resize(dv->tune_live, std::vector<float>(K, INFINITY));
        for (int site = 0; site < dv->tune_live; ++site) {
          if (!dv->tune_has[site]) continue;
          float ms = 0;
          HIPCHECK(hipEventElapsedTime(&ms, dv->tune_ev[2 * site], dv->tune_ev[2 * site + 1]));
          t[site][k] = std::min(t[site][k], ms);
        }
      }
  } catch (...) {
    dv->tuning = false;
    throw;
  }
  dv->tuning = false;
  auto &tab = dv->shape[pi][NR];
  tab.assign(t.size(), kShapes[0]);
  for (size_t site = 0; site < t.size(); ++site)
    tab[site] = kShapes[pick_shape(t[site])];
  dv->tune_times[pi][NR] = t;
  dv->tuned[pi][NR] = true;
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
  const SegTable &Sp = dv->fine_sp;
  const BCsr &FA = dv->fineA;
  BLevel &F = dv->fine;
  // per-system ints (4 arrays sized for 4 right-hand sides), mesh tickets, active count, done flag
  HIPCHECK(hipMemsetAsync(dv->ctl_ints, 0, ((size_t)nm * 4 * 4 + nm + 2) * sizeof(int), s));
  hipLaunchKernelGGL((kb_cg_init<NR>), dim3(dv->ew_blocks), dim3(BS), 0, s, dv->ew_r0, dv->ew_r1, dv->f, dv->r, dv->u,
                     dv->p, dv->partials);
  hipLaunchKernelGGL((kb_fin_init<NR>), dim3(nm), dim3(BS), 0, s, dv->ew_b0, dv->partials, tol, dv->ctl);
  b_tune<NR, T>(dv, s);  // first solve of this (precision, NR): pick the launch shapes (r = f now)
  int hst[2];
  HIPCHECK(hipMemcpyAsync(hst, dv->ctl.active, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  if (hst[0] == 0) HIPCHECK(hipMemcpyAsync(dv->ctl.gdone, &(hst[1] = 1), sizeof(int), hipMemcpyHostToDevice, s));
  b_tail<NR, T>(dv, s, false);
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
    with_lpr(FA.lpr, [&](auto cc) {
      constexpr int LP = decltype(cc)::value;
      hipLaunchKernelGGL((kb_true_res<LP, NR>), dim3(Sp.nblocks), dim3(BS), 0, s, Sp.r0, Sp.r1, Sp.b0, Sp.nseg,
                         FA.rp, FA.ci, FA.v64, F.dg64, dv->f, dv->u, dv->partials);
    });
    hipLaunchKernelGGL((kb_fin_tr<NR>), dim3(nm), dim3(BS), 0, s, Sp.b0, dv->partials, dv->ctl);
    HIPCHECK(hipMemcpyAsync(tr.data(), dv->ctl.tr, ns * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipMemcpyAsync(fn2.data(), dv->ctl.fn2, ns * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipMemcpyAsync(st.data(), dv->ctl.status, ns * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipMemcpyAsync(it.data(), dv->ctl.iter, ns * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    // a system that converged on its updated residual with the true residual above tol restarts
    // from the true residual (at most 3 rounds), or ends unconverged if its iterations are spent
    int nre = 0;
    for (int i = 0; i < ns; ++i) {
      const double rel = fn2[i] > 0 ? std::sqrt(tr[i] / fn2[i]) : 0.0;
      const bool want = st[i] == BST_OK && fn2[i] > 0 && rel > tol && restarts < 3;
      if (want && it[i] >= dv->maxit) st[i] = BST_NOCONV;
      mask[i] = (want && it[i] < dv->maxit) ? 1 : 0;
      nre += mask[i];
    }
    if (nre > 0) {
      ++restarts;
      HIPCHECK(hipMemcpyAsync(dv->mask, mask.data(), ns * sizeof(int), hipMemcpyHostToDevice, s));
      with_lpr(FA.lpr, [&](auto cc) {
        constexpr int LP = decltype(cc)::value;
        hipLaunchKernelGGL((kb_restart<LP, NR>), dim3(Sp.nblocks), dim3(BS), 0, s, Sp.r0, Sp.r1, Sp.b0, Sp.nseg,
                           FA.rp, FA.ci, FA.v64, F.dg64, dv->f, dv->u, dv->r, dv->p, dv->mask);
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
      b_tail<NR, T>(dv, s, false);
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

// The residual kernel leaves the rows of the last colour group unwritten, so they must hold
// zeros in the [row][NR] layout of this NR: after residuals with another NR, clear r (eagerly,
// never inside a captured graph).
static void b_prepare_r(BatchDevice *dv, int nr, hipStream_t s) {
  if (dv->r_nr != 0 && dv->r_nr != nr) {
    auto clear = [&](BLevel &L) {
      const size_t n = (size_t)std::max<int64_t>((int64_t)L.nrows * 4, 1);
      HIPCHECK(hipMemsetAsync(L.r64, 0, n * 8, s));
      HIPCHECK(hipMemsetAsync(L.r32, 0, n * 4, s));
    };
    clear(dv->fine);
    for (auto &L : dv->aux) clear(L);
  }
  dv->r_nr = nr;
}

template <int NR>
static int b_solve_nr(BatchDevice *dv, const double *d_F, double tol, double *d_U, int *iters, double *true_rel,
                      hipStream_t cs) {
  TraceRange tr_solve("asmg::batch_solve");
  hipStream_t s = dv->stream;
  const int n = dv->fine.nrows;
  HIPCHECK(hipEventRecord(dv->ev_in, cs));
  HIPCHECK(hipStreamWaitEvent(s, dv->ev_in, 0));
  hipLaunchKernelGGL((kb_gather<NR>), dim3(nblk(n)), dim3(BS), 0, s, n, dv->row_src0[NR], dv->row_stride, d_F, dv->f);
  b_prepare_r(dv, NR, s);
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
      case 1: mixed ? b_apply<1, float>(dv, dv->f, false, s) : b_apply<1, double>(dv, dv->f, false, s); break;
      case 2: mixed ? b_apply<2, float>(dv, dv->f, false, s) : b_apply<2, double>(dv, dv->f, false, s); break;
      default: mixed ? b_apply<4, float>(dv, dv->f, false, s) : b_apply<4, double>(dv, dv->f, false, s); break;
    }
  };
  HIPCHECK(hipMemsetAsync(dv->f, 0, (size_t)dv->fine.nrows * 4 * sizeof(double), s));
  b_prepare_r(dv, n_rhs == 1 ? 1 : n_rhs == 2 ? 2 : 4, s);
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

template <int NR>
static int b_time_kernel_nr(BatchDevice *dv, int which, int reps, bool mixed, hipStream_t s, double *ms,
                            double *bytes) {
  auto bco_on = [&](hipStream_t st) {
    if (mixed)
      b_apply<NR, float>(dv, dv->f, false, st);
    else
      b_apply<NR, double>(dv, dv->f, false, st);
  };
  HIPCHECK(hipMemsetAsync(dv->f, 0, (size_t)dv->fine.nrows * 4 * sizeof(double), s));
  b_prepare_r(dv, NR, s);
  if (which == 1) {
    // every Gauss-Seidel colour pass inside `reps` B_co applications, each launch stamped with its
    // own start and end events (one launch per pair: caches as in a solve)
    bco_on(s);  // warm-up
    dv->probe = true;
    dv->probe_used = 0;
    dv->probe_bytes.clear();
    try {
      for (int k = 0; k < reps; ++k) bco_on(s);
    } catch (...) {
      dv->probe = false;
      throw;
    }
    dv->probe = false;
    HIPCHECK(hipStreamSynchronize(s));
    double tot = 0, by = 0;
    const size_t nl = dv->probe_used / 2;
    for (size_t i = 0; i < nl; ++i) {
      float t = 0;
      HIPCHECK(hipEventElapsedTime(&t, dv->probe_ev[2 * i], dv->probe_ev[2 * i + 1]));
      tot += t;
    }
    for (double b : dv->probe_bytes) by += b;
    *ms = nl ? tot / nl : 0.0;
    *bytes = nl ? by / nl : 0.0;
    return ASMG_OK;
  }
  // which 0: one B_co application captured in a hipGraph as the solve runs it; median over
  // `reps` replays, each between its own pair of events
  dv->count_bytes = true;
  dv->bytes = 0;
  bco_on(s);
  dv->count_bytes = false;
  *bytes = dv->bytes;
  HIPCHECK(hipStreamSynchronize(s));
  hipStream_t gs = dv->stream;
  hipGraph_t g;
  hipGraphExec_t ge;
  HIPCHECK(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
  bco_on(gs);
  HIPCHECK(hipStreamEndCapture(gs, &g));
  HIPCHECK(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
  HIPCHECK(hipGraphDestroy(g));
  HIPCHECK(hipGraphLaunch(ge, gs));  // warm-up
  const int R = std::max(reps, 1);
  std::vector<hipEvent_t> ev(2 * R);
  for (auto &e : ev) HIPCHECK(hipEventCreate(&e));
  for (int k = 0; k < R; ++k) {
    HIPCHECK(hipEventRecord(ev[2 * k], gs));
    HIPCHECK(hipGraphLaunch(ge, gs));
    HIPCHECK(hipEventRecord(ev[2 * k + 1], gs));
  }
  HIPCHECK(hipStreamSynchronize(gs));
  std::vector<float> t(R);
  for (int k = 0; k < R; ++k) HIPCHECK(hipEventElapsedTime(&t[k], ev[2 * k], ev[2 * k + 1]));
  for (auto &e : ev) HIPCHECK(hipEventDestroy(e));
  HIPCHECK(hipGraphExecDestroy(ge));
  std::sort(t.begin(), t.end());
  *ms = R % 2 ? (double)t[R / 2] : 0.5 * ((double)t[R / 2 - 1] + (double)t[R / 2]);
  return ASMG_OK;
}

int batch_device_time_kernel(BatchDevice *dv, int which, int n_rhs, int reps, int precision, void *stream, double *ms,
                             double *bytes) {
  HIPCHECK(hipSetDevice(dv->ordinal));
  hipStream_t s = (hipStream_t)stream;
  const bool mixed = precision == ASMG_PREC_MIXED;
  switch (n_rhs) {
    case 1: return b_time_kernel_nr<1>(dv, which, reps, mixed, s, ms, bytes);
    case 2: return b_time_kernel_nr<2>(dv, which, reps, mixed, s, ms, bytes);
    default: return b_time_kernel_nr<4>(dv, which, reps, mixed, s, ms, bytes);
  }
}

int64_t batch_n_total(BatchDevice *dv) { return dv->dof_off.back(); }

std::vector<int64_t> batch_tuned_shapes(BatchDevice *dv, int nr, int precision) {
  std::vector<int64_t> out;
  if (nr < 1 || nr > 4 || precision < 0 || precision > 1) return out;
  for (const auto &sh : dv->shape[precision][nr]) {
    out.push_back(sh.threads);
    out.push_back(sh.xcd);
    out.push_back(sh.var);
  }
  return out;
}

std::vector<double> batch_tune_times(BatchDevice *dv, int nr, int precision) {
  std::vector<double> out;
  if (nr < 1 || nr > 4 || precision < 0 || precision > 1) return out;
  for (const auto &row : dv->tune_times[precision][nr])
    for (float t : row) out.push_back(std::isfinite(t) ? (double)t : -1.0);
  return out;
}

}  // namespace asmg
