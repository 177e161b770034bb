// Device side of the ASMG-PCG solve on gfx950 (CDNA4, wave64).
//
// Layout: every level (the original grid and the auxiliary levels above the
// bottom) is renumbered colour-major (rows of colour 0 first, ascending unknown
// id inside a colour), so one Gauss-Seidel colour pass is a contiguous row range.
// Off-diagonal parts of the level matrices and the transfers (Pi, Pi^T, P_l,
// P_l^T, stored explicitly in the internal numbering) are sliced ELL with 64-row
// slices, one row per wave lane; the diagonal is held apart (diag and 1/diag);
// values in FP64 and FP32 copies. The bottom level keeps the unknown order and
// holds the explicit inverse of its matrix (from the Cholesky factor built on the
// host), applied as a wave-per-row GEMV.
//
// A slice kernel is latency-bound on short colour passes, so its row product
// issues all loads of a row before the first gather (three dependent round trips
// per slice), and its blocks are remapped so that each XCD (own L2) takes a
// contiguous run of slices. The first colour pass of a sweep from zero runs inside
// the kernel that writes the level's right-hand side.
//
// PCG: reductions write one partial per block and a one-block finalize kernel sums
// them in a fixed order (reproducible, no atomics); the CG kernels read a device
// `done` flag and return when it is set, so the host may enqueue (replay a graph of)
// several iterations ahead and the iteration count stays exact.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <numeric>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "common.hpp"
#include "device.hpp"
#include "host_parallel.hpp"
#include "trace.hpp"

namespace asmg {

#ifndef LOWER_FIRST_SWEEP
#define LOWER_FIRST_SWEEP 1
#endif
#ifndef UPPER_RESIDUAL
#define UPPER_RESIDUAL 1
#endif

// ---------------------------------------------------------------------------
// device control block for PCG
// ---------------------------------------------------------------------------

struct Ctl {
  double rho, pq, rr, alpha, beta, fnorm2, tol2, rz, tr, mean;
  int iter, done, status, maxit, first, pad;
  unsigned ticket;
};

enum { ST_OK = 0, ST_NOTSPD = 1, ST_NAN = 2, ST_NOCONV = 3 };

// first colour pass of a sweep that starts from x = 0: colour-0 rows get b_i / a_ii, all other rows 0
template <class T>
__global__ __launch_bounds__(BS) void k_gs_first(int n, int c0, const T *__restrict__ b, const T *__restrict__ invd,
                                                 T *__restrict__ x) {
  const int i = blockIdx.x * BS + threadIdx.x;
  if (i < n) x[i] = i < c0 ? b[i] * invd[i] : T(0);
}

// mixed precision: first pass of the fine sweep also rounds the FP64 right-hand side to FP32
__global__ __launch_bounds__(BS) void k_gs_first_cvt(int n, int c0, const double *__restrict__ r64,
                                                     float *__restrict__ b32, const float *__restrict__ invd,
                                                     float *__restrict__ x) {
  const int i = blockIdx.x * BS + threadIdx.x;
  if (i < n) {
    const float bi = (float)r64[i];
    b32[i] = bi;
    x[i] = i < c0 ? bi * invd[i] : 0.0f;
  }
}

// Sliced ELL (64 rows per slice = one wave, one row per lane), per colour, rows sorted by
// length inside windows of 256 rows. Entry k of slice s, lane j sits at soff[s] + 64 k + j;
// padding entries repeat a column of the lane's row with value 0; srow = -1 marks empty lanes
// (their entries are padding too, so every lane may load its w entries).
//
// An empty volatile asm that takes v as input and output: the value must be computed on every
// active lane at this point, so the compiler cannot sink the loads feeding it under the
// `row >= 0` store condition (which would wait for srow before issuing them).
template <class T>
__device__ __forceinline__ void pin(T &v) {
  asm volatile("" : "+v"(v));
}

// A wave handles one slice. Its width w is uniform over the wave, so a row is processed by a
// switch over w into straight-line code that issues every column and value load of the row,
// then the row's own loads (`pre`: right-hand side, diagonal), then the gathers of x, and
// finally calls `post` with the row product. With the row index (srow) loaded before the
// matrix entries, a slice costs three dependent memory round trips:
// {soff, srow} -> {columns, values, row data} -> gathers.
// UP: only the entries with a column above `urow` (the row's later colours) take part; the others
// are neither gathered nor added.
template <int W, bool NT = false, bool UP = false, class T, class Pre, class Post>
__device__ __forceinline__ void sell_row_w(const int *__restrict__ cp, const T *__restrict__ vp,
                                           const T *__restrict__ x, Pre &pre, Post &post, int urow = 0) {
  int c[W];
  T v[W];
  if constexpr (NT || std::is_same<T, float>::value) {
    // FP32 passes and the transfers (NT) stream the matrix entries with nontemporal loads (each
    // is read once per pass), leaving more of L2 to the gathered x lines. Measured: mixed solves
    // 1.4 % faster on the graded and cube workloads, FP64 B_co 0.6 % (graded) and 1.4 % (cube)
    // faster with nontemporal transfers; in the FP64 colour passes the same loads made the graded
    // solve slower, so those keep plain loads.
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
  T a0 = 0, a1 = 0;
#pragma unroll
  for (int k = 0; k < W; ++k) {
    if (UP && c[k] <= urow) continue;
    if (k & 1)
      a1 += v[k] * x[c[k]];
    else
      a0 += v[k] * x[c[k]];
  }
  T acc = a0 + a1;
  pin(acc);
  post(acc);
}

template <int W, bool NT, bool UP, class T>
__device__ __forceinline__ T sell_chunk(const int *__restrict__ cp, const T *__restrict__ vp,
                                        const T *__restrict__ x, int urow) {
  T acc = 0;
  auto pre = [] {};
  auto post = [&](T a) { acc = a; };
  sell_row_w<W, NT, UP>(cp, vp, x, pre, post, urow);
  return acc;
}

// Straight-line cases up to WMAX entries (16, or 32 for matrices with longer rows such as the
// 3-D transfers); longer rows go in chunks of 8.
template <class T, int WMAX = 16, bool NT = false, bool UP = false, class Pre, class Post>
__device__ __forceinline__ void sell_row(int w, const int *__restrict__ cp, const T *__restrict__ vp,
                                         const T *__restrict__ x, Pre &pre, Post &post, int urow = 0) {
  switch (w) {
    case 0: pre(); post(T(0)); return;
    case 1: sell_row_w<1, NT, UP>(cp, vp, x, pre, post, urow); return;
    case 2: sell_row_w<2, NT, UP>(cp, vp, x, pre, post, urow); return;
    case 3: sell_row_w<3, NT, UP>(cp, vp, x, pre, post, urow); return;
    case 4: sell_row_w<4, NT, UP>(cp, vp, x, pre, post, urow); return;
    case 5: sell_row_w<5, NT, UP>(cp, vp, x, pre, post, urow); return;
    case 6: sell_row_w<6, NT, UP>(cp, vp, x, pre, post, urow); return;
    case 7: sell_row_w<7, NT, UP>(cp, vp, x, pre, post, urow); return;
    case 8: sell_row_w<8, NT, UP>(cp, vp, x, pre, post, urow); return;
    case 9: sell_row_w<9, NT, UP>(cp, vp, x, pre, post, urow); return;
    case 10: sell_row_w<10, NT, UP>(cp, vp, x, pre, post, urow); return;
    case 11: sell_row_w<11, NT, UP>(cp, vp, x, pre, post, urow); return;
    case 12: sell_row_w<12, NT, UP>(cp, vp, x, pre, post, urow); return;
    case 13: sell_row_w<13, NT, UP>(cp, vp, x, pre, post, urow); return;
    case 14: sell_row_w<14, NT, UP>(cp, vp, x, pre, post, urow); return;
    case 15: sell_row_w<15, NT, UP>(cp, vp, x, pre, post, urow); return;
    case 16: sell_row_w<16, NT, UP>(cp, vp, x, pre, post, urow); return;
    default: break;
  }
  if constexpr (WMAX > 16) {
    switch (w) {
      case 17: sell_row_w<17, NT, UP>(cp, vp, x, pre, post, urow); return;
      case 18: sell_row_w<18, NT, UP>(cp, vp, x, pre, post, urow); return;
      case 19: sell_row_w<19, NT, UP>(cp, vp, x, pre, post, urow); return;
      case 20: sell_row_w<20, NT, UP>(cp, vp, x, pre, post, urow); return;
      case 21: sell_row_w<21, NT, UP>(cp, vp, x, pre, post, urow); return;
      case 22: sell_row_w<22, NT, UP>(cp, vp, x, pre, post, urow); return;
      case 23: sell_row_w<23, NT, UP>(cp, vp, x, pre, post, urow); return;
      case 24: sell_row_w<24, NT, UP>(cp, vp, x, pre, post, urow); return;
      case 25: sell_row_w<25, NT, UP>(cp, vp, x, pre, post, urow); return;
      case 26: sell_row_w<26, NT, UP>(cp, vp, x, pre, post, urow); return;
      case 27: sell_row_w<27, NT, UP>(cp, vp, x, pre, post, urow); return;
      case 28: sell_row_w<28, NT, UP>(cp, vp, x, pre, post, urow); return;
      case 29: sell_row_w<29, NT, UP>(cp, vp, x, pre, post, urow); return;
      case 30: sell_row_w<30, NT, UP>(cp, vp, x, pre, post, urow); return;
      case 31: sell_row_w<31, NT, UP>(cp, vp, x, pre, post, urow); return;
      case 32: sell_row_w<32, NT, UP>(cp, vp, x, pre, post, urow); return;
      default: break;
    }
  }
  // long rows: chunks of 8 entries, each with its loads issued together
  pre();
  T acc = 0;
  int k = 0;
  for (; k + 8 <= w; k += 8) acc += sell_chunk<8, NT, UP>(cp + k * 64, vp + k * 64, x, urow);
  for (; k < w; ++k) {
    const int ck = cp[k * 64];
    if (!UP || ck > urow) acc += vp[k * 64] * x[ck];
  }
  post(acc);
}

// wave-uniform slice index of this wave (scalar registers, so the slice header is a scalar load)
__device__ __forceinline__ int wave_slice(int first) {
  return first + xcd_block() * (BS / 64) + __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
}

// MODE 0: Gauss-Seidel pass x_i = (b_i - sum_{j != i} a_ij x_j) / a_ii
// MODE 1: residual r_i = b_i - a_ii x_i - sum_{j != i} a_ij x_j
// (dv_ holds 1/a_ii for MODE 0 and a_ii for MODE 1)
// MODE 2: residual after a single forward sweep from x = 0, r_i = -sum_{j > i} a_ij x_j. When the
// pass of row i's colour ran, every later colour was still zero and every earlier one final, so
// b_i - a_ii x_i - sum_{j < i} a_ij x_j = 0 from then on (rows are numbered colour by colour);
// only the later colours' terms remain. Slice s starts at shi[s] (passed as soff), the widest
// prefix of entries that lie before the row in every lane; b, dv_ and x_i are not read.
template <int MODE, class T, int VAR = 0>
__global__ __launch_bounds__(BS_MAX) void k_sell(int s0, int s1, const int *__restrict__ srow,
                                                 const int *__restrict__ soff, const int *__restrict__ send,
                                                 const int *__restrict__ scol,
                                                 const T *__restrict__ sv, const T *__restrict__ dv_,
                                                 const T *__restrict__ b, T *__restrict__ x, T *__restrict__ r,
                                                 int shape) {
  const int lane = threadIdx.x & 63;
  for_slices<VAR>(s0, s1, shape, srow, soff, send, [&](int row, int o0, int w) {
    T bi = 0, di = 0, xi = 0;
    auto pre = [&] {
      if (MODE == 2) return;
      const int rr = row < 0 ? 0 : row;
      bi = b[rr];
      di = dv_[rr];
      if (MODE == 1) xi = x[rr];
    };
    auto post = [&](T acc) {
      if (MODE != 2) {
        pin(bi);
        pin(di);
      }
      if (MODE == 1) pin(xi);
      if (row < 0) return;
      if (MODE == 0)
        x[row] = (bi - acc) * di;
      else if (MODE == 1)
        r[row] = bi - di * xi - acc;
      else
        r[row] = -acc;
    };
    sell_row<T, 16, false, MODE == 2>(w, scol + o0 + lane, sv + o0 + lane, x, pre, post, row);
  });
}

// transfer products on a sliced ELL (one colour class = all rows): y = A x (ADD = 0) or y += A x.
// FIRST (with ADD = 0): y is the right-hand side of a level whose smoothing starts from zero, and
// the kernel also runs that first colour pass: xs_i = y_i / a_ii for rows i < c0 (colour 0),
// xs_i = 0 for the other rows; with rc it also copies y into rc.
template <int ADD, int FIRST, class T, int WMAX = 16, int VAR = 0>
__global__ __launch_bounds__(BS_MAX) void k_sell_spmv(int ns, const int *__restrict__ srow, const int *__restrict__ soff,
                                                  const int *__restrict__ scol, const T *__restrict__ sv,
                                                  const T *__restrict__ x, T *__restrict__ y, int c0,
                                                  const T *__restrict__ invd, T *__restrict__ xs,
                                                  T *__restrict__ rc, int shape) {
  const int lane = threadIdx.x & 63;
  for_slices<VAR>(0, ns, shape, srow, soff, soff + 1, [&](int row, int o0, int w) {
    T yi = 0, di = 0;
    auto pre = [&] {
      const int rr = row < 0 ? 0 : row;
      if (ADD) yi = y[rr];
      if (FIRST && rr < c0) di = invd[rr];
    };
    auto post = [&](T acc) {
      if (ADD) pin(yi);
      if (FIRST) pin(di);
      if (row < 0) return;
      y[row] = ADD ? yi + acc : acc;
      if (FIRST) {
        xs[row] = row < c0 ? acc * di : T(0);
        if (rc) rc[row] = acc;
      }
    };
    sell_row<T, WMAX, true>(w, scol + o0 + lane, sv + o0 + lane, x, pre, post);
  });
}

// dense y = M g (M row-major n x n: the bottom inverse A_lc^{-1}, or a near-boundary set's
// inverse). One block per row: its 256 threads stride over the row with up to four loads in
// flight each, so that some 4n waves share the memory system (one wave per row, about a
// thousand waves at the bottom level, left most of the chip idle); a fixed-order block sum
// finishes the row. Launch with gemv() (grid = n blocks).
template <class T>
__global__ __launch_bounds__(BS) void k_gemv(int n, const T *__restrict__ M, const T *__restrict__ g,
                                             T *__restrict__ y) {
  const int row = blockIdx.x;
  const T *m = M + (size_t)row * n;
  T s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  int j = threadIdx.x;
  for (; j + 3 * BS < n; j += 4 * BS) {
    s0 += m[j] * g[j];
    s1 += m[j + BS] * g[j + BS];
    s2 += m[j + 2 * BS] * g[j + 2 * BS];
    s3 += m[j + 3 * BS] * g[j + 3 * BS];
  }
  for (; j < n; j += BS) s0 += m[j] * g[j];
  double v[1] = {(double)((s0 + s1) + (s2 + s3))};
  block_sum_n<1>(v);
  if (threadIdx.x == 0) y[row] = (T)v[0];
}

template <class T>
static void gemv(int n, const T *M, const T *g, T *y, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL((k_gemv<T>), dim3(n), dim3(BS), 0, s, n, M, g, y);
}

// ---------------------------------------------------------------------------
// PCG kernels (FP64 on the original grid)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(BS) void k_gather(int n, const int *__restrict__ perm, const double *__restrict__ src,
                                               double *__restrict__ dst) {
  const int i = blockIdx.x * BS + threadIdx.x;
  if (i < n) dst[i] = src[perm[i]];
}

__global__ __launch_bounds__(BS) void k_scatter(int n, const int *__restrict__ perm, const double *__restrict__ src,
                                                double *__restrict__ dst) {
  const int i = blockIdx.x * BS + threadIdx.x;
  if (i < n) dst[perm[i]] = src[i];
}

template <class T>
__global__ __launch_bounds__(BS) void k_scatter_cvt(int n, const int *__restrict__ perm, const T *__restrict__ src,
                                                    double *__restrict__ dst) {
  const int i = blockIdx.x * BS + threadIdx.x;
  if (i < n) dst[perm[i]] = (double)src[i];
}

// Reductions: a producer kernel runs a bounded grid-stride grid (at most RED_BLOCKS blocks, or
// the handle's smaller cap) and writes one partial per block; a one-block finalize kernel
// reduces the partials in a fixed order and updates the PCG scalars. No atomics, reproducible
// results.
static constexpr int RED_BLOCKS = 2048;

// r = f, u = 0, p = 0; partials of ||f||^2
__global__ __launch_bounds__(BS) void k_cg_init(int n, const double *__restrict__ f, double *__restrict__ r,
                                                double *__restrict__ u, double *__restrict__ p,
                                                double *__restrict__ partials) {
  double v = 0.0;
  for (int i = blockIdx.x * BS + threadIdx.x; i < n; i += gridDim.x * BS) {
    const double fi = f[i];
    r[i] = fi;
    u[i] = 0.0;
    p[i] = 0.0;
    v += fi * fi;
  }
  v = block_sum(v);
  if (threadIdx.x == 0) partials[blockIdx.x] = v;
}

__device__ __forceinline__ double sum_partials(const double *__restrict__ partials, int nb) {
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += BS) s += partials[i];
  return block_sum(s);
}

__global__ __launch_bounds__(BS) void k_fin_init(const double *__restrict__ partials, int nb, double tol, int maxit,
                                                 Ctl *ctl) {
  const double t = sum_partials(partials, nb);
  if (threadIdx.x == 0) {
    ctl->fnorm2 = t;
    ctl->tol2 = tol * tol * t;
    ctl->iter = 0;
    ctl->status = ST_OK;
    ctl->done = (t == 0.0) ? 1 : 0;
    ctl->first = 1;
    ctl->maxit = maxit;
  }
}

// restart from the true residual: r = f - A u, p = 0 (mixed precision)
template <int LPR>
__global__ __launch_bounds__(BS) void k_cg_restart(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                   const double *__restrict__ av, const double *__restrict__ dg,
                                                   const double *__restrict__ f, const double *__restrict__ u,
                                                   double *__restrict__ r, double *__restrict__ p, Ctl *ctl) {
  const int t = blockIdx.x * BS + threadIdx.x;
  const int row = t / LPR, lane = t % LPR;
  const bool act = row < n;
  const double s = row_dot<LPR>(rp, ci, av, u, row, act, lane);
  if (act && lane == 0) {
    r[row] = f[row] - dg[row] * u[row] - s;
    p[row] = 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->done = 0;
    ctl->first = 1;
  }
}

// partials of ||f - A u||^2 (grid-stride over row groups)
template <int LPR>
__global__ __launch_bounds__(BS) void k_true_res(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                 const double *__restrict__ av, const double *__restrict__ dg,
                                                 const double *__restrict__ f, const double *__restrict__ u,
                                                 double *__restrict__ partials) {
  constexpr int RPB = BS / LPR;
  const int lane = threadIdx.x % LPR;
  double v = 0.0;
  for (int base = blockIdx.x * RPB; base < n; base += gridDim.x * RPB) {
    const int row = base + threadIdx.x / LPR;
    const bool act = row < n;
    const double s = row_dot<LPR>(rp, ci, av, u, row, act, lane);
    if (act && lane == 0) {
      const double e = f[row] - dg[row] * u[row] - s;
      v += e * e;
    }
  }
  v = block_sum(v);
  if (threadIdx.x == 0) partials[blockIdx.x] = v;
}

__global__ __launch_bounds__(BS) void k_fin_tr(const double *__restrict__ partials, int nb, Ctl *ctl) {
  const double t = sum_partials(partials, nb);
  if (threadIdx.x == 0) ctl->tr = t;
}

// PCG start from a guess u: r = f - A u, p = 0, partials of ||r||^2 (grid-stride over row groups)
template <int LPR>
__global__ __launch_bounds__(BS) void k_cg_guess(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                 const double *__restrict__ av, const double *__restrict__ dg,
                                                 const double *__restrict__ f, const double *__restrict__ u,
                                                 double *__restrict__ r, double *__restrict__ p,
                                                 double *__restrict__ partials) {
  constexpr int RPB = BS / LPR;
  const int lane = threadIdx.x % LPR;
  double v = 0.0;
  for (int base = blockIdx.x * RPB; base < n; base += gridDim.x * RPB) {
    const int row = base + threadIdx.x / LPR;
    const bool act = row < n;
    const double s = row_dot<LPR>(rp, ci, av, u, row, act, lane);
    if (act && lane == 0) {
      const double e = f[row] - dg[row] * u[row] - s;
      r[row] = e;
      p[row] = 0.0;
      v += e * e;
    }
  }
  v = block_sum(v);
  if (threadIdx.x == 0) partials[blockIdx.x] = v;
}

// a guess that already meets the stopping rule ends the solve before its first iteration
__global__ __launch_bounds__(BS) void k_fin_guess(const double *__restrict__ partials, int nb, Ctl *ctl) {
  const double t = sum_partials(partials, nb);
  if (threadIdx.x == 0 && t <= ctl->tol2) ctl->done = 1;
}

// e += x
template <class T>
__global__ __launch_bounds__(BS) void k_add(int n, const T *__restrict__ x, T *__restrict__ e) {
  const int i = blockIdx.x * BS + threadIdx.x;
  if (i < n) e[i] += x[i];
}

// b = a, rounded to the destination type
template <class S, class D>
__global__ __launch_bounds__(BS) void k_convert(int n, const S *__restrict__ a, D *__restrict__ b) {
  const int i = blockIdx.x * BS + threadIdx.x;
  if (i < n) b[i] = (D)a[i];
}

// q = A p on the sliced ELL of the original grid (all colours); partials of p.q
__global__ __launch_bounds__(BS) void k_cg_spmv(int ns, const int *__restrict__ srow, const int *__restrict__ soff,
                                                const int *__restrict__ scol, const double *__restrict__ sv,
                                                const double *__restrict__ dg, const double *__restrict__ p,
                                                double *__restrict__ q, const Ctl *ctl,
                                                double *__restrict__ partials) {
  if (ctl->done) return;
  const int lane = threadIdx.x & 63;
  double v = 0.0;
  for (int s = wave_slice(0); s < ns; s += gridDim.x * (BS / 64)) {
    const int row = srow[(size_t)s * 64 + lane];
    const int o0 = soff[s];
    const int w = (soff[s + 1] - o0) >> 6;
    double pi = 0, di = 0;
    auto pre = [&] {
      const int rr = row < 0 ? 0 : row;
      pi = p[rr];
      di = dg[rr];
    };
    auto post = [&](double acc) {
      pin(pi);
      pin(di);
      if (row < 0) return;
      const double qi = di * pi + acc;
      q[row] = qi;
      v += pi * qi;
    };
    sell_row<double>(w, scol + o0 + lane, sv + o0 + lane, p, pre, post);
  }
  v = block_sum(v);
  if (threadIdx.x == 0) partials[blockIdx.x] = v;
}

// The PCG product with its x gathers staged in LDS (a measured alternative to k_cg_spmv, reached
// only through the kernel-timing entry point). A block owns tiles of BS/64 consecutive slices;
// the distinct columns of a tile's entries are listed at setup (tlist, sorted), the block loads
// p at those columns into LDS once, and each entry then reads LDS through its 16-bit position in
// the tile's list (lcol) instead of gathering p from global memory.
template <int W>
__device__ __forceinline__ double lds_row_w(const uint16_t *__restrict__ cp, const double *__restrict__ vp,
                                            const double *xs) {
  int c[W];
  double v[W];
#pragma unroll
  for (int k = 0; k < W; ++k) c[k] = cp[k * 64];
#pragma unroll
  for (int k = 0; k < W; ++k) v[k] = vp[k * 64];
  double a0 = 0, a1 = 0;
#pragma unroll
  for (int k = 0; k < W; ++k) {
    if (k & 1)
      a1 += v[k] * xs[c[k]];
    else
      a0 += v[k] * xs[c[k]];
  }
  return a0 + a1;
}

__device__ __forceinline__ double lds_row(int w, const uint16_t *__restrict__ cp, const double *__restrict__ vp,
                                          const double *xs) {
  switch (w) {
    case 0: return 0.0;
    case 1: return lds_row_w<1>(cp, vp, xs);
    case 2: return lds_row_w<2>(cp, vp, xs);
    case 3: return lds_row_w<3>(cp, vp, xs);
    case 4: return lds_row_w<4>(cp, vp, xs);
    case 5: return lds_row_w<5>(cp, vp, xs);
    case 6: return lds_row_w<6>(cp, vp, xs);
    case 7: return lds_row_w<7>(cp, vp, xs);
    case 8: return lds_row_w<8>(cp, vp, xs);
    case 9: return lds_row_w<9>(cp, vp, xs);
    case 10: return lds_row_w<10>(cp, vp, xs);
    case 11: return lds_row_w<11>(cp, vp, xs);
    case 12: return lds_row_w<12>(cp, vp, xs);
    case 13: return lds_row_w<13>(cp, vp, xs);
    case 14: return lds_row_w<14>(cp, vp, xs);
    case 15: return lds_row_w<15>(cp, vp, xs);
    case 16: return lds_row_w<16>(cp, vp, xs);
    default: break;
  }
  double acc = 0;
  int k = 0;
  for (; k + 8 <= w; k += 8) acc += lds_row_w<8>(cp + k * 64, vp + k * 64, xs);
  for (; k < w; ++k) acc += vp[k * 64] * xs[cp[k * 64]];
  return acc;
}

__global__ __launch_bounds__(BS) void k_cg_spmv_lds(int ntiles, int ns, const int *__restrict__ srow,
                                                    const int *__restrict__ soff, const uint16_t *__restrict__ lcol,
                                                    const double *__restrict__ sv, const int *__restrict__ toff,
                                                    const int *__restrict__ tlist, const double *__restrict__ dg,
                                                    const double *__restrict__ p, double *__restrict__ q,
                                                    double *__restrict__ partials) {
  extern __shared__ double xs[];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  double v = 0.0;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int b0 = toff[t], m = toff[t + 1] - b0;
    for (int k = threadIdx.x; k < m; k += BS) xs[k] = p[tlist[b0 + k]];
    const int sl = t * (BS / 64) + wv;
    int row = -1, o0 = 0, w = 0;
    if (sl < ns) {
      row = srow[(size_t)sl * 64 + lane];
      o0 = soff[sl];
      w = (soff[sl + 1] - o0) >> 6;
    }
    __syncthreads();
    const double acc = lds_row(w, lcol + o0 + lane, sv + o0 + lane, xs);
    if (row >= 0) {
      const double pi = p[row];
      const double qi = dg[row] * pi + acc;
      q[row] = qi;
      v += pi * qi;
    }
    __syncthreads();
  }
  v = block_sum(v);
  if (threadIdx.x == 0) partials[blockIdx.x] = v;
}

// alpha = rho / p.q, iteration count
__global__ __launch_bounds__(BS) void k_fin_spmv(const double *__restrict__ partials, int nb, Ctl *ctl) {
  if (ctl->done) return;
  const double pq = sum_partials(partials, nb);
  if (threadIdx.x == 0) {
    ctl->pq = pq;
    ctl->iter += 1;
    if (!(pq > 0.0) || !isfinite(pq)) {
      ctl->status = isfinite(pq) ? ST_NOTSPD : ST_NAN;
      ctl->done = 1;
    } else {
      ctl->alpha = ctl->rho / pq;
    }
  }
}

// u += alpha p, r -= alpha q; partials of ||r||^2. The same pass runs the colour-0 Gauss-Seidel
// pass of the next B_co application (sweep from zero) on the new r, in the precision T of B_co:
// xf_i = r_i / a_ii on colour-0 rows (i < c0), 0 elsewhere; in FP32 r is also rounded into bf.
template <class T>
__global__ __launch_bounds__(BS) void k_cg_axpy(int n, double *__restrict__ u, double *__restrict__ r,
                                                const double *__restrict__ p, const double *__restrict__ q,
                                                const Ctl *ctl, double *__restrict__ partials, int c0,
                                                const T *__restrict__ invd, T *__restrict__ bf, T *__restrict__ xf) {
  if (ctl->done) return;
  const double alpha = ctl->alpha;
  double v = 0.0;
  for (int i = blockIdx.x * BS + threadIdx.x; i < n; i += gridDim.x * BS) {
    u[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    v += ri * ri;
    if constexpr (sizeof(T) == 4) {
      const float bi = (float)ri;
      bf[i] = bi;
      xf[i] = i < c0 ? bi * invd[i] : 0.0f;
    } else {
      xf[i] = i < c0 ? ri * invd[i] : 0.0;
    }
  }
  v = block_sum(v);
  if (threadIdx.x == 0) partials[blockIdx.x] = v;
}

// convergence test on ||r||^2
__global__ __launch_bounds__(BS) void k_fin_axpy(const double *__restrict__ partials, int nb, Ctl *ctl) {
  if (ctl->done) return;
  const double rr = sum_partials(partials, nb);
  if (threadIdx.x == 0) {
    ctl->rr = rr;
    if (!isfinite(rr)) {
      ctl->status = ST_NAN;
      ctl->done = 1;
    } else if (rr <= ctl->tol2) {
      ctl->done = 1;
    } else if (ctl->iter >= ctl->maxit) {
      ctl->status = ST_NOCONV;
      ctl->done = 1;
    }
  }
}

// partials of r.z (z = B_co r in precision T)
template <class T>
__global__ __launch_bounds__(BS) void k_cg_rz(int n, const double *__restrict__ r, const T *__restrict__ z,
                                              const Ctl *ctl, double *__restrict__ partials) {
  if (ctl->done) return;
  double v = 0.0;
  for (int i = blockIdx.x * BS + threadIdx.x; i < n; i += gridDim.x * BS) v += r[i] * (double)z[i];
  v = block_sum(v);
  if (threadIdx.x == 0) partials[blockIdx.x] = v;
}

// rho' = r.z -> beta
__global__ __launch_bounds__(BS) void k_fin_rz(const double *__restrict__ partials, int nb, Ctl *ctl) {
  if (ctl->done) return;
  const double rz = sum_partials(partials, nb);
  if (threadIdx.x == 0) {
    ctl->rz = rz;
    if (!(rz > 0.0) || !isfinite(rz)) {
      ctl->status = isfinite(rz) ? ST_NOTSPD : ST_NAN;
      ctl->done = 1;
    } else if (ctl->first) {
      ctl->beta = 0.0;
      ctl->rho = rz;
      ctl->first = 0;
    } else {
      ctl->beta = rz / ctl->rho;
      ctl->rho = rz;
    }
  }
}

// p = z + beta p
template <class T>
__global__ __launch_bounds__(BS) void k_cg_p(int n, const T *__restrict__ z, double *__restrict__ p, const Ctl *ctl) {
  if (ctl->done) return;
  const double beta = ctl->beta;
  const int i = blockIdx.x * BS + threadIdx.x;
  if (i < n) p[i] = (double)z[i] + beta * p[i];
}

// Operator refresh from a new per-element coefficient: every matrix entry is a fixed list of
// (element, kappa-free element-matrix value) contributions, summed in element order.
__global__ __launch_bounds__(BS) void k_refresh_off(int nnz, const int *__restrict__ ptr, const int *__restrict__ el,
                                                    const double *__restrict__ w, const double *__restrict__ kappa,
                                                    double *__restrict__ v64, float *__restrict__ v32) {
  const int p = blockIdx.x * BS + threadIdx.x;
  if (p >= nnz) return;
  double s = 0.0;
  for (int q = ptr[p]; q < ptr[p + 1]; ++q) s += w[q] * kappa[el[q]];
  v64[p] = s;
  v32[p] = (float)s;
}

__global__ __launch_bounds__(BS) void k_refresh_diag(int n, const int *__restrict__ ptr, const int *__restrict__ el,
                                                     const double *__restrict__ w, const double *__restrict__ kappa,
                                                     double *__restrict__ dg64, double *__restrict__ id64,
                                                     float *__restrict__ dg32, float *__restrict__ id32) {
  const int i = blockIdx.x * BS + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int q = ptr[i]; q < ptr[i + 1]; ++q) s += w[q] * kappa[el[q]];
  dg64[i] = s;
  id64[i] = 1.0 / s;
  dg32[i] = (float)s;
  id32[i] = 1.0f / (float)s;
}

__global__ __launch_bounds__(BS) void k_refresh_sell(int nslots, const int *__restrict__ map,
                                                     const double *__restrict__ v64, double *__restrict__ s64,
                                                     float *__restrict__ s32) {
  const int t = blockIdx.x * BS + threadIdx.x;
  if (t >= nslots) return;
  const int p = map[t];
  const double v = p >= 0 ? v64[p] : 0.0;
  s64[t] = v;
  s32[t] = (float)v;
}

// plain y = A x (diag + off), for the matvec entry point
template <int LPR>
__global__ __launch_bounds__(BS) void k_matvec(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                               const double *__restrict__ av, const double *__restrict__ dg,
                                               const double *__restrict__ x, double *__restrict__ y) {
  const int t = blockIdx.x * BS + threadIdx.x;
  const int row = t / LPR, lane = t % LPR;
  const bool act = row < n;
  const double s = row_dot<LPR>(rp, ci, av, x, row, act, lane);
  if (act && lane == 0) y[row] = dg[row] * x[row] + s;
}

// per-element g_e = scale kappa_e lam_e^T K1_e u_e (u, lam per unknown in unknown order; scale 1
// for the derivative of lam^T A u in m_e = log kappa_e, -1 for the adjoint gradient)
template <int D>
__global__ __launch_bounds__(BS) void k_elem_grad(int ne, const double *__restrict__ coords,
                                                  const int *__restrict__ elems, const double *__restrict__ kappa,
                                                  const int *__restrict__ dof_of_vertex, const double *__restrict__ u,
                                                  const double *__restrict__ lam, double *__restrict__ g,
                                                  double scale) {
  const int e = blockIdx.x * BS + threadIdx.x;
  if (e >= ne) return;
  constexpr int K = D + 1;
  int v[K];
  double ue[K], le[K];
  for (int i = 0; i < K; ++i) {
    v[i] = elems[(size_t)e * K + i];
    const int di = dof_of_vertex[v[i]];
    ue[i] = di >= 0 ? u[di] : 0.0;
    le[i] = di >= 0 ? lam[di] : 0.0;
  }
  double M[3][3], G[K][3];
  for (int k = 0; k < D; ++k)
    for (int r = 0; r < D; ++r) M[r][k] = coords[(size_t)v[k + 1] * D + r] - coords[(size_t)v[0] * D + r];
  double det;
  double inv[3][3];
  if (D == 2) {
    det = M[0][0] * M[1][1] - M[0][1] * M[1][0];
    inv[0][0] = M[1][1] / det;
    inv[0][1] = -M[0][1] / det;
    inv[1][0] = -M[1][0] / det;
    inv[1][1] = M[0][0] / det;
  } else {
    double c[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const int r0 = (j + 1) % 3, r1 = (j + 2) % 3, c0 = (i + 1) % 3, c1 = (i + 2) % 3;
        c[i][j] = M[r0][c0] * M[r1][c1] - M[r0][c1] * M[r1][c0];
      }
    det = M[0][0] * c[0][0] + M[0][1] * c[1][0] + M[0][2] * c[2][0];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) inv[i][j] = c[i][j] / det;
  }
  for (int k = 0; k < D; ++k)
    for (int r = 0; r < D; ++r) G[k + 1][r] = inv[k][r];
  for (int r = 0; r < D; ++r) {
    double s = 0;
    for (int k = 0; k < D; ++k) s += inv[k][r];
    G[0][r] = -s;
  }
  const double vol = fabs(det) / (D == 2 ? 2.0 : 6.0);
  // lam^T G G^T u = (G^T lam) . (G^T u)
  double gl[3] = {0, 0, 0}, gu[3] = {0, 0, 0};
  for (int i = 0; i < K; ++i)
    for (int r = 0; r < D; ++r) {
      gl[r] += G[i][r] * le[i];
      gu[r] += G[i][r] * ue[i];
    }
  double s = 0;
  for (int r = 0; r < D; ++r) s += gl[r] * gu[r];
  g[e] = scale * (kappa[e] * vol * s);
}

// kappa_e = exp(m_e)
__global__ __launch_bounds__(BS) void k_exp(int ne, const double *__restrict__ m, double *__restrict__ kappa) {
  const int e = blockIdx.x * BS + threadIdx.x;
  if (e < ne) kappa[e] = exp(m[e]);
}

// ---------------------------------------------------------------------------
// pure Neumann problems: the mean of a vector and its removal
// ---------------------------------------------------------------------------

// partials of sum_i x_i (grid-stride)
__global__ __launch_bounds__(BS) void k_sum(int n, const double *__restrict__ x, double *__restrict__ partials) {
  double v = 0.0;
  for (int i = blockIdx.x * BS + threadIdx.x; i < n; i += gridDim.x * BS) v += x[i];
  v = block_sum(v);
  if (threadIdx.x == 0) partials[blockIdx.x] = v;
}

__global__ __launch_bounds__(BS) void k_fin_mean(const double *__restrict__ partials, int nb, int n, Ctl *ctl) {
  const double t = sum_partials(partials, nb);
  if (threadIdx.x == 0) ctl->mean = t / (double)n;
}

// x -= mean (the projection onto the vectors with zero sum)
__global__ __launch_bounds__(BS) void k_sub_mean(int n, double *__restrict__ x, const Ctl *ctl) {
  const int i = blockIdx.x * BS + threadIdx.x;
  if (i < n) x[i] -= ctl->mean;
}

// ---------------------------------------------------------------------------
// near-boundary correction (Section 3.5, Algorithm 3): e|_J += (A|_JJ)^-1 (g - A e)|_J
// Positions k of J are in the solver's order; jrow[k] is the level's internal row.
// ---------------------------------------------------------------------------

// rJ_k = g_i - a_ii e_i - sum_{j != i} a_ij e_j, i = jrow[k] (sliced ELL over the positions)
template <class T>
__global__ __launch_bounds__(BS) void k_nb_res(int ns, const int *__restrict__ srow, const int *__restrict__ soff,
                                               const int *__restrict__ scol, const T *__restrict__ sv,
                                               const int *__restrict__ jrow, const T *__restrict__ dg,
                                               const T *__restrict__ g, const T *__restrict__ e, T *__restrict__ rJ) {
  const int lane = threadIdx.x & 63;
  for_slices<0>(0, ns, 2 * (BS / 64) + 1, srow, soff, soff + 1, [&](int k, int o0, int w) {
    T gi = 0, di = 0, ei = 0;
    auto pre = [&] {
      const int i = jrow[k < 0 ? 0 : k];
      gi = g[i];
      di = dg[i];
      ei = e[i];
    };
    auto post = [&](T acc) {
      pin(gi);
      pin(di);
      pin(ei);
      if (k >= 0) rJ[k] = gi - di * ei - acc;
    };
    sell_row<T>(w, scol + o0 + lane, sv + o0 + lane, e, pre, post);
  });
}

// one wave per row i of the interiors: s = sum_j B_p[i - q0, j] in[q0 + j] over the dense inverse
// of row i's piece p; out_i = s, or base_i - s
template <class T>
__global__ __launch_bounds__(BS) void k_nb_blk(int nI, const int *__restrict__ rowpiece, const int *__restrict__ poff,
                                               const int64_t *__restrict__ boff, const T *__restrict__ blk,
                                               const T *__restrict__ in, const T *__restrict__ base,
                                               T *__restrict__ out) {
  const int i = blockIdx.x * (BS / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= nI) return;  // the whole wave leaves together
  const int p = rowpiece[i], q0 = poff[p], m = poff[p + 1] - q0;
  const T *B = blk + boff[p] + (int64_t)(i - q0) * m;
  T acc = 0;
  for (int j = lane; j < m; j += 64) acc += B[j] * in[q0 + j];
  acc = group_sum<64>(acc);
  if (lane == 0) out[i] = base ? base[i] - acc : acc;
}

// one thread per row of a small CSR coupling: out_i = s or base_i - s, s = sum_p v_p x[ci_p]
template <class T>
__global__ __launch_bounds__(BS) void k_nb_csr(int nrows, const int *__restrict__ rp, const int *__restrict__ ci,
                                               const T *__restrict__ v, const T *__restrict__ x,
                                               const T *__restrict__ base, T *__restrict__ out) {
  const int i = blockIdx.x * BS + threadIdx.x;
  if (i >= nrows) return;
  T acc = 0;
  for (int p = rp[i]; p < rp[i + 1]; ++p) acc += v[p] * x[ci[p]];
  out[i] = base ? base[i] - acc : acc;
}

// e_i += xJ_k, i = jrow[k] (distinct rows)
template <class T>
__global__ __launch_bounds__(BS) void k_nb_add(int n, const int *__restrict__ jrow, const T *__restrict__ xJ,
                                               T *__restrict__ e) {
  const int k = blockIdx.x * BS + threadIdx.x;
  if (k < n) e[jrow[k]] += xJ[k];
}

// ---------------------------------------------------------------------------
// device data
// ---------------------------------------------------------------------------

struct DSell;
using Ranges = std::vector<std::pair<int, int>>;  // row ranges [first, second)
struct DCsr {
  int nrows = 0, ncols = 0;
  int64_t nnz = 0;
  int *rp = nullptr, *ci = nullptr;
  double *v64 = nullptr;
  float *v32 = nullptr;
  int lpr = 4;
  DSell *sell = nullptr;       // sliced ELL copy used by the transfer products
  // transfers inside B_co (whole-level smoothing): the prolongation without the rows of the target
  // level's last colour (the first backward pass overwrites them unread), the restriction without
  // the columns of the source level's last colour (its residual is zero there); null = use `sell`
  DSell *vsell = nullptr;
};

struct DSell {
  int nslices = 0;
  int wmax = 0;               // widest slice (entries per row)
  std::vector<int> cslice;    // slice range of each colour, C + 1 (host)
  int *srow = nullptr, *soff = nullptr, *scol = nullptr;
  int *slo = nullptr;         // per slice: end of its entries before the group's first row
  int *shi = nullptr;         // per slice: end of the narrowest such prefix over its rows
  double *sv64 = nullptr;
  float *sv32 = nullptr;
  int64_t entries = 0;        // stored entries including padding
  int64_t nnz = 0;            // byte model: nonzeros, rows, distinct columns referenced
  int nrows = 0, ncols_used = 0;
};

// near-boundary set of an auxiliary level on the device (positions in the solver's order)
struct DNb {
  int n = 0, nI = 0, nS = 0, P = 0;
  bool dense = true;
  int *jrow = nullptr;                 // internal level row of each position
  DSell sell;                          // off-diagonal rows of A_l at the positions (srow = position)
  int64_t nnz = 0;                     // byte model
  double *inv64 = nullptr;             // dense path: n x n inverse
  float *inv32 = nullptr;
  int *rowpiece = nullptr, *poff = nullptr;  // decomposition: piece of each interior row, offsets
  int64_t *boff = nullptr;
  double *blk64 = nullptr, *asi64 = nullptr, *ais64 = nullptr, *sinv64 = nullptr;
  float *blk32 = nullptr, *asi32 = nullptr, *ais32 = nullptr, *sinv32 = nullptr;
  int *asi_rp = nullptr, *asi_ci = nullptr, *ais_rp = nullptr, *ais_ci = nullptr;
  int64_t nblk = 0, nasi = 0, nais = 0;
  double *r64 = nullptr, *x64 = nullptr, *y64 = nullptr, *t64 = nullptr;  // work vectors
  float *r32 = nullptr, *x32 = nullptr, *y32 = nullptr, *t32 = nullptr;
};

struct DLevel {
  int n = 0;
  DSell sell;                 // off-diagonal part of the smoothed rows, one slice group per range below
  std::vector<int> coff;      // colour offsets, C + 1
  int C = 0;                  // colours; Gauss-Seidel pass c runs slice group c
  // slice groups: colour c (full smoothing), or with local smoothing (auxiliary levels) first the
  // rows of N~ in colour c (groups 0..C-1, the smoothed rows), then the other rows of N~+ (rows
  // coupled to N~) in colour c (groups C..2C-1): the residual runs over all groups
  Ranges groups;
  int first_rows = 0;         // rows [0, first_rows): colour-0 rows of the first pass from zero
  bool local = false;         // local smoothing: r is written only on N~+, elsewhere r = b
  std::vector<int64_t> cnnz;  // off-diagonal nonzeros of each group's rows
  std::vector<int64_t> ucols; // distinct columns referenced by each group's rows
  std::vector<int64_t> cnnz_lo, ucols_lo;  // the same over columns before the group's first row
  std::vector<int64_t> cnnz_up, ucols_up;  // the same over columns after the group's last row
  std::vector<int> perm;      // internal -> unknown
  std::vector<int> iperm;     // unknown -> internal
  DCsr A;                     // off-diagonal part
  double *dg64 = nullptr, *id64 = nullptr;
  float *dg32 = nullptr, *id32 = nullptr;
  double *x64 = nullptr, *b64 = nullptr, *r64 = nullptr;
  float *x32 = nullptr, *b32 = nullptr, *r32 = nullptr;
  double *ng64 = nullptr, *ne64 = nullptr;  // nested iteration: load vector g_l and iterate e_l
  float *ng32 = nullptr, *ne32 = nullptr;
  DCsr P, PT;                 // from the next coarser level (aux levels only)
  DNb nb;                     // near-boundary correction (n = 0: none)
};

struct Device {
  std::vector<std::unique_ptr<DSell>> sells;  // sliced ELL copies of the transfers
  int ordinal = 0;
  int d = 2;
  int J = 1, lc = 1;
  int nu_aux = 2, nu_fine = 1, maxit = 1000, precision = 0, check_every = 0;
  std::vector<void *> allocs;
  DLevel fine;
  std::vector<DLevel> aux;    // index l (lc+1..J used)
  DCsr Pi, PiT;
  int nc = 0;
  double *cinv64 = nullptr, *cb64 = nullptr, *cx64 = nullptr;
  float *cinv32 = nullptr, *cb32 = nullptr, *cx32 = nullptr;
  double *cng64 = nullptr, *cne64 = nullptr;  // nested iteration at the bottom level
  float *cng32 = nullptr, *cne32 = nullptr;
  int nested = 0;             // V-cycles per level of the nested iteration (0 = u_0 = 0)
  bool pure_neumann = false;  // every vertex an unknown: A singular, f projected, u mean-free
  int *perm_d = nullptr;      // fine internal -> unknown
  // PCG vectors (internal order, FP64)
  double *f = nullptr, *u = nullptr, *r = nullptr, *p = nullptr, *q = nullptr;
  double *io_in = nullptr, *io_out = nullptr;   // staging for host-pointer calls
  Ctl *ctl = nullptr;
  Ctl *ctl_host = nullptr;    // pinned
  double *partials = nullptr;
  int max_blocks = 1;          // cap of the reduction grids (grid-stride loops beyond it)
  int restarts = 0;            // restarts from the true residual in the last solve
  int solve_iters = 0;         // PCG iterations of the last solve
  // operator refresh from a device coefficient (original grid)
  int *rf_off_ptr = nullptr, *rf_off_el = nullptr, *rf_dg_ptr = nullptr, *rf_dg_el = nullptr, *rf_sell_map = nullptr;
  double *rf_off_w = nullptr, *rf_dg_w = nullptr;
  int rf_nslots = 0;
  bool rf_ready = false;      // the refresh maps are built at the first device coefficient refresh
  // element data for the gradient
  double *coords = nullptr, *kappa = nullptr;
  int *elems = nullptr, *dof_of_vertex = nullptr;
  int64_t ne = 0, nv = 0;
  // execution: an internal stream carries the PCG loop (joined to the caller's stream with
  // events); one PCG iteration is captured per precision as a HIP graph
  hipStream_t stream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  // launch shapes of the V-cycle slice kernels per precision and launch site (the k-th slice
  // launch of one B_co application), chosen by the autotuner at the first solve
  std::vector<Shape> shape[2];  // (threads per block, xcd order, kernel variant)
  std::vector<std::vector<float>> tune_times[2];  // autotuner: best ms per site and candidate
  bool tuned[2] = {false, false};
  bool tuning = false;
  int site = 0, shape_pi = 0;
  int autotune = 1;
  int tune_k = 0, tune_live = 0;       // autotuner: candidate under trial, sites seen
  std::vector<hipEvent_t> tune_ev;     // two events per launch site
  std::vector<uint8_t> tune_has;       // site launched something
  int last_iters[2] = {0, 0};
  bool use_graph = true;
  bool no_alloc = false;      // inside asmg_solve_device_noalloc: no autotuning, no graph
  // byte model accumulation, and per-launch HIP event timing of one GS kernel instance
  bool count_bytes = false;
  double bytes = 0.0;
  int probe_lpr = 0, probe_prec = -1;          // GS launches to bracket with events (0 = none)
  std::vector<hipEvent_t> probe_ev;            // pairs (start, stop)
  std::vector<double> probe_bytes;
  size_t probe_used = 0;
  std::string last_kernel;
  // LDS-staged PCG product (kernel-timing mode 7 only): per tile of BS/64 slices the sorted
  // distinct columns, their offsets, and each entry's position in its tile's list
  int *lds_toff = nullptr, *lds_list = nullptr;
  uint16_t *lds_lcol = nullptr;
  int lds_ntiles = 0, lds_maxm = 0;
  int64_t lds_nlist = 0;
};

template <class T>
static T *dalloc(Device *dv, int64_t n) {
  if (n <= 0) n = 1;
  void *p = nullptr;
  HIPCHECK(hipMalloc(&p, (size_t)n * sizeof(T)));
  dv->allocs.push_back(p);
  return (T *)p;
}

template <class T>
static T *dupload(Device *dv, const std::vector<T> &v) {
  T *p = dalloc<T>(dv, (int64_t)v.size());
  if (!v.empty()) HIPCHECK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return p;
}


// host CSR triple in an internal numbering
struct HCsr {
  int nrows = 0, ncols = 0;
  std::vector<int> rp, ci;
  std::vector<double> v;
};

// permute rows/cols of a host CSR: new row i = old row rperm[i]; column c -> cmap[c]; optional diagonal split
static HCsr permute(const Csr &A, const std::vector<int> &rperm, const std::vector<int> *cmap, bool split_diag,
                    std::vector<double> *diag) {
  HCsr B;
  B.nrows = (int)rperm.size();
  B.ncols = (int)A.ncols;
  B.rp.assign(B.nrows + 1, 0);
  if (diag) diag->assign(B.nrows, 0.0);
  std::vector<std::pair<int, double>> row;
  for (int i = 0; i < B.nrows; ++i) {
    const int64_t o = rperm[i];
    row.clear();
    for (int64_t p = A.rp[o]; p < A.rp[o + 1]; ++p) {
      if (split_diag && A.ci[p] == o) {
        (*diag)[i] = A.v[p];
        continue;
      }
      const int c = cmap ? (*cmap)[A.ci[p]] : A.ci[p];
      row.push_back({c, A.v[p]});
    }
    std::sort(row.begin(), row.end());
    for (auto &e : row) {
      B.ci.push_back(e.first);
      B.v.push_back(e.second);
    }
    B.rp[i + 1] = (int)B.ci.size();
  }
  return B;
}

static HCsr transpose(const HCsr &A) {
  HCsr T;
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

// host image of a sliced ELL: built on host threads, uploaded afterwards
struct SellHost {
  // slo[s]: end of the entries of slice s that lie before its group's first row in every lane
  // (the widest such prefix over the lanes; rows store their columns in ascending order);
  // shi[s]: end of the narrowest such prefix over the slice's rows (entries beyond it may still
  // lie before some lanes' group)
  std::vector<int> srow, soff, scol, cs, slo, shi;
  std::vector<double> sv;
  std::vector<float> sv32;
  int widest = 0;
};

static SellHost sell_host(const HCsr &H, const Ranges &groups, std::vector<int> *slot_map = nullptr,
                          int wround = 1, const std::vector<int> *order = nullptr);
static void sell_upload(Device *dv, DSell &S, const SellHost &X, bool first_time);

static void build_sell_ranges(Device *dv, DSell &S, const HCsr &H, const Ranges &groups, bool first_time,
                              std::vector<int> *slot_map = nullptr, int wround = 1,
                              const std::vector<int> *order = nullptr) {
  sell_upload(dv, S, sell_host(H, groups, slot_map, wround, order), first_time);
}

// sizes only: the kernels read the auxiliary levels and the transfers through their sliced ELL
// copies; only the original-grid operator keeps a device CSR (PCG products)
static void csr_shape(const HCsr &H, DCsr &D) {
  D.nrows = H.nrows;
  D.ncols = H.ncols;
  D.nnz = (int64_t)H.ci.size();
}

static void upload_csr(Device *dv, const HCsr &H, DCsr &D) {
  csr_shape(H, D);
  D.rp = dupload(dv, H.rp);
  D.ci = dupload(dv, H.ci);
  D.v64 = dupload(dv, H.v);
  std::vector<float> f(H.v.begin(), H.v.end());
  D.v32 = dupload(dv, f);
  D.lpr = pick_lpr(D.nnz, D.nrows);
}

static void upload_values(DCsr &D, const HCsr &H) {
  if (H.v.empty() || !D.v64) return;
  HIPCHECK(hipMemcpy(D.v64, H.v.data(), H.v.size() * sizeof(double), hipMemcpyHostToDevice));
  std::vector<float> f(H.v.begin(), H.v.end());
  HIPCHECK(hipMemcpy(D.v32, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
}

// A transfer product may visit its rows in any order (each row is written once), so its slices
// follow `order` (rows in a spatially coherent order: the level's Morton numbering, or Morton
// order of the vertices on the original grid): neighbouring rows then gather neighbouring
// entries of x, whereas the colour-major numbering would interleave four distant ranges.
struct SellStats {
  int64_t nnz = 0;
  int nrows = 0, ncols_used = 0;
};

struct TransferStage {
  int nrows = 0, ncols = 0;
  int64_t nnz = 0;
  SellHost sell, vsell;
  SellStats st, vst;
  bool has_v = false;
};

// byte-model counts of the rows `order` (all rows when null) of H
static SellStats sell_stats(const HCsr &H, const std::vector<int> *order) {
  SellStats st;
  std::vector<uint8_t> seen(std::max(H.ncols, 1), 0);
  auto row = [&](int i) {
    ++st.nrows;
    for (int p = H.rp[i]; p < H.rp[i + 1]; ++p) {
      ++st.nnz;
      if (!seen[H.ci[p]]) {
        seen[H.ci[p]] = 1;
        ++st.ncols_used;
      }
    }
  };
  if (order)
    for (int i : *order) row(i);
  else
    for (int i = 0; i < H.nrows; ++i) row(i);
  return st;
}

static void stage_transfer(const HCsr &H, const std::vector<int> *order, TransferStage &X) {
  X.nrows = H.nrows;
  X.ncols = H.ncols;
  X.nnz = (int64_t)H.ci.size();
  X.sell = sell_host(H, Ranges{{0, H.nrows}}, nullptr, 4, order);
  X.st = sell_stats(H, nullptr);
}

// The V-cycle's copy of a prolongation: the rows of `order` outside [skip0, skip1) (the target
// level's last colour, which the first backward pass overwrites without reading).
static void stage_prolong_v(const HCsr &H, const std::vector<int> &order, int skip0, int skip1, TransferStage &X) {
  std::vector<int> keep;
  keep.reserve(order.size());
  for (int i : order)
    if (i < skip0 || i >= skip1) keep.push_back(i);
  X.vsell = sell_host(H, Ranges{{0, (int)keep.size()}}, nullptr, 4, &keep);
  X.vst = sell_stats(H, &keep);
  X.has_v = true;
}

// The V-cycle's copy of a restriction: without the entries of columns in [skip0, skip1) (the
// source level's last colour, where the residual it restricts is zero after a forward sweep).
static void stage_restrict_v(const HCsr &H, const std::vector<int> *order, int skip0, int skip1, TransferStage &X) {
  HCsr R;
  R.nrows = H.nrows;
  R.ncols = H.ncols;
  R.rp.assign(H.nrows + 1, 0);
  for (int i = 0; i < H.nrows; ++i) {
    for (int p = H.rp[i]; p < H.rp[i + 1]; ++p)
      if (H.ci[p] < skip0 || H.ci[p] >= skip1) {
        R.ci.push_back(H.ci[p]);
        R.v.push_back(H.v[p]);
      }
    R.rp[i + 1] = (int)R.ci.size();
  }
  X.vsell = sell_host(R, Ranges{{0, R.nrows}}, nullptr, 4, order);
  X.vst = sell_stats(R, nullptr);
  X.has_v = true;
}

static DSell *upload_stage_sell(Device *dv, const SellHost &H, const SellStats &st) {
  dv->sells.emplace_back(new DSell());
  DSell *S = dv->sells.back().get();
  sell_upload(dv, *S, H, true);
  S->nnz = st.nnz;
  S->nrows = st.nrows;
  S->ncols_used = st.ncols_used;
  return S;
}

static void commit_transfer(Device *dv, const TransferStage &X, DCsr &D) {
  D.nrows = X.nrows;
  D.ncols = X.ncols;
  D.nnz = X.nnz;
  D.sell = upload_stage_sell(dv, X.sell, X.st);
  if (X.has_v) D.vsell = upload_stage_sell(dv, X.vsell, X.vst);
}

// colour-major numbering: colour classes in order, inside a class ascending (part, rank), with
// rank the unknown id when null and part 0 when null. Sets coff, C, the full-smoothing slice
// groups (one per colour) and the colour-0 prefix of the first pass.
static void colour_order(const std::vector<int32_t> &col, DLevel &L, const std::vector<int> *rank = nullptr,
                         const std::vector<uint8_t> *part = nullptr) {
  const int n = (int)col.size();
  L.n = n;
  int C = 0;
  for (int c : col) C = std::max(C, c + 1);
  L.C = C;
  L.coff.assign(C + 1, 0);
  for (int c : col) L.coff[c + 1]++;
  for (int c = 0; c < C; ++c) L.coff[c + 1] += L.coff[c];
  std::vector<int> seq(n);
  if (rank)
    for (int i = 0; i < n; ++i) seq[(*rank)[i]] = i;
  else
    std::iota(seq.begin(), seq.end(), 0);
  if (part) std::stable_sort(seq.begin(), seq.end(), [&](int a, int b) { return (*part)[a] < (*part)[b]; });
  L.perm.resize(n);
  std::vector<int> pos(L.coff.begin(), L.coff.end() - 1);
  for (int i : seq) L.perm[pos[col[i]]++] = i;
  L.iperm.resize(n);
  for (int i = 0; i < n; ++i) L.iperm[L.perm[i]] = i;
  L.groups.clear();
  for (int c = 0; c < C; ++c) L.groups.push_back({L.coff[c], L.coff[c + 1]});
  L.first_rows = C > 0 ? L.coff[1] : 0;
  L.local = false;
}

// Local smoothing on an auxiliary level: rows of N~ first, then the rest of N~+ (N~ and the rows
// coupled to it in A_l), inside every colour; the slice groups cover N~ (smoothing) and then
// the rest of N~+ (residual only).
static void local_order(const std::vector<int32_t> &col, const std::vector<uint8_t> &nt, const Csr &A, DLevel &L) {
  const int n = (int)col.size();
  std::vector<uint8_t> part(n, 2);
  for (int i = 0; i < n; ++i)
    if (nt[i]) {
      part[i] = 0;
      for (int64_t p = A.rp[i]; p < A.rp[i + 1]; ++p)
        if (!nt[A.ci[p]]) part[A.ci[p]] = 1;
    }
  colour_order(col, L, nullptr, &part);
  std::vector<int> cnt0(L.C, 0), cnt1(L.C, 0);
  for (int i = 0; i < n; ++i) {
    if (part[i] == 0) ++cnt0[col[i]];
    if (part[i] == 1) ++cnt1[col[i]];
  }
  L.groups.clear();
  for (int c = 0; c < L.C; ++c) L.groups.push_back({L.coff[c], L.coff[c] + cnt0[c]});
  for (int c = 0; c < L.C; ++c) L.groups.push_back({L.coff[c] + cnt0[c], L.coff[c] + cnt0[c] + cnt1[c]});
  L.first_rows = L.C > 0 ? cnt0[0] : 0;
  L.local = true;
}

static void alloc_vectors(Device *dv, DLevel &L) {
  L.x64 = dalloc<double>(dv, L.n);
  L.b64 = dalloc<double>(dv, L.n);
  L.r64 = dalloc<double>(dv, L.n);
  L.x32 = dalloc<float>(dv, L.n);
  L.b32 = dalloc<float>(dv, L.n);
  L.r32 = dalloc<float>(dv, L.n);
  // the residual kernel never writes the last colour's rows (zero after a forward sweep)
  HIPCHECK(hipMemset(L.r64, 0, (size_t)std::max(L.n, 1) * 8));
  HIPCHECK(hipMemset(L.r32, 0, (size_t)std::max(L.n, 1) * 4));
}

// sliced ELL of a host CSR: one slice group per row range (a colour class, or part of one),
// rows sorted by length inside windows of 256 rows, 64 rows per slice. Slice widths above 16 are
// rounded up to a multiple of `wround` (extra zero entries), so that matrices with long, uneven
// rows use a few of the kernel's straight-line widths rather than many. With `order` (one range
// only), position i of the range is row order[i].
static SellHost sell_host(const HCsr &H, const Ranges &groups, std::vector<int> *slot_map, int wround,
                          const std::vector<int> *order) {
  if (slot_map) slot_map->clear();
  const int C = (int)groups.size();
  SellHost X;
  std::vector<int> &srow = X.srow, &soff = X.soff, &scol = X.scol, &cs = X.cs;
  std::vector<double> &sv = X.sv;
  soff.push_back(0);
  cs.push_back(0);
  std::vector<int> idx;
  int &widest = X.widest;
  for (int c = 0; c < C; ++c) {
    for (int w0 = groups[c].first; w0 < groups[c].second; w0 += 256) {
      const int w1 = std::min(w0 + 256, groups[c].second);
      idx.resize(w1 - w0);
      std::iota(idx.begin(), idx.end(), w0);
      if (order)
        for (int &i : idx) i = (*order)[i];
      std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
        return (H.rp[a + 1] - H.rp[a]) > (H.rp[b + 1] - H.rp[b]);
      });
      for (size_t s0 = 0; s0 < idx.size(); s0 += 64) {
        const size_t s1 = std::min(s0 + 64, idx.size());
        int wmax = 0, wlo = 0, whi = INT_MAX;
        for (size_t i = s0; i < s1; ++i) {
          const int r = idx[i];
          wmax = std::max(wmax, H.rp[r + 1] - H.rp[r]);
          int lo = 0;
          while (H.rp[r] + lo < H.rp[r + 1] && H.ci[H.rp[r] + lo] < groups[c].first) ++lo;
          wlo = std::max(wlo, lo);
          whi = std::min(whi, lo);
        }
        if (wmax > 16) wmax = (wmax + wround - 1) / wround * wround;
        const int base = soff.back();
        scol.resize(base + 64 * wmax);
        sv.resize(base + 64 * wmax);
        for (int lane = 0; lane < 64; ++lane) {
          const size_t i = s0 + lane;
          const int row = i < s1 ? idx[i] : -1;
          srow.push_back(row);
          for (int k = 0; k < wmax; ++k) {
            int cc = 0;  // padding: column 0 with value 0 (a valid index of x)
            double v = 0.0;
            if (row >= 0 && k < H.rp[row + 1] - H.rp[row]) {
              cc = H.ci[H.rp[row] + k];
              v = H.v[H.rp[row] + k];
            } else if (row >= 0 && H.rp[row + 1] > H.rp[row]) {
              cc = H.ci[H.rp[row]];  // repeat the row's first column: no extra cache line
            }
            scol[base + 64 * k + lane] = cc;
            sv[base + 64 * k + lane] = v;
            if (slot_map) {
              if ((int)slot_map->size() < base + 64 * wmax) slot_map->resize(base + 64 * wmax, -1);
              (*slot_map)[base + 64 * k + lane] =
                  (row >= 0 && k < H.rp[row + 1] - H.rp[row]) ? H.rp[row] + k : -1;
            }
          }
        }
        soff.push_back(base + 64 * wmax);
        X.slo.push_back(base + 64 * std::min(wlo, wmax));
        X.shi.push_back(base + 64 * std::min(whi, wmax));
        widest = std::max(widest, wmax);
      }
    }
    cs.push_back((int)srow.size() / 64);
  }
  X.sv32.assign(sv.begin(), sv.end());
  return X;
}

static void sell_upload(Device *dv, DSell &S, const SellHost &X, bool first_time) {
  if (first_time) {
    S.nslices = (int)X.srow.size() / 64;
    S.wmax = X.widest;
    S.cslice = X.cs;
    S.entries = (int64_t)X.sv.size();
    S.srow = dupload(dv, X.srow);
    S.soff = dupload(dv, X.soff);
    S.slo = dupload(dv, X.slo);
    S.shi = dupload(dv, X.shi);
    S.scol = dupload(dv, X.scol);
    S.sv64 = dupload(dv, X.sv);
    S.sv32 = dupload(dv, X.sv32);
  } else if (!X.sv.empty()) {
    HIPCHECK(hipMemcpy(S.sv64, X.sv.data(), X.sv.size() * 8, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(S.sv32, X.sv32.data(), X.sv32.size() * 4, hipMemcpyHostToDevice));
  }
}

static void build_sell(Device *dv, DLevel &L, const HCsr &H, bool first_time, std::vector<int> *slot_map = nullptr) {
  build_sell_ranges(dv, L.sell, H, L.groups, first_time, slot_map);
}

// host image of a level operator in the level's internal numbering: off-diagonal CSR, its sliced
// ELL, the diagonal and its inverse in both precisions. With first_time it also sets the per-group
// byte-model counts of L (host-only: safe on a host thread, one level per thread).
struct LevelStage {
  HCsr H;
  SellHost sell;
  std::vector<double> diag, inv;
  std::vector<float> d32, i32;
};

static void stage_level(DLevel &L, const Csr &A, bool first_time, LevelStage &X) {
  X.H = permute(A, L.perm, &L.iperm, true, &X.diag);
  const HCsr &H = X.H;
  const size_t n = X.diag.size();
  X.inv.resize(n);
  for (size_t i = 0; i < n; ++i) X.inv[i] = 1.0 / X.diag[i];
  X.d32.assign(X.diag.begin(), X.diag.end());
  X.i32.resize(n);
  for (size_t i = 0; i < n; ++i) X.i32[i] = 1.0f / (float)X.diag[i];
  if (first_time) {
    const int G = (int)L.groups.size();
    L.cnnz.assign(G, 0);
    L.ucols.assign(G, 0);
    L.cnnz_lo.assign(G, 0);
    L.ucols_lo.assign(G, 0);
    L.cnnz_up.assign(G, 0);
    L.ucols_up.assign(G, 0);
    std::vector<int> seen(L.n, -1);
    for (int c = 0; c < G; ++c)
      for (int i = L.groups[c].first; i < L.groups[c].second; ++i)
        for (int p = H.rp[i]; p < H.rp[i + 1]; ++p) {
          const bool lo = H.ci[p] < L.groups[c].first, up = H.ci[p] >= L.groups[c].second;
          ++L.cnnz[c];
          L.cnnz_lo[c] += lo;
          L.cnnz_up[c] += up;
          if (seen[H.ci[p]] != c) {
            seen[H.ci[p]] = c;
            ++L.ucols[c];
            L.ucols_lo[c] += lo;
            L.ucols_up[c] += up;
          }
        }
  }
  X.sell = sell_host(H, L.groups);
}

// host image of a level's near-boundary solver in the level's internal numbering
struct NbStage {
  bool has = false;
  std::vector<int> jrow, rowpiece, poff, asi_rp, asi_ci, ais_rp, ais_ci;
  std::vector<int64_t> boff;
  std::vector<double> inv, blk, asi, ais, sinv;
  SellHost sell;
  int64_t nnz = 0;
  int nI = 0, nS = 0, P = 0;
  bool dense = true;
};

static void stage_nb(const NearBnd &nb, const DLevel &L, const HCsr &H, NbStage &X) {
  const int n = (int)nb.J.size();
  X.has = n > 0;
  if (!X.has) return;
  X.jrow.resize(n);
  for (int k = 0; k < n; ++k) X.jrow[k] = L.iperm[nb.J[k]];
  HCsr R;
  R.nrows = n;
  R.ncols = H.ncols;
  R.rp.assign(n + 1, 0);
  for (int k = 0; k < n; ++k) {
    const int i = X.jrow[k];
    for (int p = H.rp[i]; p < H.rp[i + 1]; ++p) {
      R.ci.push_back(H.ci[p]);
      R.v.push_back(H.v[p]);
    }
    R.rp[k + 1] = (int)R.ci.size();
  }
  X.nnz = (int64_t)R.ci.size();
  X.sell = sell_host(R, Ranges{{0, n}});
  X.dense = nb.dense;
  if (nb.dense) {
    X.inv = nb.inv;
    return;
  }
  X.nI = nb.nI;
  X.nS = n - nb.nI;
  X.P = (int)nb.poff.size() - 1;
  X.poff.assign(nb.poff.begin(), nb.poff.end());
  X.boff = nb.boff;
  X.rowpiece.resize(nb.nI);
  for (int p = 0; p < X.P; ++p)
    for (int64_t i = nb.poff[p]; i < nb.poff[p + 1]; ++i) X.rowpiece[i] = p;
  X.blk = nb.blocks;
  X.asi_rp.assign(nb.ASI.rp.begin(), nb.ASI.rp.end());
  X.asi_ci.assign(nb.ASI.ci.begin(), nb.ASI.ci.end());
  X.asi = nb.ASI.v;
  X.ais_rp.assign(nb.AIS.rp.begin(), nb.AIS.rp.end());
  X.ais_ci.assign(nb.AIS.ci.begin(), nb.AIS.ci.end());
  X.ais = nb.AIS.v;
  X.sinv = nb.sinv;
}

static std::vector<float> to32(const std::vector<double> &v) { return std::vector<float>(v.begin(), v.end()); }

template <class T>
static void dcopy(T *d, const std::vector<T> &v) {
  if (!v.empty()) HIPCHECK(hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
}

static void commit_nb(Device *dv, DNb &D, const NbStage &X, bool first_time) {
  if (!X.has) return;
  if (first_time) {
    D.n = (int)X.jrow.size();
    D.dense = X.dense;
    D.nI = X.nI;
    D.nS = X.nS;
    D.P = X.P;
    D.nnz = X.nnz;
    D.jrow = dupload(dv, X.jrow);
    sell_upload(dv, D.sell, X.sell, true);
    if (X.dense) {
      D.inv64 = dupload(dv, X.inv);
      D.inv32 = dupload(dv, to32(X.inv));
    } else {
      D.rowpiece = dupload(dv, X.rowpiece);
      D.poff = dupload(dv, X.poff);
      D.boff = dupload(dv, X.boff);
      D.blk64 = dupload(dv, X.blk);
      D.blk32 = dupload(dv, to32(X.blk));
      D.asi_rp = dupload(dv, X.asi_rp);
      D.asi_ci = dupload(dv, X.asi_ci);
      D.asi64 = dupload(dv, X.asi);
      D.asi32 = dupload(dv, to32(X.asi));
      D.ais_rp = dupload(dv, X.ais_rp);
      D.ais_ci = dupload(dv, X.ais_ci);
      D.ais64 = dupload(dv, X.ais);
      D.ais32 = dupload(dv, to32(X.ais));
      D.sinv64 = dupload(dv, X.sinv);
      D.sinv32 = dupload(dv, to32(X.sinv));
      D.nblk = (int64_t)X.blk.size();
      D.nasi = (int64_t)X.asi.size();
      D.nais = (int64_t)X.ais.size();
    }
    D.r64 = dalloc<double>(dv, D.n);
    D.x64 = dalloc<double>(dv, D.n);
    D.y64 = dalloc<double>(dv, D.n);
    D.t64 = dalloc<double>(dv, D.n);
    D.r32 = dalloc<float>(dv, D.n);
    D.x32 = dalloc<float>(dv, D.n);
    D.y32 = dalloc<float>(dv, D.n);
    D.t32 = dalloc<float>(dv, D.n);
    return;
  }
  // new coefficient: the same structure, new values
  sell_upload(dv, D.sell, X.sell, false);
  if (X.dense) {
    dcopy(D.inv64, X.inv);
    dcopy(D.inv32, to32(X.inv));
  } else {
    dcopy(D.blk64, X.blk);
    dcopy(D.blk32, to32(X.blk));
    dcopy(D.asi64, X.asi);
    dcopy(D.asi32, to32(X.asi));
    dcopy(D.ais64, X.ais);
    dcopy(D.ais32, to32(X.ais));
    dcopy(D.sinv64, X.sinv);
    dcopy(D.sinv32, to32(X.sinv));
  }
}

// upload a staged level; `csr`: also keep a device CSR of the off-diagonal part (original grid)
static void commit_level(Device *dv, DLevel &L, const LevelStage &X, bool first_time, bool csr) {
  if (first_time) {
    if (csr)
      upload_csr(dv, X.H, L.A);
    else
      csr_shape(X.H, L.A);
    sell_upload(dv, L.sell, X.sell, true);
    L.dg64 = dupload(dv, X.diag);
    L.id64 = dupload(dv, X.inv);
    L.dg32 = dupload(dv, X.d32);
    L.id32 = dupload(dv, X.i32);
  } else {
    upload_values(L.A, X.H);
    sell_upload(dv, L.sell, X.sell, false);
    HIPCHECK(hipMemcpy(L.dg64, X.diag.data(), X.diag.size() * 8, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(L.id64, X.inv.data(), X.inv.size() * 8, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(L.dg32, X.d32.data(), X.d32.size() * 4, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(L.id32, X.i32.data(), X.i32.size() * 4, hipMemcpyHostToDevice));
  }
}

// contribution lists of the original-grid operator (internal numbering): entry value =
// sum over elements e of kappa_e * K1_e[a][b], elements in ascending order
static void build_refresh(Device *dv, Hierarchy &h, const HCsr &H, const std::vector<int> &slot_map) {
  const int d = h.d, k = d + 1, n = dv->fine.n;
  const std::vector<int> &ip = dv->fine.iperm;
  const int64_t nnz = (int64_t)H.ci.size();
  std::vector<int> cnt_off(nnz + 1, 0), cnt_dg(n + 1, 0);
  auto pos_of = [&](int i, int j) {
    const int *b = H.ci.data() + H.rp[i], *e = H.ci.data() + H.rp[i + 1];
    return (int)(std::lower_bound(b, e, j) - H.ci.data());
  };
  for (int pass = 0; pass < 2; ++pass) {
    std::vector<int> eo, ed;
    std::vector<double> wo, wd;
    std::vector<int> fo, fd;
    if (pass == 1) {
      for (int64_t p = 0; p < nnz; ++p) cnt_off[p + 1] += cnt_off[p];
      for (int i = 0; i < n; ++i) cnt_dg[i + 1] += cnt_dg[i];
      eo.resize(cnt_off[nnz]);
      wo.resize(cnt_off[nnz]);
      ed.resize(cnt_dg[n]);
      wd.resize(cnt_dg[n]);
      fo.assign(cnt_off.begin(), cnt_off.end() - 1);
      fd.assign(cnt_dg.begin(), cnt_dg.end() - 1);
    }
    double K[4][4];
    for (int64_t e = 0; e < h.ne; ++e) {
      int in[4];
      for (int a = 0; a < k; ++a) {
        const int64_t u = h.dof_of_vertex[h.elems[e * k + a]];
        in[a] = u >= 0 ? ip[u] : -1;
      }
      if (pass == 1) element_unit_stiffness(h, e, K);
      for (int a = 0; a < k; ++a) {
        if (in[a] < 0) continue;
        for (int b = 0; b < k; ++b) {
          if (in[b] < 0) continue;
          if (a == b) {
            if (pass == 0) {
              cnt_dg[in[a] + 1]++;
            } else {
              const int q = fd[in[a]]++;
              ed[q] = (int)e;
              wd[q] = K[a][b];
            }
          } else {
            const int p = pos_of(in[a], in[b]);
            if (pass == 0) {
              cnt_off[p + 1]++;
            } else {
              const int q = fo[p]++;
              eo[q] = (int)e;
              wo[q] = K[a][b];
            }
          }
        }
      }
    }
    if (pass == 1) {
      dv->rf_off_ptr = dupload(dv, cnt_off);
      dv->rf_off_el = dupload(dv, eo);
      dv->rf_off_w = dupload(dv, wo);
      dv->rf_dg_ptr = dupload(dv, cnt_dg);
      dv->rf_dg_el = dupload(dv, ed);
      dv->rf_dg_w = dupload(dv, wd);
    }
  }
  dv->rf_sell_map = dupload(dv, slot_map);
  dv->rf_nslots = (int)slot_map.size();
}

static void upload_coarse(Device *dv, Hierarchy &h, bool first_time) {
  const int64_t n = h.nc;
  std::vector<float> f(h.coarse_inv.begin(), h.coarse_inv.end());
  if (first_time) {
    dv->nc = (int)n;
    dv->cinv64 = dupload(dv, h.coarse_inv);
    dv->cinv32 = dupload(dv, f);
    dv->cb64 = dalloc<double>(dv, n);
    dv->cx64 = dalloc<double>(dv, n);
    dv->cb32 = dalloc<float>(dv, n);
    dv->cx32 = dalloc<float>(dv, n);
  } else if (n > 0) {
    HIPCHECK(hipMemcpy(dv->cinv64, h.coarse_inv.data(), n * n * 8, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(dv->cinv32, f.data(), n * n * 4, hipMemcpyHostToDevice));
  }
}

Device *device_create(Hierarchy &h, int ordinal) {
  int count = 0;
  HIPCHECK(hipGetDeviceCount(&count));
  if (ordinal < 0 || ordinal >= count) throw AsmgError{ASMG_EDEVICE, "no such HIP device"};
  HIPCHECK(hipSetDevice(ordinal));
  Device *dv = new Device();
  const bool tm = std::getenv("ASMG_SETUP_TIMING") != nullptr;
  auto t0 = std::chrono::steady_clock::now();
  auto lap = [&](const char *what) {
    if (!tm) return;
    auto t1 = std::chrono::steady_clock::now();
    std::fprintf(stderr, "[asmg upload] %-16s %8.3f s\n", what, std::chrono::duration<double>(t1 - t0).count());
    t0 = t1;
  };
  try {
    dv->ordinal = ordinal;
    dv->d = h.d;
    dv->J = h.J;
    dv->lc = h.lc;
    dv->nu_aux = h.opt.nu_aux;
    dv->nu_fine = h.opt.nu_fine;
    dv->maxit = h.opt.max_iter;
    dv->precision = h.opt.precision;
    dv->check_every = h.opt.check_every;
    dv->autotune = h.opt.autotune;
    // fine level: colour-major, Morton order of the vertices inside a colour (rows that are
    // neighbours in the numbering are neighbours in space, whatever the mesh's own numbering)
    const std::vector<int> mrank = morton_rank(h);
    colour_order(h.colour_fine, dv->fine, &mrank);
    // auxiliary levels
    dv->aux.resize(h.J + 1);
    for (int l = h.J; l > h.lc; --l) {
      DLevel &L = dv->aux[l];
      if (h.opt.smoothing == 1)
        local_order(h.colour_aux.at(l), h.local_set.at(l), h.Al.at(l), L);
      else
        colour_order(h.colour_aux.at(l), L);
    }
    lap("orders");
    // Host images of every matrix, built on host threads (each task writes only its own stage
    // and, for a level, that level's byte-model counts), then uploaded in a fixed order.
    // Prolongations are in internal numbering; their slices visit the rows in each level's own
    // (Morton) numbering: position k holds internal row iperm[k] (the bottom level keeps its
    // numbering). Pi: rows fine internal, columns level-J internal (or unknown order if J is the
    // bottom); its slices visit the original-grid unknowns in Morton order of their vertices.
    const int naux = h.J - h.lc;
    LevelStage fine_st;
    std::vector<LevelStage> aux_st(naux);
    std::vector<NbStage> nb_st(naux);
    std::vector<TransferStage> p_st(naux), pt_st(naux);
    TransferStage pi_st, pit_st;
    const std::vector<int> *pi_cmap = h.J > h.lc ? &dv->aux[h.J].iperm : nullptr;
    std::vector<int> forder(mrank.size());
    for (size_t i = 0; i < mrank.size(); ++i) forder[mrank[i]] = dv->fine.iperm[i];
    // tasks: Pi and Pi^T first (the largest), then the fine operator, the levels, the prolongations
    // last colour of a level with whole-level smoothing, [first row, end) in internal numbering
    auto last_colour = [&](const DLevel &L, int l) {
      // a level with the near-boundary correction computes its residual on every row and
      // prolongs onto every row (the correction reads them)
      if (L.local || L.C < 1 || (l > 0 && h.nb.count(l))) return std::make_pair(0, 0);
      return std::make_pair(L.coff[L.C - 1], L.coff[L.C]);
    };
    const auto fl = last_colour(dv->fine, 0);
    host_parallel(h.threads, 3 + 2 * naux, [&](int t) {
      if (t == 0) {
        const HCsr Pi = permute(h.Pi, dv->fine.perm, pi_cmap, false, nullptr);
        stage_transfer(Pi, &forder, pi_st);
        if (fl.second > fl.first) stage_prolong_v(Pi, forder, fl.first, fl.second, pi_st);
      } else if (t == 1) {
        const HCsr PiT = transpose(permute(h.Pi, dv->fine.perm, pi_cmap, false, nullptr));
        stage_transfer(PiT, pi_cmap, pit_st);
        if (fl.second > fl.first) stage_restrict_v(PiT, pi_cmap, fl.first, fl.second, pit_st);
      } else if (t == 2) {
        stage_level(dv->fine, h.A, true, fine_st);
      } else if (t < 3 + naux) {
        const int l = h.J - (t - 3);
        stage_level(dv->aux[l], h.Al.at(l), true, aux_st[t - 3]);
        auto it = h.nb.find(l);
        if (it != h.nb.end()) stage_nb(it->second, dv->aux[l], aux_st[t - 3].H, nb_st[t - 3]);
      } else {
        const int i = t - 3 - naux, l = h.J - i;
        DLevel &L = dv->aux[l];
        const std::vector<int> *cmap = l - 1 > h.lc ? &dv->aux[l - 1].iperm : nullptr;
        HCsr P = permute(h.P.at(l), L.perm, cmap, false, nullptr);
        const HCsr PT = transpose(P);
        stage_transfer(P, &L.iperm, p_st[i]);
        stage_transfer(PT, cmap, pt_st[i]);
        const auto ll = last_colour(L, l);
        if (ll.second > ll.first) {
          stage_prolong_v(P, L.iperm, ll.first, ll.second, p_st[i]);
          stage_restrict_v(PT, cmap, ll.first, ll.second, pt_st[i]);
        }
      }
    });
    lap("host layout");
    commit_level(dv, dv->fine, fine_st, true, true);
    fine_st = LevelStage();
    alloc_vectors(dv, dv->fine);
    dv->perm_d = dupload(dv, dv->fine.perm);
    for (int l = h.J; l > h.lc; --l) {
      LevelStage &X = aux_st[h.J - l];
      commit_level(dv, dv->aux[l], X, true, false);
      X = LevelStage();
      alloc_vectors(dv, dv->aux[l]);
      commit_nb(dv, dv->aux[l].nb, nb_st[h.J - l], true);
      nb_st[h.J - l] = NbStage();
    }
    dv->pure_neumann = h.n() == h.nv;
    for (int l = h.J; l > h.lc; --l) {
      commit_transfer(dv, p_st[h.J - l], dv->aux[l].P);
      commit_transfer(dv, pt_st[h.J - l], dv->aux[l].PT);
    }
    commit_transfer(dv, pi_st, dv->Pi);
    commit_transfer(dv, pit_st, dv->PiT);
    lap("upload");
    upload_coarse(dv, h, true);
    dv->nested = h.opt.nested;
    if (dv->nested > 0) {
      for (int l = dv->J; l > dv->lc; --l) {
        DLevel &L = dv->aux[l];
        L.ng64 = dalloc<double>(dv, L.n);
        L.ne64 = dalloc<double>(dv, L.n);
        L.ng32 = dalloc<float>(dv, L.n);
        L.ne32 = dalloc<float>(dv, L.n);
      }
      dv->cng64 = dalloc<double>(dv, dv->nc);
      dv->cne64 = dalloc<double>(dv, dv->nc);
      dv->cng32 = dalloc<float>(dv, dv->nc);
      dv->cne32 = dalloc<float>(dv, dv->nc);
    }
    const int n = dv->fine.n;
    dv->f = dalloc<double>(dv, n);
    dv->u = dalloc<double>(dv, n);
    dv->r = dalloc<double>(dv, n);
    dv->p = dalloc<double>(dv, n);
    dv->q = dalloc<double>(dv, n);
    dv->io_in = dalloc<double>(dv, n);
    dv->io_out = dalloc<double>(dv, n);
    dv->ctl = dalloc<Ctl>(dv, 1);
    HIPCHECK(hipMemset(dv->ctl, 0, sizeof(Ctl)));
    HIPCHECK(hipHostMalloc((void **)&dv->ctl_host, sizeof(Ctl), hipHostMallocDefault));
    HIPCHECK(hipStreamCreateWithFlags(&dv->stream, hipStreamNonBlocking));
    HIPCHECK(hipEventCreateWithFlags(&dv->ev_in, hipEventDisableTiming));
    HIPCHECK(hipEventCreateWithFlags(&dv->ev_out, hipEventDisableTiming));
    dv->max_blocks = h.opt.red_blocks > 0 ? std::min(h.opt.red_blocks, RED_BLOCKS) : RED_BLOCKS;
    dv->partials = dalloc<double>(dv, RED_BLOCKS);
    // element data for the gradient kernel
    dv->ne = h.ne;
    dv->nv = h.nv;
    dv->coords = dupload(dv, h.coords);
    std::vector<int> el(h.elems.begin(), h.elems.end());
    dv->elems = dupload(dv, el);
    dv->kappa = dupload(dv, h.kappa);
    std::vector<int> dov(h.dof_of_vertex.begin(), h.dof_of_vertex.end());
    dv->dof_of_vertex = dupload(dv, dov);
    HIPCHECK(hipDeviceSynchronize());
  } catch (...) {
    device_destroy(dv);
    throw;
  }
  return dv;
}

void device_update_values(Device *dv, Hierarchy &h) {
  HIPCHECK(hipSetDevice(dv->ordinal));
  const int naux = h.J - h.lc;
  std::vector<LevelStage> st(1 + naux);
  std::vector<NbStage> nst(1 + naux);
  host_parallel(h.threads, 1 + naux, [&](int t) {
    if (t == 0) {
      stage_level(dv->fine, h.A, false, st[0]);
    } else {
      const int l = h.J - (t - 1);
      stage_level(dv->aux[l], h.Al.at(l), false, st[t]);
      auto it = h.nb.find(l);
      if (it != h.nb.end()) stage_nb(it->second, dv->aux[l], st[t].H, nst[t]);
    }
  });
  commit_level(dv, dv->fine, st[0], false, true);
  for (int l = h.J; l > h.lc; --l) {
    commit_level(dv, dv->aux[l], st[h.J - l + 1], false, false);
    commit_nb(dv, dv->aux[l].nb, nst[h.J - l + 1], false);
  }
  upload_coarse(dv, h, false);
  HIPCHECK(hipMemcpy(dv->kappa, h.kappa.data(), h.kappa.size() * 8, hipMemcpyHostToDevice));
  HIPCHECK(hipDeviceSynchronize());
}

void device_set_precision(Device *dv, int precision) { dv->precision = precision; }

void device_destroy(Device *dv) {
  if (!dv) return;
  (void)hipSetDevice(dv->ordinal);
  if (dv->stream) (void)hipStreamSynchronize(dv->stream);
  for (int k = 0; k < 2; ++k)
    if (dv->graph[k]) (void)hipGraphExecDestroy(dv->graph[k]);
  for (hipEvent_t e : dv->tune_ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : dv->probe_ev) (void)hipEventDestroy(e);
  if (dv->ev_in) (void)hipEventDestroy(dv->ev_in);
  if (dv->ev_out) (void)hipEventDestroy(dv->ev_out);
  if (dv->stream) (void)hipStreamDestroy(dv->stream);
  for (void *p : dv->allocs) (void)hipFree(p);
  if (dv->ctl_host) (void)hipHostFree(dv->ctl_host);
  delete dv;
}

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------


// grid of a reducing kernel: enough blocks for one pass, capped at the handle's reduction cap
static inline int red_grid(const Device *dv, int64_t rows, int lpr) {
  return std::min<int>(dv->max_blocks, nblk(rows * lpr));
}

static inline double csr_bytes(const DCsr &A, int vbytes) {
  return (double)A.nnz * (vbytes + 4) + 4.0 * (A.nrows + 1);
}

template <class T>
static const T *vals(const DCsr &A);
template <>
const double *vals<double>(const DCsr &A) { return A.v64; }
template <>
const float *vals<float>(const DCsr &A) { return A.v32; }

template <class T>
static const T *sell_vals(const DSell &S);
template <>
const double *sell_vals<double>(const DSell &S) { return S.sv64; }
template <>
const float *sell_vals<float>(const DSell &S) { return S.sv32; }

template <class T>
struct LV {
  static T *x(DLevel &L);
  static T *b(DLevel &L);
  static T *r(DLevel &L);
  static const T *dg(DLevel &L);
  static const T *id(DLevel &L);
};
template <>
struct LV<double> {
  static double *x(DLevel &L) { return L.x64; }
  static double *b(DLevel &L) { return L.b64; }
  static double *r(DLevel &L) { return L.r64; }
  static const double *dg(DLevel &L) { return L.dg64; }
  static const double *id(DLevel &L) { return L.id64; }
};
template <>
struct LV<float> {
  static float *x(DLevel &L) { return L.x32; }
  static float *b(DLevel &L) { return L.b32; }
  static float *r(DLevel &L) { return L.r32; }
  static const float *dg(DLevel &L) { return L.dg32; }
  static const float *id(DLevel &L) { return L.id32; }
};



// algorithmic bytes of one colour pass: the colour's matrix rows (values, columns, row pointers),
// b, 1/diag and the x write of its rows, and each distinct x entry it gathers once
template <class T>
static double gs_bytes(const DLevel &L, int c, bool lower = false) {
  const double rows = L.groups[c].second - L.groups[c].first;
  const double nz = (double)(lower ? L.cnnz_lo[c] : L.cnnz[c]);
  const double uc = (double)(lower ? L.ucols_lo[c] : L.ucols[c]);
  return nz * (sizeof(T) + 4) + 4.0 * (rows + 1) + 3.0 * sizeof(T) * rows + (double)sizeof(T) * uc;
}

// One slice-kernel launch site of B_co: launch(threads, xcd, e0, e1) enqueues the kernel over
// `nslices` slices (launch_timed: with events, they are stamped with the kernel's own start and
// end). While tuning, the site runs the candidate shape under trial with its pair of events, so
// that its time is measured inside a whole B_co application (caches as in a solve); otherwise
// it runs the shape stored for the site (or the default). The tuned kernels have no
// reductions, so the shape does not change any result.
// With probe_bytes >= 0 (GS pass timing of device_time_kernel) the launch is stamped with the
// next pair of probe events and counted with that many algorithmic bytes.
template <class F>
static void slice_launch(Device *dv, int nslices, hipStream_t s, F &&launch, double probe_bytes = -1.0) {
  auto &tab = dv->shape[dv->shape_pi];
  const int site = dv->site >= 0 ? dv->site++ : -1;  // -1: outside B_co (default shape)
  if (nslices <= 0) return;
  auto sh = site >= 0 && site < (int)tab.size() ? tab[site] : kShapes[0];
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (dv->tuning && site >= 0) {
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
  } else if (probe_bytes >= 0.0) {
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
  }
  launch(sh.threads, sh.xcd, sh.var, e0, e1);
}


template <class T>
static void gs_pass(Device *dv, DLevel &L, int c, T *x, const T *b, hipStream_t s, bool lower = false) {
  const bool probe = dv->probe_lpr != 0 && dv->probe_prec == (sizeof(T) == 4 ? 1 : 0);
  const DSell &S = L.sell;
  const int s0 = S.cslice[c], s1 = S.cslice[c + 1];
  slice_launch(
      dv, s1 - s0, s,
      [&](int th, int xcd, int var, hipEvent_t e0, hipEvent_t e1) {
        with_var(var, [&](auto vc) {
          launch_timed((k_sell<0, T, decltype(vc)::value>), slice_blocks(s1 - s0, th, var), th, s, e0, e1, s0, s1,
                       S.srow, S.soff, lower ? S.slo : S.soff + 1, S.scol, sell_vals<T>(S), LV<T>::id(L), b, x,
                       (T *)nullptr, shape_arg(th, xcd));
        });
      },
      probe ? gs_bytes<T>(L, c, lower) : -1.0);
  if (dv->count_bytes) dv->bytes += gs_bytes<T>(L, c, lower);
}

// bytes of the first colour pass of a sweep from zero when it runs on its own:
// x written on every row, b and 1/diag read on colour 0
template <class T>
static double first_pass_bytes(const DLevel &L) {
  return (double)L.n * sizeof(T) + (double)L.first_rows * 2 * sizeof(T);
}

// Gauss-Seidel sweep over colours. `first_done`: the sweep starts from zero and its colour-0
// pass has already been run by the kernel that produced b.
template <class T>
static void sweep(Device *dv, DLevel &L, T *x, const T *b, bool from_zero, bool first_done, bool forward,
                  hipStream_t s) {
  const int C = L.C;
  if (forward) {
    int c = 0;
    if (from_zero) {
      if (!first_done) {
        hipLaunchKernelGGL((k_gs_first<T>), dim3(nblk(L.n)), dim3(BS), 0, s, L.n, L.first_rows, b, LV<T>::id(L), x);
        if (dv->count_bytes) dv->bytes += first_pass_bytes<T>(L);
      }
      c = 1;
    }
    // in a sweep from zero, the rows of colour c see zero at every neighbour of a later colour:
    // their passes read only the prefix of each row's entries that holds the earlier colours
    // (rows store their columns in ascending order, colours in ascending ranges)
    const bool lower = LOWER_FIRST_SWEEP && from_zero && !L.local;
    for (; c < C; ++c) gs_pass<T>(dv, L, c, x, b, s, lower);
  } else {
    for (int c = C - 1; c >= 0; --c) gs_pass<T>(dv, L, c, x, b, s);
  }
}

// r = b - A x on the rows of every slice group (all rows; with local smoothing the rows of N~+,
// r = b elsewhere having been written with b).
// B_co and the V-cycle take the residual right after a forward sweep, whose last colour pass
// solved that colour's rows with every neighbour final: their residual is zero in exact
// arithmetic. With whole-level smoothing the kernel skips that colour's slices; their r entries
// are zeroed at setup and nothing else writes them. `full` covers every row (the residual of an
// arbitrary iterate, for the nested iteration).
// `upper`: x is the result of a single forward sweep from zero over the whole level, so each row's
// residual is minus its later colours' terms (k_sell MODE 2), which reads neither b, the diagonal
// nor x at the row, and only the entries after each slice's shi.
template <class T>
static void residual(Device *dv, DLevel &L, const T *b, const T *x, T *r, hipStream_t s, bool full = false,
                     bool upper = false) {
  const DSell &S = L.sell;
  const bool skip = !full && !L.local && L.C >= 1;
  upper = upper && skip;
  const int s1 = skip ? S.cslice[L.C - 1] : S.nslices;
  slice_launch(dv, s1, s, [&](int th, int xcd, int var, hipEvent_t e0, hipEvent_t e1) {
    with_var(var, [&](auto vc) {
      if (upper)
        launch_timed((k_sell<2, T, decltype(vc)::value>), slice_blocks(s1, th, var), th, s, e0, e1, 0, s1, S.srow,
                     S.shi, S.soff + 1, S.scol, sell_vals<T>(S), (const T *)nullptr, (const T *)nullptr, (T *)x, r,
                     shape_arg(th, xcd));
      else
        launch_timed((k_sell<1, T, decltype(vc)::value>), slice_blocks(s1, th, var), th, s, e0, e1, 0, s1, S.srow,
                     S.soff, S.soff + 1, S.scol, sell_vals<T>(S), LV<T>::dg(L), b, (T *)x, r, shape_arg(th, xcd));
    });
  });
  if (S.nslices == 0) return;
  if (dv->count_bytes)
    for (size_t g = 0; g < (skip ? (size_t)(L.C - 1) : L.groups.size()); ++g) {
      const double rows = L.groups[g].second - L.groups[g].first;
      if (upper)  // the later colours' entries, row index, r written, each gathered x entry once
        dv->bytes += (double)L.cnnz_up[g] * (sizeof(T) + 4) + 4.0 * rows + sizeof(T) * (rows + (double)L.ucols_up[g]);
      else
        dv->bytes += (double)L.cnnz[g] * (sizeof(T) + 4) + 4.0 * rows + 4.0 * sizeof(T) * rows;
    }
}

// y = A x (ADD 0) or y += A x (ADD 1) for a transfer matrix A
template <class T, int ADD>
static void spmv(Device *dv, const DCsr &A, const T *x, T *y, hipStream_t s, bool vcyc = false) {
  if (A.nrows == 0) return;
  const DSell &S = vcyc && A.vsell ? *A.vsell : *A.sell;
  slice_launch(dv, S.nslices, s, [&](int th, int xcd, int var, hipEvent_t e0, hipEvent_t e1) {
    with_var(var, [&](auto vc) {
      constexpr int O = decltype(vc)::value;
      if (S.wmax > 16)
        launch_timed((k_sell_spmv<ADD, 0, T, 32, O>), slice_blocks(S.nslices, th, var), th, s, e0, e1, S.nslices, S.srow,
                     S.soff, S.scol, sell_vals<T>(S), x, y, 0, (const T *)nullptr, (T *)nullptr, (T *)nullptr,
                     shape_arg(th, xcd));
      else
        launch_timed((k_sell_spmv<ADD, 0, T, 16, O>), slice_blocks(S.nslices, th, var), th, s, e0, e1, S.nslices, S.srow,
                     S.soff, S.scol, sell_vals<T>(S), x, y, 0, (const T *)nullptr, (T *)nullptr, (T *)nullptr,
                     shape_arg(th, xcd));
    });
  });
  if (dv->count_bytes)
    dv->bytes += (double)S.nnz * (sizeof(T) + 4) + 4.0 * (S.nrows + 1) + (double)S.ncols_used * sizeof(T) +
                 (1 + ADD) * (double)S.nrows * sizeof(T);
}

// restriction y = A x into the right-hand side of level L, fused with the colour-0 pass of the
// first (from zero) forward sweep on L; with local smoothing also r = y (the residual kernel
// then overwrites r on N~+ only)
template <class T>
static void spmv_first(Device *dv, const DCsr &A, const T *x, DLevel &L, hipStream_t s) {
  if (A.nrows == 0) return;
  const DSell &S = A.vsell ? *A.vsell : *A.sell;  // restrictions of residuals inside B_co only
  T *rc = L.local ? LV<T>::r(L) : (T *)nullptr;
  slice_launch(dv, S.nslices, s, [&](int th, int xcd, int var, hipEvent_t e0, hipEvent_t e1) {
    with_var(var, [&](auto vc) {
      constexpr int O = decltype(vc)::value;
      if (S.wmax > 16)
        launch_timed((k_sell_spmv<0, 1, T, 32, O>), slice_blocks(S.nslices, th, var), th, s, e0, e1, S.nslices, S.srow,
                     S.soff, S.scol, sell_vals<T>(S), x, LV<T>::b(L), L.first_rows, LV<T>::id(L), LV<T>::x(L), rc,
                     shape_arg(th, xcd));
      else
        launch_timed((k_sell_spmv<0, 1, T, 16, O>), slice_blocks(S.nslices, th, var), th, s, e0, e1, S.nslices, S.srow,
                     S.soff, S.scol, sell_vals<T>(S), x, LV<T>::b(L), L.first_rows, LV<T>::id(L), LV<T>::x(L), rc,
                     shape_arg(th, xcd));
    });
  });
  if (dv->count_bytes)
    dv->bytes += (double)S.nnz * (sizeof(T) + 4) + 4.0 * (S.nrows + 1) + (double)S.ncols_used * sizeof(T) +
                 (2.0 + (rc ? 1 : 0)) * S.nrows * sizeof(T) + (double)L.first_rows * sizeof(T);
}

template <class T>
static T *cvec_b(Device *dv);
template <>
double *cvec_b<double>(Device *dv) { return dv->cb64; }
template <>
float *cvec_b<float>(Device *dv) { return dv->cb32; }
template <class T>
static T *cvec_x(Device *dv);
template <>
double *cvec_x<double>(Device *dv) { return dv->cx64; }
template <>
float *cvec_x<float>(Device *dv) { return dv->cx32; }
template <class T>
static const T *cinv(Device *dv);
template <>
const double *cinv<double>(Device *dv) { return dv->cinv64; }
template <>
const float *cinv<float>(Device *dv) { return dv->cinv32; }

// rhs / solution vectors of level l (the bottom level has its own)
template <class T>
static T *lvl_b(Device *dv, int l) { return l == dv->lc ? cvec_b<T>(dv) : LV<T>::b(dv->aux[l]); }
template <class T>
static T *lvl_x(Device *dv, int l) { return l == dv->lc ? cvec_x<T>(dv) : LV<T>::x(dv->aux[l]); }

// restriction into level l's right-hand side (with its first colour pass above the bottom)
template <class T>
static void restrict_to(Device *dv, const DCsr &A, const T *x, int l, hipStream_t s) {
  if (l == dv->lc)
    spmv<T, 0>(dv, A, x, cvec_b<T>(dv), s, true);
  else
    spmv_first<T>(dv, A, x, dv->aux[l], s);
}

// per-precision arrays of a near-boundary set
template <class T>
struct NbV;
template <>
struct NbV<double> {
  static const double *inv(const DNb &N) { return N.inv64; }
  static const double *blk(const DNb &N) { return N.blk64; }
  static const double *asi(const DNb &N) { return N.asi64; }
  static const double *ais(const DNb &N) { return N.ais64; }
  static const double *sinv(const DNb &N) { return N.sinv64; }
  static double *r(const DNb &N) { return N.r64; }
  static double *x(const DNb &N) { return N.x64; }
  static double *t(const DNb &N) { return N.t64; }
};
template <>
struct NbV<float> {
  static const float *inv(const DNb &N) { return N.inv32; }
  static const float *blk(const DNb &N) { return N.blk32; }
  static const float *asi(const DNb &N) { return N.asi32; }
  static const float *ais(const DNb &N) { return N.ais32; }
  static const float *sinv(const DNb &N) { return N.sinv32; }
  static float *r(const DNb &N) { return N.r32; }
  static float *x(const DNb &N) { return N.x32; }
  static float *t(const DNb &N) { return N.t32; }
};

// Near-boundary correction of level L (Section 3.5, Algorithm 3): x|_J += (A|_JJ)^-1 (b - A x)|_J.
// The solve is a dense inverse, or over the decomposition of J into interiors I (pieces with
// dense inverses) and separator S: y = A_II^-1 r_I, x_S = S^-1 (r_S - A_SI y),
// x_I = A_II^-1 (r_I - A_IS x_S), with S = A_SS - A_SI A_II^-1 A_IS inverted at setup.
template <class T>
static void nb_correct(Device *dv, DLevel &L, T *x, const T *b, hipStream_t s) {
  const DNb &N = L.nb;
  if (N.n == 0) return;
  T *r = NbV<T>::r(N), *xj = NbV<T>::x(N), *t = NbV<T>::t(N);
  const DSell &S = N.sell;
  if (S.nslices > 0)
    hipLaunchKernelGGL((k_nb_res<T>), dim3(slice_blocks(S.nslices, BS)), dim3(BS), 0, s, S.nslices, S.srow, S.soff,
                       S.scol, sell_vals<T>(S), N.jrow, LV<T>::dg(L), b, (const T *)x, r);
  if (N.dense) {
    gemv<T>(N.n, NbV<T>::inv(N), (const T *)r, xj, s);
  } else {
    const int nI = N.nI, nS = N.nS;
    T *y = sizeof(T) == 8 ? (T *)N.y64 : (T *)N.y32;
    if (nI > 0)
      hipLaunchKernelGGL((k_nb_blk<T>), dim3(nblk((int64_t)nI * 64)), dim3(BS), 0, s, nI, N.rowpiece, N.poff, N.boff,
                         NbV<T>::blk(N), (const T *)r, (const T *)nullptr, y);
    if (nS > 0) {
      hipLaunchKernelGGL((k_nb_csr<T>), dim3(nblk(nS)), dim3(BS), 0, s, nS, N.asi_rp, N.asi_ci, NbV<T>::asi(N),
                         (const T *)y, (const T *)(r + nI), t);
      gemv<T>(nS, NbV<T>::sinv(N), (const T *)t, xj + nI, s);
    }
    if (nI > 0) {
      hipLaunchKernelGGL((k_nb_csr<T>), dim3(nblk(nI)), dim3(BS), 0, s, nI, N.ais_rp, N.ais_ci, NbV<T>::ais(N),
                         (const T *)(xj + nI), (const T *)r, t);
      hipLaunchKernelGGL((k_nb_blk<T>), dim3(nblk((int64_t)nI * 64)), dim3(BS), 0, s, nI, N.rowpiece, N.poff, N.boff,
                         NbV<T>::blk(N), (const T *)t, (const T *)nullptr, xj);
    }
  }
  hipLaunchKernelGGL((k_nb_add<T>), dim3(nblk(N.n)), dim3(BS), 0, s, N.n, N.jrow, (const T *)xj, x);
  if (dv->count_bytes) {
    // residual: matrix entries, position and row index, b, diagonal and x at the row, the result;
    // the solve's matrices once; the add: row index, the correction, x read and written
    double by = (double)N.nnz * (sizeof(T) + 4) + (double)N.n * (8 + 4 * sizeof(T));
    if (N.dense)
      by += (double)N.n * N.n * sizeof(T) + 2.0 * N.n * sizeof(T);
    else
      by += 2.0 * N.nblk * sizeof(T) + (double)(N.nasi + N.nais) * (sizeof(T) + 4) + (double)N.nS * N.nS * sizeof(T) +
            6.0 * N.n * sizeof(T);
    by += (double)N.n * (4 + 3 * sizeof(T));
    dv->bytes += by;
  }
}

// Algorithm 2: B_l applied to the level's b, result in the level's x. Above the bottom, the
// colour-0 pass of the first forward sweep has been run by the restriction that wrote b. A level
// with a near-boundary set corrects on it before and after the coarse-grid correction (the
// symmetric form of Algorithm 3: B_l stays symmetric); its residual then covers every row.
template <class T>
static void vcycle(Device *dv, int l, hipStream_t s) {
  if (l == dv->lc) {
    if (dv->nc > 0) {
      gemv<T>(dv->nc, cinv<T>(dv), cvec_b<T>(dv), cvec_x<T>(dv), s);
      if (dv->count_bytes) dv->bytes += (double)dv->nc * dv->nc * sizeof(T) + 2.0 * dv->nc * sizeof(T);
    }
    return;
  }
  DLevel &L = dv->aux[l];
  T *x = LV<T>::x(L);
  T *b = LV<T>::b(L);
  const bool nb = L.nb.n > 0;
  for (int k = 0; k < dv->nu_aux; ++k) sweep<T>(dv, L, x, b, k == 0, true, true, s);
  if (nb) nb_correct<T>(dv, L, x, b, s);
  residual<T>(dv, L, b, x, LV<T>::r(L), s, nb, UPPER_RESIDUAL && dv->nu_aux == 1 && !nb);
  restrict_to<T>(dv, L.PT, LV<T>::r(L), l - 1, s);
  vcycle<T>(dv, l - 1, s);
  spmv<T, 1>(dv, L.P, lvl_x<T>(dv, l - 1), x, s, true);
  if (nb) nb_correct<T>(dv, L, x, b, s);
  for (int k = 0; k < dv->nu_aux; ++k) sweep<T>(dv, L, x, b, false, false, false, s);
}

// Algorithm 1 (u_0 = 0): x_fine = B_co r; r in FP64 (internal order), result in fine.x{64,32}.
// `first_done`: the colour-0 pass of the fine forward sweep (and, in FP32, the rounding of r
// into fine.b32) has already been run by the CG update that produced r.
template <class T>
static void apply_Bco(Device *dv, const double *r, bool first_done, hipStream_t s) {
  DLevel &F = dv->fine;
  dv->site = 0;
  dv->shape_pi = sizeof(T) == 4 ? 1 : 0;
  T *x = LV<T>::x(F);
  const T *b;
  if constexpr (sizeof(T) == 8) {
    b = r;
  } else {
    if (!first_done) {
      hipLaunchKernelGGL(k_gs_first_cvt, dim3(nblk(F.n)), dim3(BS), 0, s, F.n, F.first_rows,
                         r, F.b32, F.id32, F.x32);
      if (dv->count_bytes) dv->bytes += (double)F.n * (8 + 4 + 4) + (double)F.first_rows * 4;
      first_done = true;
    }
    b = F.b32;
  }
  for (int k = 0; k < dv->nu_fine; ++k) sweep<T>(dv, F, x, b, k == 0, first_done, true, s);
  residual<T>(dv, F, b, x, LV<T>::r(F), s, false, UPPER_RESIDUAL && dv->nu_fine == 1);
  restrict_to<T>(dv, dv->PiT, LV<T>::r(F), dv->J, s);
  vcycle<T>(dv, dv->J, s);
  spmv<T, 1>(dv, dv->Pi, lvl_x<T>(dv, dv->J), x, s, true);
  for (int k = 0; k < dv->nu_fine; ++k) sweep<T>(dv, F, x, b, false, false, false, s);
}

// nested-iteration vectors of an auxiliary level / of the bottom level
template <class T>
struct NV;
template <>
struct NV<double> {
  static double *g(Device *dv, int l) { return l == dv->lc ? dv->cng64 : dv->aux[l].ng64; }
  static double *e(Device *dv, int l) { return l == dv->lc ? dv->cne64 : dv->aux[l].ne64; }
};
template <>
struct NV<float> {
  static float *g(Device *dv, int l) { return l == dv->lc ? dv->cng32 : dv->aux[l].ng32; }
  static float *e(Device *dv, int l) { return l == dv->lc ? dv->cne32 : dv->aux[l].ne32; }
};

// Nested iteration over the auxiliary levels (Section 5.2), in the V-cycle's precision T:
// g_J = Pi^T f, g_(l-1) = P_l^T g_l; e_(l_c) = A_(l_c)^-1 g_(l_c); on each finer level
// e_l = P_l e_(l-1), then `nested` times e_l += B_l (g_l - A_l e_l) with the V-cycle of
// Algorithm 2 (its right-hand side written by the residual kernel, its first colour pass from
// zero run on its own); finally u = Pi e_J in FP64 (internal order). Whole-level smoothing.
template <class T>
static void nested_start(Device *dv, hipStream_t s) {
  TraceRange tr_nested("asmg::nested_start");
  DLevel &F = dv->fine;
  const int J = dv->J, lc = dv->lc;
  dv->site = -1;  // these launches are not B_co's tuned sites
  const T *fT;
  if constexpr (sizeof(T) == 8) {
    fT = dv->f;
  } else {
    hipLaunchKernelGGL((k_convert<double, float>), dim3(nblk(F.n)), dim3(BS), 0, s, F.n, (const double *)dv->f,
                       F.b32);
    fT = F.b32;
  }
  spmv<T, 0>(dv, dv->PiT, fT, NV<T>::g(dv, J), s);
  for (int l = J; l > lc; --l) spmv<T, 0>(dv, dv->aux[l].PT, NV<T>::g(dv, l), NV<T>::g(dv, l - 1), s);
  if (dv->nc > 0)
    gemv<T>(dv->nc, cinv<T>(dv), (const T *)NV<T>::g(dv, lc), NV<T>::e(dv, lc), s);
  for (int l = lc + 1; l <= J; ++l) {
    DLevel &L = dv->aux[l];
    T *e = NV<T>::e(dv, l);
    const T *g = NV<T>::g(dv, l);
    spmv<T, 0>(dv, L.P, NV<T>::e(dv, l - 1), e, s);
    for (int k = 0; k < dv->nested; ++k) {
      residual<T>(dv, L, g, e, LV<T>::b(L), s, true);
      hipLaunchKernelGGL((k_gs_first<T>), dim3(nblk(L.n)), dim3(BS), 0, s, L.n, L.first_rows,
                         (const T *)LV<T>::b(L), LV<T>::id(L), LV<T>::x(L));
      vcycle<T>(dv, l, s);
      hipLaunchKernelGGL((k_add<T>), dim3(nblk(L.n)), dim3(BS), 0, s, L.n, (const T *)LV<T>::x(L), e);
    }
  }
  if constexpr (sizeof(T) == 8) {
    spmv<T, 0>(dv, dv->Pi, NV<T>::e(dv, J), dv->u, s);
  } else {
    spmv<T, 0>(dv, dv->Pi, NV<T>::e(dv, J), F.x32, s);
    hipLaunchKernelGGL((k_convert<float, double>), dim3(nblk(F.n)), dim3(BS), 0, s, F.n, (const float *)F.x32,
                       dv->u);
  }
  dv->site = 0;
  // r = f - A u, p = 0; done if the guess already meets the rule
  const int gt = red_grid(dv, F.n, F.A.lpr);
  with_lpr(F.A.lpr, [&](auto c) {
    constexpr int LP = decltype(c)::value;
    hipLaunchKernelGGL((k_cg_guess<LP>), dim3(gt), dim3(BS), 0, s, F.n, F.A.rp, F.A.ci, F.A.v64, F.dg64, dv->f,
                       dv->u, dv->r, dv->p, dv->partials);
  });
  hipLaunchKernelGGL(k_fin_guess, dim3(1), dim3(BS), 0, s, dv->partials, gt, dv->ctl);
}

// ---------------------------------------------------------------------------
// PCG driver
// ---------------------------------------------------------------------------

// z = B_co r, rho/beta, p = z + beta p (`first_done`: the CG update already ran the first
// colour pass of B_co on r)
template <class T>
static void pcg_tail(Device *dv, hipStream_t s, bool first_done) {
  const int n = dv->fine.n;
  apply_Bco<T>(dv, dv->r, first_done, s);
  const int g = red_grid(dv, n, 1);
  hipLaunchKernelGGL((k_cg_rz<T>), dim3(g), dim3(BS), 0, s, n, dv->r, (const T *)LV<T>::x(dv->fine), dv->ctl,
                     dv->partials);
  hipLaunchKernelGGL(k_fin_rz, dim3(1), dim3(BS), 0, s, dv->partials, g, dv->ctl);
  hipLaunchKernelGGL((k_cg_p<T>), dim3(nblk(n)), dim3(BS), 0, s, n, (const T *)LV<T>::x(dv->fine), dv->p, dv->ctl);
}

// Autotuner: for every candidate shape (twice), one eager B_co application on the current r with
// all slice sites in that shape and HIP events around each; every site then keeps the shape of
// its shortest time if that beats the default clearly (pick_shape). The solve that follows starts
// B_co from scratch.
template <class T>
static void tune(Device *dv, hipStream_t s) {
  const int pi = sizeof(T) == 4 ? 1 : 0;
  if (dv->tuned[pi] || !dv->autotune || dv->no_alloc) return;
  TraceRange tr_tune("asmg::autotune");
  const int K = kNumShapes;
  std::vector<std::vector<float>> t;
  dv->tuning = true;
  try {
    for (int round = 0; round < kTuneRounds; ++round)
      for (int k = 0; k < K; ++k) {
        dv->tune_k = k;
        dv->tune_live = 0;
        apply_Bco<T>(dv, dv->r, false, s);
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
  auto &tab = dv->shape[pi];
  tab.assign(t.size(), kShapes[0]);
  for (size_t site = 0; site < t.size(); ++site)
    tab[site] = kShapes[pick_shape(t[site])];
  dv->tune_times[pi] = t;
  dv->tuned[pi] = true;
}

template <class T>
static void pcg_iteration(Device *dv, hipStream_t s) {
  const int n = dv->fine.n;
  DLevel &F = dv->fine;
  int g = std::min<int>(dv->max_blocks, nblk((int64_t)F.sell.nslices * 64));
  hipLaunchKernelGGL(k_cg_spmv, dim3(g), dim3(BS), 0, s, F.sell.nslices, F.sell.srow, F.sell.soff, F.sell.scol,
                     F.sell.sv64, F.dg64, dv->p, dv->q, dv->ctl, dv->partials);
  hipLaunchKernelGGL(k_fin_spmv, dim3(1), dim3(BS), 0, s, dv->partials, g, dv->ctl);
  g = red_grid(dv, n, 1);
  hipLaunchKernelGGL((k_cg_axpy<T>), dim3(g), dim3(BS), 0, s, n, dv->u, dv->r, dv->p, dv->q, dv->ctl, dv->partials,
                     F.first_rows, LV<T>::id(F), LV<T>::b(F), LV<T>::x(F));
  hipLaunchKernelGGL(k_fin_axpy, dim3(1), dim3(BS), 0, s, dv->partials, g, dv->ctl);
  pcg_tail<T>(dv, s, true);
}

static void read_ctl(Device *dv, hipStream_t s) {
  HIPCHECK(hipMemcpyAsync(dv->ctl_host, dv->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
}

template <class T>
static void launch_iterations(Device *dv, int k, hipStream_t s) {
  const int pi = sizeof(T) == 4 ? 1 : 0;
  if (dv->use_graph && !dv->graph[pi]) {
    hipGraph_t g;
    HIPCHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    pcg_iteration<T>(dv, s);
    HIPCHECK(hipStreamEndCapture(s, &g));
    HIPCHECK(hipGraphInstantiate(&dv->graph[pi], g, nullptr, nullptr, 0));
    HIPCHECK(hipGraphDestroy(g));
  }
  for (int i = 0; i < k; ++i) {
    if (dv->use_graph)
      HIPCHECK(hipGraphLaunch(dv->graph[pi], s));
    else
      pcg_iteration<T>(dv, s);
  }
}

// x -= mean(x) over the fine unknowns (pure Neumann problems: the constants span the kernel of A)
static void project_mean(Device *dv, double *x, hipStream_t s) {
  const int n = dv->fine.n;
  const int g = red_grid(dv, n, 1);
  hipLaunchKernelGGL(k_sum, dim3(g), dim3(BS), 0, s, n, (const double *)x, dv->partials);
  hipLaunchKernelGGL(k_fin_mean, dim3(1), dim3(BS), 0, s, (const double *)dv->partials, g, n, dv->ctl);
  hipLaunchKernelGGL(k_sub_mean, dim3(nblk(n)), dim3(BS), 0, s, n, x, (const Ctl *)dv->ctl);
}

template <class T>
static int pcg(Device *dv, double tol, int *iters, double *true_rel, hipStream_t s) {
  TraceRange tr_pcg(sizeof(T) == 4 ? "asmg::pcg(mixed)" : "asmg::pcg(fp64)");
  const int n = dv->fine.n;
  const int pi = sizeof(T) == 4 ? 1 : 0;
  DLevel &F = dv->fine;
  const int gi = red_grid(dv, n, 1);
  if (dv->pure_neumann) project_mean(dv, dv->f, s);  // the part of f in the range of A
  hipLaunchKernelGGL(k_cg_init, dim3(gi), dim3(BS), 0, s, n, dv->f, dv->r, dv->u, dv->p, dv->partials);
  hipLaunchKernelGGL(k_fin_init, dim3(1), dim3(BS), 0, s, dv->partials, gi, tol, dv->maxit, dv->ctl);
  if (dv->nested > 0) nested_start<T>(dv, s);  // u = u_0, r = f - A u_0
  tune<T>(dv, s);  // first solve in this precision: pick the launch shapes
  pcg_tail<T>(dv, s, false);
  // host checks of the device flag: first after (previous count - 1) iterations, then every
  // iteration; with no history, every `check_every` (default 4) iterations
  int first = dv->last_iters[pi] > 1 ? dv->last_iters[pi] - 1 : 0;
  const int K = dv->check_every > 0 ? dv->check_every : (dv->last_iters[pi] > 0 ? 1 : 4);
  int restarts = 0;
  if (first > 0) {
    launch_iterations<T>(dv, std::min(first, dv->maxit), s);
  }
  while (true) {
    read_ctl(dv, s);
    if (!dv->ctl_host->done) {
      launch_iterations<T>(dv, K, s);
      continue;
    }
    // converged, broke down or hit max_iter: true residual in FP64
    const int gt = red_grid(dv, n, F.A.lpr);
    with_lpr(F.A.lpr, [&](auto c) {
      constexpr int LP = decltype(c)::value;
      hipLaunchKernelGGL((k_true_res<LP>), dim3(gt), dim3(BS), 0, s, n, F.A.rp, F.A.ci, F.A.v64, F.dg64, dv->f,
                         dv->u, dv->partials);
    });
    hipLaunchKernelGGL(k_fin_tr, dim3(1), dim3(BS), 0, s, dv->partials, gt, dv->ctl);
    read_ctl(dv, s);
    const Ctl &c = *dv->ctl_host;
    const double rel = c.fnorm2 > 0 ? std::sqrt(c.tr / c.fnorm2) : 0.0;
    // Converged on the recursively updated residual but the true residual is above tol: CG
    // restarts from the true residual (at most 3 times), as the oracle does. With the iteration
    // budget already spent the restart cannot take a step, and the solve ends unconverged.
    int status = c.status;
    if (status == ST_OK && rel > tol && restarts < 3) {
      if (c.iter >= dv->maxit) {
        status = ST_NOCONV;
      } else {
        ++restarts;
        with_lpr(F.A.lpr, [&](auto cc) {
          constexpr int LP = decltype(cc)::value;
          hipLaunchKernelGGL((k_cg_restart<LP>), dim3(nblk((int64_t)n * LP)), dim3(BS), 0, s, n, F.A.rp, F.A.ci,
                             F.A.v64, F.dg64, dv->f, dv->u, dv->r, dv->p, dv->ctl);
        });
        pcg_tail<T>(dv, s, false);
        continue;
      }
    }
    dv->restarts = restarts;
    dv->solve_iters = c.iter;
    if (iters) *iters = c.iter;
    if (true_rel) *true_rel = rel;
    if (status == ST_OK) dv->last_iters[pi] = c.iter;
    switch (status) {
      case ST_OK: return ASMG_OK;
      case ST_NOTSPD: return ASMG_ENOTSPD;
      case ST_NAN: return ASMG_ENAN;
      default: return ASMG_ENOCONV;
    }
  }
}

int device_solve(Device *dv, const double *d_f, double tol, double *d_u, int *iters, double *true_rel, void *stream) {
  HIPCHECK(hipSetDevice(dv->ordinal));
  hipStream_t cs = (hipStream_t)stream;
  hipStream_t s = dv->stream;
  const int n = dv->fine.n;
  if (n == 0) {
    if (iters) *iters = 0;
    if (true_rel) *true_rel = 0;
    return ASMG_OK;
  }
  HIPCHECK(hipEventRecord(dv->ev_in, cs));
  HIPCHECK(hipStreamWaitEvent(s, dv->ev_in, 0));
  hipLaunchKernelGGL(k_gather, dim3(nblk(n)), dim3(BS), 0, s, n, dv->perm_d, d_f, dv->f);
  const int rc = dv->precision == ASMG_PREC_MIXED ? pcg<float>(dv, tol, iters, true_rel, s)
                                                   : pcg<double>(dv, tol, iters, true_rel, s);
  if (dv->pure_neumann) project_mean(dv, dv->u, s);  // the solution with zero mean
  hipLaunchKernelGGL(k_scatter, dim3(nblk(n)), dim3(BS), 0, s, n, dv->perm_d, dv->u, d_u);
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipEventRecord(dv->ev_out, s));
  HIPCHECK(hipStreamWaitEvent(cs, dv->ev_out, 0));
  HIPCHECK(hipStreamSynchronize(s));
  return rc;
}

// Operator refresh from dv->kappa (already written on `s`)
static int refresh_operator(Device *dv, Hierarchy &h, hipStream_t s) {
  DLevel &F = dv->fine;
  if (!dv->rf_ready) {
    // element lists of every entry of A and the sliced-ELL slot of every entry: built once, at
    // the first refresh (they do not depend on kappa), so that setups that never refresh skip them
    std::vector<double> diag;
    HCsr H = permute(h.A, F.perm, &F.iperm, true, &diag);
    std::vector<int> slots;
    build_sell(dv, F, H, false, &slots);
    build_refresh(dv, h, H, slots);
    dv->rf_ready = true;
  }
  hipLaunchKernelGGL(k_refresh_off, dim3(nblk(F.A.nnz)), dim3(BS), 0, s, (int)F.A.nnz, dv->rf_off_ptr, dv->rf_off_el,
                     dv->rf_off_w, dv->kappa, F.A.v64, F.A.v32);
  hipLaunchKernelGGL(k_refresh_diag, dim3(nblk(F.n)), dim3(BS), 0, s, F.n, dv->rf_dg_ptr, dv->rf_dg_el, dv->rf_dg_w,
                     dv->kappa, F.dg64, F.id64, F.dg32, F.id32);
  hipLaunchKernelGGL(k_refresh_sell, dim3(nblk(dv->rf_nslots)), dim3(BS), 0, s, dv->rf_nslots, dv->rf_sell_map,
                     F.A.v64, F.sell.sv64, F.sell.sv32);
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipStreamSynchronize(s));
  return ASMG_OK;
}

// ---------------------------------------------------------------------------
// solve without allocation
// ---------------------------------------------------------------------------

// Scratch of device_solve_noalloc: the PCG control block at offset 0, the reduction partials
// (at most RED_BLOCKS doubles) from offset kScratchPartials. One copy per GPU, held until the
// process ends. In host code `scratch` names a host-side stand-in: only the address that
// hipGetSymbolAddress returns for the current device may reach a kernel or a copy.
static constexpr size_t kScratchPartials = 256;
static constexpr size_t kScratchBytes = kScratchPartials + sizeof(double) * RED_BLOCKS;
static_assert(sizeof(Ctl) <= kScratchPartials, "control block larger than its scratch slot");
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxScratchDevices] = {};

// device address of `scratch` on device `ordinal`, looked up once per device with that device
// current (the caller has made it current)
static void *scratch_address(int ordinal) {
  if (ordinal < 0 || ordinal >= kMaxScratchDevices)
    throw AsmgError{ASMG_EDEVICE, "device ordinal beyond the scratch table"};
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[ordinal]) {
    void *p = nullptr;
    HIPCHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw AsmgError{ASMG_EDEVICE, "no device address for the solver scratch"};
    g_scratch_ptr[ordinal] = p;
  }
  return g_scratch_ptr[ordinal];
}

int device_solve_noalloc(Device *dv, const double *d_f, double tol, double *d_u, int *iters, double *true_rel,
                         void *stream) {
  HIPCHECK(hipSetDevice(dv->ordinal));
  if (kScratchPartials + sizeof(double) * (size_t)dv->max_blocks > kScratchBytes)
    throw AsmgError{ASMG_EINVAL, "reduction grid of this handle exceeds the solver scratch (" +
                                     std::to_string(kScratchBytes) + " bytes)"};
  unsigned char *base = (unsigned char *)scratch_address(dv->ordinal);
  // the handle's own control block and partials are swapped for the scratch for this call; the
  // iteration runs as eager launches (a captured graph holds the handle's own pointers) and
  // never autotunes (the shapes tuned by earlier solves, or the defaults, are used). k_fin_init
  // writes every control field a later kernel or the host reads, so nothing needs clearing.
  struct Swap {
    Device *dv;
    Ctl *ctl;
    double *partials;
    bool graph;
    ~Swap() {
      dv->ctl = ctl;
      dv->partials = partials;
      dv->use_graph = graph;
      dv->no_alloc = false;
    }
  } swap{dv, dv->ctl, dv->partials, dv->use_graph};
  dv->ctl = (Ctl *)base;
  dv->partials = (double *)(base + kScratchPartials);
  dv->use_graph = false;
  dv->no_alloc = true;
  return device_solve(dv, d_f, tol, d_u, iters, true_rel, stream);
}

int device_set_coefficient(Device *dv, Hierarchy &h, const double *d_kappa, void *stream) {
  HIPCHECK(hipSetDevice(dv->ordinal));
  hipStream_t s = (hipStream_t)stream;
  HIPCHECK(hipMemcpyAsync(dv->kappa, d_kappa, (size_t)dv->ne * 8, hipMemcpyDeviceToDevice, s));
  return refresh_operator(dv, h, s);
}

int device_set_log_coefficient(Device *dv, Hierarchy &h, const double *d_m, void *stream) {
  HIPCHECK(hipSetDevice(dv->ordinal));
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_exp, dim3(nblk(dv->ne)), dim3(BS), 0, s, (int)dv->ne, d_m, dv->kappa);
  return refresh_operator(dv, h, s);
}

int device_restarts(const Device *dv) { return dv->restarts; }
int device_last_iterations(const Device *dv) { return dv->solve_iters; }

int device_solve_host(Device *dv, const double *f, double tol, double *u, int *iters, double *true_rel) {
  HIPCHECK(hipSetDevice(dv->ordinal));
  const int n = dv->fine.n;
  if (n > 0) HIPCHECK(hipMemcpy(dv->io_in, f, (size_t)n * 8, hipMemcpyHostToDevice));
  const int rc = device_solve(dv, dv->io_in, tol, dv->io_out, iters, true_rel, nullptr);
  if (n > 0) HIPCHECK(hipMemcpy(u, dv->io_out, (size_t)n * 8, hipMemcpyDeviceToHost));
  return rc;
}

int device_apply_B(Device *dv, const double *d_r, double *d_z, int precision, void *stream) {
  HIPCHECK(hipSetDevice(dv->ordinal));
  hipStream_t s = (hipStream_t)stream;
  const int n = dv->fine.n;
  if (n == 0) return ASMG_OK;
  hipLaunchKernelGGL(k_gather, dim3(nblk(n)), dim3(BS), 0, s, n, dv->perm_d, d_r, dv->f);
  if (precision == ASMG_PREC_MIXED) {
    apply_Bco<float>(dv, dv->f, false, s);
    hipLaunchKernelGGL((k_scatter_cvt<float>), dim3(nblk(n)), dim3(BS), 0, s, n, dv->perm_d,
                       (const float *)dv->fine.x32, d_z);
  } else {
    apply_Bco<double>(dv, dv->f, false, s);
    hipLaunchKernelGGL((k_scatter_cvt<double>), dim3(nblk(n)), dim3(BS), 0, s, n, dv->perm_d,
                       (const double *)dv->fine.x64, d_z);
  }
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipStreamSynchronize(s));
  return ASMG_OK;
}

int device_matvec(Device *dv, const double *d_x, double *d_y, void *stream) {
  HIPCHECK(hipSetDevice(dv->ordinal));
  hipStream_t s = (hipStream_t)stream;
  const int n = dv->fine.n;
  if (n == 0) return ASMG_OK;
  DLevel &F = dv->fine;
  hipLaunchKernelGGL(k_gather, dim3(nblk(n)), dim3(BS), 0, s, n, dv->perm_d, d_x, dv->p);
  with_lpr(F.A.lpr, [&](auto c) {
    constexpr int LP = decltype(c)::value;
    hipLaunchKernelGGL((k_matvec<LP>), dim3(nblk((int64_t)n * LP)), dim3(BS), 0, s, n, F.A.rp, F.A.ci, F.A.v64,
                       F.dg64, dv->p, dv->q);
  });
  hipLaunchKernelGGL(k_scatter, dim3(nblk(n)), dim3(BS), 0, s, n, dv->perm_d, dv->q, d_y);
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipStreamSynchronize(s));
  return ASMG_OK;
}

int device_element_gradient(Device *dv, const double *d_u, const double *d_lam, double *d_g, double scale,
                            void *stream) {
  HIPCHECK(hipSetDevice(dv->ordinal));
  hipStream_t s = (hipStream_t)stream;
  if (dv->d == 2)
    hipLaunchKernelGGL((k_elem_grad<2>), dim3(nblk(dv->ne)), dim3(BS), 0, s, (int)dv->ne, dv->coords, dv->elems,
                       dv->kappa, dv->dof_of_vertex, d_u, d_lam, d_g, scale);
  else
    hipLaunchKernelGGL((k_elem_grad<3>), dim3(nblk(dv->ne)), dim3(BS), 0, s, (int)dv->ne, dv->coords, dv->elems,
                       dv->kappa, dv->dof_of_vertex, d_u, d_lam, d_g, scale);
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipStreamSynchronize(s));
  return ASMG_OK;
}

// tile lists of the LDS-staged product, built from the fine sliced ELL on the device (once)
static void build_lds_tiles(Device *dv) {
  if (dv->lds_toff) return;
  const DSell &S = dv->fine.sell;
  const int ns = S.nslices;
  std::vector<int> soff(ns + 1), scol(S.entries);
  HIPCHECK(hipMemcpy(soff.data(), S.soff, (size_t)(ns + 1) * 4, hipMemcpyDeviceToHost));
  if (S.entries) HIPCHECK(hipMemcpy(scol.data(), S.scol, (size_t)S.entries * 4, hipMemcpyDeviceToHost));
  const int per = BS / 64;
  const int nt = (ns + per - 1) / per;
  std::vector<int> toff(nt + 1, 0), list;
  std::vector<uint16_t> lcol(S.entries);
  int maxm = 0;
  for (int t = 0; t < nt; ++t) {
    const int e0 = soff[t * per], e1 = soff[std::min(ns, (t + 1) * per)];
    std::vector<int> u(scol.begin() + e0, scol.begin() + e1);
    std::sort(u.begin(), u.end());
    u.erase(std::unique(u.begin(), u.end()), u.end());
    if (u.size() > 65535) throw AsmgError{ASMG_EINVAL, "tile with more than 65535 distinct columns"};
    for (int e = e0; e < e1; ++e)
      lcol[e] = (uint16_t)(std::lower_bound(u.begin(), u.end(), scol[e]) - u.begin());
    list.insert(list.end(), u.begin(), u.end());
    toff[t + 1] = (int)list.size();
    maxm = std::max(maxm, (int)u.size());
  }
  if ((size_t)maxm * 8 > 65536) throw AsmgError{ASMG_EINVAL, "LDS-staged product: a tile needs more than 64 KiB"};
  dv->lds_toff = dupload(dv, toff);
  dv->lds_list = dupload(dv, list);
  dv->lds_lcol = dupload(dv, lcol);
  dv->lds_ntiles = nt;
  dv->lds_maxm = maxm;
  dv->lds_nlist = (int64_t)list.size();
}

__global__ __launch_bounds__(BS) void k_pattern(int n, double *__restrict__ x) {
  const int i = blockIdx.x * BS + threadIdx.x;
  if (i < n) x[i] = 1.0 + 0.25 * (double)((i * 7919) % 61) - 0.5 * (double)(i % 3);
}

int device_time_kernel(Device *dv, int which, int reps, int precision, void *stream, double *ms, double *bytes) {
  HIPCHECK(hipSetDevice(dv->ordinal));
  hipStream_t s = (hipStream_t)stream;
  DLevel &F = dv->fine;
  const int n = F.n;
  const bool mixed = which == 3 ? dv->precision == ASMG_PREC_MIXED : precision == ASMG_PREC_MIXED;
  auto bco_on = [&](hipStream_t st) {
    if (mixed)
      apply_Bco<float>(dv, dv->f, false, st);
    else
      apply_Bco<double>(dv, dv->f, false, st);
  };
  auto bco = [&]() { bco_on(s); };
  int g6 = std::min<int>(dv->max_blocks, nblk((int64_t)F.sell.nslices * 64));
  if (which == 7) build_lds_tiles(dv);
  const int g7 = std::max(1, std::min(dv->lds_ntiles, 8 * 256));
  auto one = [&]() {
    if (which == 7) {
      hipLaunchKernelGGL(k_cg_spmv_lds, dim3(g7), dim3(BS), (size_t)std::max(dv->lds_maxm, 1) * 8, s, dv->lds_ntiles,
                         F.sell.nslices, F.sell.srow, F.sell.soff, dv->lds_lcol, F.sell.sv64, dv->lds_toff,
                         dv->lds_list, F.dg64, dv->p, dv->q, dv->partials);
    } else if (which == 6) {
      hipLaunchKernelGGL(k_cg_spmv, dim3(g6), dim3(BS), 0, s, F.sell.nslices, F.sell.srow, F.sell.soff, F.sell.scol,
                         F.sell.sv64, F.dg64, dv->p, dv->q, dv->ctl, dv->partials);
    } else if (which == 0) {
      with_lpr(F.A.lpr, [&](auto c) {
        constexpr int LP = decltype(c)::value;
        hipLaunchKernelGGL((k_matvec<LP>), dim3(nblk((int64_t)n * LP)), dim3(BS), 0, s, n, F.A.rp, F.A.ci, F.A.v64,
                           F.dg64, dv->p, dv->q);
      });
    } else if (which == 1) {
      if (mixed)
        sweep<float>(dv, F, F.x32, F.b32, false, false, true, s);
      else
        sweep<double>(dv, F, F.x64, F.b64, false, false, true, s);
    } else {
      bco();
    }
  };
  if (which == 7 && n > 0) {
    // check the staged product against the solve's product on a nonzero p before timing it
    hipLaunchKernelGGL(k_pattern, dim3(nblk(n)), dim3(BS), 0, s, n, dv->p);
    HIPCHECK(hipMemsetAsync(dv->ctl, 0, sizeof(Ctl), s));
    hipLaunchKernelGGL(k_cg_spmv, dim3(g6), dim3(BS), 0, s, F.sell.nslices, F.sell.srow, F.sell.soff, F.sell.scol,
                       F.sell.sv64, F.dg64, dv->p, dv->q, dv->ctl, dv->partials);
    std::vector<double> q6(n), q7(n);
    HIPCHECK(hipMemcpyAsync(q6.data(), dv->q, (size_t)n * 8, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    one();
    HIPCHECK(hipMemcpyAsync(q7.data(), dv->q, (size_t)n * 8, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    double dmax = 0, qmax = 0;
    for (int i = 0; i < n; ++i) {
      dmax = std::max(dmax, std::fabs(q6[i] - q7[i]));
      qmax = std::max(qmax, std::fabs(q6[i]));
    }
    if (dmax > 1e-14 * qmax) throw AsmgError{ASMG_EDEVICE, "LDS-staged product differs from the solve's product"};
  }
  HIPCHECK(hipMemsetAsync(dv->p, 0, (size_t)n * 8, s));
  HIPCHECK(hipMemsetAsync(dv->f, 0, (size_t)n * 8, s));
  HIPCHECK(hipMemsetAsync(F.b64, 0, (size_t)n * 8, s));
  HIPCHECK(hipMemsetAsync(F.b32, 0, (size_t)n * 4, s));
  if (which == 4 || which == 5) {
    // every Gauss-Seidel colour pass (k_sell<0, T>) inside `reps` full B_co applications, each
    // launch stamped with its own start and end events (one launch per event pair: the caches
    // are as in a solve)
    bco();  // warm-up
    dv->probe_lpr = 1;
    dv->probe_prec = mixed ? 1 : 0;
    dv->probe_used = 0;
    dv->probe_bytes.clear();
    for (int k = 0; k < reps; ++k) bco();
    dv->probe_lpr = 0;
    HIPCHECK(hipStreamSynchronize(s));
    double tot = 0;
    const size_t nl = dv->probe_used / 2;
    for (size_t i = 0; i < nl; ++i) {
      float t = 0;
      HIPCHECK(hipEventElapsedTime(&t, dv->probe_ev[2 * i], dv->probe_ev[2 * i + 1]));
      tot += t;
    }
    double by = 0;
    for (double b : dv->probe_bytes) by += b;
    *ms = nl ? tot / nl : 0.0;
    *bytes = nl ? by / nl : 0.0;
    return ASMG_OK;
  }
  hipEvent_t e0, e1;
  HIPCHECK(hipEventCreate(&e0));
  HIPCHECK(hipEventCreate(&e1));
  // byte model of one launch
  dv->count_bytes = true;
  dv->bytes = 0;
  if (which == 0 || which == 6)
    dv->bytes = csr_bytes(F.A, 8) + 8.0 * n * 3 + (which == 6 ? 8.0 * g6 : 8.0 * n);
  else if (which == 7)  // entries (8-byte value, 2-byte position), the lists and the staged p, rows
    dv->bytes = 10.0 * (double)F.A.nnz + 12.0 * (double)dv->lds_nlist + 4.0 * (dv->lds_ntiles + 1) + 8.0 * n * 3 +
                8.0 * g7;
  else
    one();
  if (which == 6) {
    // the PCG product reads the control block's `done` flag: clear it (the next solve sets
    // every field it reads)
    HIPCHECK(hipMemsetAsync(dv->ctl, 0, sizeof(Ctl), s));
  }
  dv->count_bytes = false;
  *bytes = dv->bytes;
  if (which == 2 || which == 3) {
    // one B_co application captured in a hipGraph, as the solve runs it: median over `reps`
    // replays, each between its own pair of events (on the handle's stream, after `s` drained)
    HIPCHECK(hipEventDestroy(e0));
    HIPCHECK(hipEventDestroy(e1));
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
    HIPCHECK(hipGetLastError());
    return ASMG_OK;
  }
  one();  // warm-up
  HIPCHECK(hipEventRecord(e0, s));
  for (int k = 0; k < reps; ++k) one();
  HIPCHECK(hipEventRecord(e1, s));
  HIPCHECK(hipEventSynchronize(e1));
  float t = 0;
  HIPCHECK(hipEventElapsedTime(&t, e0, e1));
  *ms = (double)t / reps;
  HIPCHECK(hipEventDestroy(e0));
  HIPCHECK(hipEventDestroy(e1));
  HIPCHECK(hipGetLastError());
  return ASMG_OK;
}

std::vector<int64_t> device_tuned_shapes(Device *dv, int precision) {
  std::vector<int64_t> out;
  if (precision < 0 || precision > 1) return out;
  for (const auto &sh : dv->shape[precision]) {
    out.push_back(sh.threads);
    out.push_back(sh.xcd);
    out.push_back(sh.var);
  }
  return out;
}

std::vector<double> device_tune_times(Device *dv, int precision) {
  std::vector<double> out;
  if (precision < 0 || precision > 1) return out;
  for (const auto &row : dv->tune_times[precision])
    for (float t : row) out.push_back(std::isfinite(t) ? (double)t : -1.0);
  return out;
}

}  // namespace asmg
