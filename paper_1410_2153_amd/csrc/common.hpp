// Device helpers shared by the single-mesh engine (device.hip) and the batched engine (batch.hip).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "setup.hpp"

namespace asmg {

#define HIPCHECK(x)                                                                                    \
  do {                                                                                                 \
    hipError_t e_ = (x);                                                                               \
    if (e_ != hipSuccess) throw AsmgError{ASMG_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)}; \
  } while (0)

static constexpr int BS = 256;  // threads per block (4 waves)

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------

template <int W, class T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, W);
  return v;
}

// Sums of NR values over a 256-thread block in one pass; results valid in thread 0. Every wave
// stores its NR partial sums, one barrier, then thread 0 adds them in wave order. The shared
// array is not reused after the barrier, so a kernel calls this at most once (a second call
// could overwrite sm while thread 0 still reads it).
template <int NR>
__device__ __forceinline__ void block_sum_n(double v[NR]) {
  __shared__ double sm[NR][BS / 64];
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    v[q] = group_sum<64>(v[q]);
    if ((threadIdx.x & 63) == 0) sm[q][w] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    double r = 0.0;
    if (threadIdx.x == 0) {
      for (int i = 0; i < BS / 64; ++i) r += sm[q][i];
    }
    v[q] = r;
  }
}

// sum over a 256-thread block; result valid in thread 0 (once per kernel, as block_sum_n)
__device__ __forceinline__ double block_sum(double v) {
  double a[1] = {v};
  block_sum_n<1>(a);
  return a[0];
}

// XCD-aware block index. Workgroups are dealt to the 8 XCDs round-robin (block b to XCD b % 8),
// and each XCD has its own L2. This bijection of [0, gridDim.x) gives XCD x a contiguous run of
// logical blocks, so rows that are neighbours in the numbering (and gather the same entries of
// x) are served by one L2.
__device__ __forceinline__ int xcd_block() {
  const int nb = (int)gridDim.x, b = (int)blockIdx.x;
  const int x = b & 7, i = b >> 3, per = nb >> 3, rem = nb & 7;
  return x * per + (x < rem ? x : rem) + i;
}

// Tunable launch shape of the V-cycle slice kernels: blocks of `threads` / 64 waves (one slice
// per wave), taken in XCD-contiguous order (xcd = 1) or in dispatch order (xcd = 0), passed to
// the kernel as one int shape = 2 * waves per block + xcd. (The block size comes in as an
// argument because blockDim.x is a 16-bit field of the dispatch packet: reading it costs a
// vector memory load at kernel start, on the critical path of these latency-bound kernels.)
static constexpr int BS_MAX = 512;

static inline int shape_arg(int threads, int xcd) { return 2 * (threads >> 6) + (xcd ? 1 : 0); }

__device__ __forceinline__ int tuned_slice(int first, int shape) {
  const int xb = xcd_block();  // both orders computed: no branch between the kernel-argument loads
  const int blk = (shape & 1) ? xb : (int)blockIdx.x;
  return first + blk * (shape >> 1) + __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
}

// Candidate launch shapes of the autotuner: threads per block, XCD order, and the kernel variant
// `var`: 0 = one slice per wave; 1 = a grid of at most kLoopWaves waves loops over the slices
// (grid-stride), loading the next slice's header (row index per lane, entry offsets) before the
// current slice's entries, so its latency overlaps the current slice's work. The first candidate
// is the default. Each candidate is timed kTuneRounds times per launch site (best of), and a site
// leaves the default only for a candidate faster by kTuneMargin of the default's time and by at
// least kTuneFloorMs: timings of kernels of a few microseconds are noisy, and a pick on noise
// costs more than it gains.
struct Shape {
  int threads, xcd, var;
};
static const Shape kShapes[] = {{256, 1, 0}, {128, 1, 0}, {512, 1, 0}, {256, 0, 0}, {128, 0, 0},
                                {512, 0, 0}, {256, 1, 1}, {512, 1, 1}, {256, 0, 1}, {512, 0, 1}};
static constexpr int kNumShapes = (int)(sizeof(kShapes) / sizeof(kShapes[0]));
static constexpr int kTuneRounds = 3;
static constexpr float kTuneMargin = 0.02f;
static constexpr float kTuneFloorMs = 0.0005f;
// resident waves of one round of the loop variant: 256 CUs x 16 waves
static constexpr int kLoopWaves = 4096;

// calls f(std::integral_constant<int, var>) for the compiled kernel variants
template <class F>
static void with_var(int var, F &&f) {
  if (var == 1)
    f(std::integral_constant<int, 1>());
  else
    f(std::integral_constant<int, 0>());
}

// blocks of a slice-kernel launch over `nslices` slices (64 rows each) with `threads`-thread blocks
static inline int slice_blocks(int nslices, int threads, int var = 0) {
  const int b = std::max(1, (nslices * 64 + threads - 1) / threads);
  return var == 1 ? std::min(b, std::max(1, kLoopWaves / (threads / 64))) : b;
}

// The slices [s0, s1) of a slice-kernel launch, each handed to body(row, o0, w): the lane's row
// (-1 on empty lanes), the slice's first entry offset and its width. Slice s's entries end at
// send[s]: soff + 1 for whole slices, or an array of earlier ends (a prefix of every row's
// entries). VAR 0: one slice per wave. VAR 1: grid-stride loop, with the next slice's header
// loaded before body runs on this one.
template <int VAR, class F>
__device__ __forceinline__ void for_slices(int s0, int s1, int shape, const int *__restrict__ srow,
                                           const int *__restrict__ soff, const int *__restrict__ send, F &&body) {
  int s = tuned_slice(s0, shape);
  if (s >= s1) return;
  const int lane = threadIdx.x & 63;
  int row = srow[(size_t)s * 64 + lane];
  int o0 = soff[s], o1 = send[s];
  if constexpr (VAR == 0) {
    body(row, o0, (o1 - o0) >> 6);
  } else {
    const int stride = (int)gridDim.x * (shape >> 1);
    while (true) {
      const int sn = s + stride;
      int rn = -1, p0 = 0, p1 = 0;
      if (sn < s1) {
        rn = srow[(size_t)sn * 64 + lane];
        p0 = soff[sn];
        p1 = send[sn];
      }
      body(row, o0, (o1 - o0) >> 6);
      if (sn >= s1) break;
      s = sn;
      row = rn;
      o0 = p0;
      o1 = p1;
    }
  }
}

// Launch of a kernel over `grid` blocks of `threads`; with an event pair (timing runs only, never
// under stream capture) the events are stamped with the kernel's own start and end
// (hipExtLaunchKernel), so that their interval excludes the launch gaps around the kernel.
template <class K, class... A>
static void launch_timed(K kernel, int grid, int threads, hipStream_t s, hipEvent_t e0, hipEvent_t e1, A... args) {
  if (e0) {
    hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(threads), 0, s, e0, e1, 0, args...);
    HIPCHECK(hipGetLastError());
  } else {
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(threads), 0, s, args...);
  }
}

// index into kShapes picked from one site's best times per candidate (INFINITY = not timed)
static inline int pick_shape(const std::vector<float> &t) {
  const int k = (int)(std::min_element(t.begin(), t.end()) - t.begin());
  return t[0] - t[k] > std::max(kTuneMargin * t[0], kTuneFloorMs) ? k : 0;
}

// ---------------------------------------------------------------------------
// sparse kernels
// ---------------------------------------------------------------------------

template <int LPR, class T>
__device__ __forceinline__ T row_dot(const int *__restrict__ rp, const int *__restrict__ ci,
                                     const T *__restrict__ av, const T *__restrict__ x, int row, bool act,
                                     int lane) {
  T s = 0;
  if (act) {
    const int b = rp[row], e = rp[row + 1];
    for (int k = b + lane; k < e; k += LPR) s += av[k] * x[ci[k]];
  }
  return group_sum<LPR>(s);
}

template <class F>
static void with_lpr(int lpr, F &&f) {
  switch (lpr) {
    case 2: f(std::integral_constant<int, 2>()); break;
    case 4: f(std::integral_constant<int, 4>()); break;
    case 8: f(std::integral_constant<int, 8>()); break;
    default: f(std::integral_constant<int, 16>()); break;
  }
}

static inline int nblk(int64_t threads) { return (int)std::max<int64_t>(1, (threads + BS - 1) / BS); }

static inline int pick_lpr(int64_t nnz, int64_t rows) {
  if (rows <= 0) return 4;
  const double avg = (double)nnz / (double)rows;
  if (avg <= 2.0) return 2;
  if (avg <= 4.0) return 4;
  if (avg <= 8.0) return 8;
  return 16;
}

}  // namespace asmg
