// Device helpers shared by the single-mesh engine (device.hip) and the batched engine (batch.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <type_traits>

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

// sum over a 256-thread block; result valid in thread 0
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double sm[BS / 64];
  v = group_sum<64>(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sm[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < BS / 64; ++i) r += sm[i];
  }
  return r;
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
