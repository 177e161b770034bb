// Multicolour orderings on the device (the Gauss-Seidel smoother's colouring, setup step of the
// smoother of Section 4.1), for the hash order: every row i has the priority
// (fmix32(i ^ seed), i), compared lexicographically, and the host's greedy colouring visits the
// rows by decreasing priority, each row taking the smallest colour that none of its already
// coloured neighbours holds.
//
// Jones-Plassmann rounds give the same colouring: in each round, every uncoloured row whose
// priority exceeds that of all its uncoloured neighbours takes the smallest colour unused by its
// coloured neighbours. When such a row is coloured, exactly its higher-priority neighbours are
// coloured, with the colours the sequential order gives them (induction over the priority
// order), so its colour is the sequential one too. Two rows coloured in one round are never
// neighbours, and each round reads the colours of the round before (two arrays), so the result
// does not depend on the order in which the device runs the rows.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "common.hpp"
#include "setup.hpp"
#include "tree.hpp"

namespace asmg {
namespace {

constexpr int CB = 256;

__device__ __forceinline__ uint32_t d_fmix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x85ebca6bu;
  x ^= x >> 13;
  x *= 0xc2b2ae35u;
  x ^= x >> 16;
  return x;
}

// a before b in the host's visiting order
__device__ __forceinline__ bool d_before(uint32_t wa, int a, uint32_t wb, int b) {
  return wa > wb || (wa == wb && a > b);
}

__global__ __launch_bounds__(CB) void k_jp_round(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                  uint32_t seed, const int *__restrict__ cin, int *__restrict__ cout,
                                                  int *__restrict__ left) {
  const int i = blockIdx.x * CB + threadIdx.x;
  if (i >= n) return;
  const int ci0 = cin[i];
  if (ci0 >= 0) {
    cout[i] = ci0;
    return;
  }
  const uint32_t wi = d_fmix32((uint32_t)i ^ seed);
  uint64_t used = 0;  // colours 0..63 held by coloured neighbours
  bool ready = true, wide = false;
  for (int p = rp[i]; p < rp[i + 1]; ++p) {
    const int j = ci[p];
    if (j == i) continue;
    const int cj = cin[j];
    if (cj < 0) {
      if (d_before(d_fmix32((uint32_t)j ^ seed), j, wi, i)) {
        ready = false;
        break;
      }
    } else if (cj < 64) {
      used |= (uint64_t)1 << cj;
    } else {
      wide = true;
    }
  }
  if (!ready) {
    cout[i] = -1;
    atomicAdd(left, 1);
    return;
  }
  int c = 64;
  if (!wide && used != ~(uint64_t)0) c = __ffsll((long long)~used) - 1;  // lowest clear bit
  if (wide || c >= 64) {
    // more than 64 colours around this row: smallest colour not held, by scanning upwards
    for (c = 0;; ++c) {
      bool held = false;
      for (int p = rp[i]; p < rp[i + 1] && !held; ++p) {
        const int j = ci[p];
        held = j != i && cin[j] == c;
      }
      if (!held) break;
    }
  }
  cout[i] = c;
}

__global__ __launch_bounds__(CB) void k_fill_int(int n, int *__restrict__ x, int v) {
  const int i = blockIdx.x * CB + threadIdx.x;
  if (i < n) x[i] = v;
}

std::vector<int32_t> jp_colouring(const Csr &A, uint32_t seed, int *d_rp, int *d_ci, int *d_c0, int *d_c1,
                                  int *d_left, hipStream_t s) {
  const int n = (int)A.nrows;
  std::vector<int32_t> col(n);
  if (n == 0) return col;
  std::vector<int> rp(A.rp.begin(), A.rp.end());
  HIPCHECK(hipMemcpyAsync(d_rp, rp.data(), (size_t)(n + 1) * 4, hipMemcpyHostToDevice, s));
  if (A.nnz()) HIPCHECK(hipMemcpyAsync(d_ci, A.ci.data(), (size_t)A.nnz() * 4, hipMemcpyHostToDevice, s));
  const int nb = (n + CB - 1) / CB;
  hipLaunchKernelGGL(k_fill_int, dim3(nb), dim3(CB), 0, s, n, d_c0, -1);
  int *cin = d_c0, *cout = d_c1;
  int left = n;
  // each round colours at least the uncoloured row of highest priority: at most n rounds
  for (int round = 0; left > 0 && round <= n; ++round) {
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(CB), 0, s, 1, d_left, 0);
    hipLaunchKernelGGL(k_jp_round, dim3(nb), dim3(CB), 0, s, n, d_rp, d_ci, seed, (const int *)cin, cout, d_left);
    HIPCHECK(hipMemcpyAsync(&left, d_left, 4, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    std::swap(cin, cout);
  }
  if (left > 0) throw AsmgError{ASMG_EDEVICE, "device colouring did not finish"};
  HIPCHECK(hipMemcpyAsync(col.data(), cin, (size_t)n * 4, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  return col;
}

}  // namespace

void build_colourings_device(Hierarchy &h, int ordinal) {
  if (h.opt.colouring != 1) throw AsmgError{ASMG_EINVAL, "the device colouring runs the hash order only"};
  HIPCHECK(hipSetDevice(ordinal));
  std::vector<const Csr *> mats{&h.A};
  std::vector<int> lv{0};
  for (int l = h.lc + 1; l <= h.J; ++l) {
    mats.push_back(&h.Al.at(l));
    lv.push_back(l);
  }
  int64_t nmax = 1, zmax = 1;
  for (const Csr *A : mats) {
    nmax = std::max<int64_t>(nmax, A->nrows);
    zmax = std::max<int64_t>(zmax, A->nnz());
  }
  if (nmax >= (int64_t)1 << 31 || zmax >= (int64_t)1 << 31)
    throw AsmgError{ASMG_EINVAL, "matrix too large for the device colouring"};
  int *d_rp = nullptr, *d_ci = nullptr, *d_c0 = nullptr, *d_c1 = nullptr, *d_left = nullptr;
  hipStream_t s = nullptr;
  auto release = [&]() {
    if (s) (void)hipStreamSynchronize(s);  // nothing in flight reads the buffers below
    if (d_rp) (void)hipFree(d_rp);
    if (d_ci) (void)hipFree(d_ci);
    if (d_c0) (void)hipFree(d_c0);
    if (d_c1) (void)hipFree(d_c1);
    if (d_left) (void)hipFree(d_left);
    if (s) (void)hipStreamDestroy(s);
  };
  try {
    HIPCHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    HIPCHECK(hipMalloc(&d_rp, (size_t)(nmax + 1) * 4));
    HIPCHECK(hipMalloc(&d_ci, (size_t)zmax * 4));
    HIPCHECK(hipMalloc(&d_c0, (size_t)nmax * 4));
    HIPCHECK(hipMalloc(&d_c1, (size_t)nmax * 4));
    HIPCHECK(hipMalloc(&d_left, 4));
    std::vector<std::vector<int32_t>> out(mats.size());
    for (size_t t = 0; t < mats.size(); ++t)
      out[t] = jp_colouring(*mats[t], h.opt.colour_seed, d_rp, d_ci, d_c0, d_c1, d_left, s);
    h.colour_fine = std::move(out[0]);
    h.colour_aux.clear();
    for (size_t t = 1; t < mats.size(); ++t) h.colour_aux[lv[t]] = std::move(out[t]);
  } catch (...) {
    release();
    throw;
  }
  release();
}

}  // namespace asmg
