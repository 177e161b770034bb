// Cluster tree on the device (Sections 3.1-3.2): root box, barycenter keys, Morton sort,
// refinement by cluster size, closure, leaves and the leaf coefficients kappa~.
//
// The host setup (build_tree in setup.cpp) computes the same objects with hash sets; this path
// produces identical results (same IEEE operations for the keys, the same least closed set,
// the same summation order for kappa~) and hands them to the rest of the host setup.
//
// Data on the device: box codes are 64-bit Morton codes with a leading marker bit (level l box:
// 1 << d(l-1) | interleaved index bits, axis 0 most significant within a bit group), so that
// the codes of one level are contiguous and a sorted code array is sorted by (level, Morton).
//   - Elements: code at level D+1 (D = 30 in 2-D, 20 in 3-D), sorted with the element id as
//     the tie-break (stable radix sort of (code, id) pairs).
//   - R0: a box of level l <= D is refined iff more than n_min barycenters fall in it; in the
//     sorted codes that is "the code n_min places further has the same level-l prefix".
//   - Closure: least superset of R0 closed under "b refined (level >= 2), q a same-level box
//     sharing a facet (3-D: or an edge) with b => parent(q) refined". Rounds over a frontier:
//     candidates from the frontier, sorted and deduplicated, merged into the sorted R.
//   - Leaves: children of refined boxes that are not refined (the root if R is empty).
//   - kappa~: mean coefficient of the leaf's cluster, or of the nearest non-empty ancestor's,
//     summed sequentially in sorted order.
//   - The leaves go back in the host's order, (level, index tuple): two stable radix passes,
//     by the packed index tuple and then by the level.
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

constexpr int TB = 256;

__device__ __forceinline__ int d_level(uint64_t c, int d) { return (63 - __clzll((long long)c)) / d + 1; }

__device__ __forceinline__ void d_index(uint64_t c, int d, int64_t *idx) {
  const int bits = d_level(c, d) - 1;
  for (int k = 0; k < d; ++k) idx[k] = 0;
  for (int b = 0; b < bits; ++b)
    for (int k = 0; k < d; ++k) idx[k] |= (int64_t)((c >> (b * d + (d - 1 - k))) & 1) << b;
}

__device__ __forceinline__ uint64_t d_code(int level, const int64_t *idx, int d) {
  uint64_t m = 0;
  const int bits = level - 1;
  for (int b = 0; b < bits; ++b)
    for (int k = 0; k < d; ++k) m |= (uint64_t)((idx[k] >> b) & 1) << (b * d + (d - 1 - k));
  return m | ((uint64_t)1 << (d * bits));
}

// first position in sorted a[0, n) with a[i] >= v
__device__ __forceinline__ int64_t d_lower(const uint64_t *a, int64_t n, uint64_t v) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

__device__ __forceinline__ bool d_member(const uint64_t *a, int64_t n, uint64_t v) {
  const int64_t i = d_lower(a, n, v);
  return i < n && a[i] == v;
}

// per-block minima and maxima of each coordinate axis
__global__ __launch_bounds__(TB) void k_extent(int64_t nv, int d, const double *__restrict__ X,
                                               double *__restrict__ part) {
  __shared__ double smin[3][TB], smax[3][TB];
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t v = blockIdx.x * (int64_t)TB + threadIdx.x; v < nv; v += (int64_t)gridDim.x * TB)
    for (int q = 0; q < d; ++q) {
      const double x = X[v * d + q];
      lo[q] = fmin(lo[q], x);
      hi[q] = fmax(hi[q], x);
    }
  for (int q = 0; q < 3; ++q) {
    smin[q][threadIdx.x] = lo[q];
    smax[q][threadIdx.x] = hi[q];
  }
  __syncthreads();
  for (int s = TB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int q = 0; q < 3; ++q) {
        smin[q][threadIdx.x] = fmin(smin[q][threadIdx.x], smin[q][threadIdx.x + s]);
        smax[q][threadIdx.x] = fmax(smax[q][threadIdx.x], smax[q][threadIdx.x + s]);
      }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int q = 0; q < 3; ++q) {
      part[blockIdx.x * 6 + q] = smin[q][0];
      part[blockIdx.x * 6 + 3 + q] = smax[q][0];
    }
}

// barycenter (((p0 + p1) + p2) [+ p3]) / (d+1) per axis, key floor((xi - a) / L * 2^D) clamped to
// [0, 2^D - 1], and the level-(D+1) code of the element
__global__ __launch_bounds__(TB) void k_keys(int64_t ne, int d, int D, const double *__restrict__ X,
                                             const int *__restrict__ E, double a0, double a1, double a2, double L,
                                             int64_t *__restrict__ keys, uint64_t *__restrict__ code,
                                             int *__restrict__ eid) {
  const int64_t e = blockIdx.x * (int64_t)TB + threadIdx.x;
  if (e >= ne) return;
  const int k = d + 1;
  const double a[3] = {a0, a1, a2};
  const double scale = ldexp(1.0, D);
  const int64_t kmax = ((int64_t)1 << D) - 1;
  int64_t kk[3] = {0, 0, 0};
  for (int q = 0; q < d; ++q) {
    double s = __dadd_rn(X[(int64_t)E[e * k] * d + q], X[(int64_t)E[e * k + 1] * d + q]);
    for (int m = 2; m < k; ++m) s = __dadd_rn(s, X[(int64_t)E[e * k + m] * d + q]);
    const double xi = __ddiv_rn(s, (double)k);
    const double t = __ddiv_rn(__dsub_rn(xi, a[q]), L);
    const double f = floor(__dmul_rn(t, scale));
    int64_t ki = f < 0 ? 0 : (int64_t)f;
    if (ki > kmax) ki = kmax;
    kk[q] = ki;
    keys[e * d + q] = ki;
  }
  code[e] = d_code(D + 1, kk, d);
  eid[e] = (int)e;
}

// boxes of one level (prefix = code >> shift) holding more than n_min barycenters
__global__ __launch_bounds__(TB) void k_r0(int64_t ne, const uint64_t *__restrict__ code, int shift, int n_min,
                                           uint64_t *__restrict__ out, unsigned long long *__restrict__ cnt) {
  const int64_t i = blockIdx.x * (int64_t)TB + threadIdx.x;
  if (i >= ne) return;
  const uint64_t p = code[i] >> shift;
  if (i > 0 && (code[i - 1] >> shift) == p) return;  // not the first of its run
  if (i + n_min < ne && (code[i + n_min] >> shift) == p) out[atomicAdd(cnt, 1ull)] = p;
}

// closure candidates: for a refined box b of level >= 2 and every same-level box q sharing a
// facet (3-D: or an edge) with b, parent(q) if it is not refined yet
__global__ __launch_bounds__(TB) void k_close(int64_t nf, const uint64_t *__restrict__ frontier,
                                              const uint64_t *__restrict__ R, int64_t nR, int d,
                                              uint64_t *__restrict__ cand, unsigned long long *__restrict__ cnt) {
  const int64_t i = blockIdx.x * (int64_t)TB + threadIdx.x;
  if (i >= nf) return;
  const uint64_t b = frontier[i];
  const int lev = d_level(b, d);
  if (lev < 2) return;
  int64_t idx[3] = {0, 0, 0};
  d_index(b, d, idx);
  const int64_t n = (int64_t)1 << (lev - 1);
  for (int x = -1; x <= 1; ++x)
    for (int y = -1; y <= 1; ++y)
      for (int z = (d == 3 ? -1 : 0); z <= (d == 3 ? 1 : 0); ++z) {
        const int nz = (x != 0) + (y != 0) + (z != 0);
        if (!(nz == 1 || (d == 3 && nz == 2))) continue;
        const int o[3] = {x, y, z};
        int64_t q[3];
        bool ok = true;
        for (int k = 0; k < d; ++k) {
          q[k] = idx[k] + o[k];
          if (q[k] < 0 || q[k] >= n) ok = false;
        }
        if (!ok) continue;
        for (int k = 0; k < d; ++k) q[k] >>= 1;
        const uint64_t p = d_code(lev - 1, q, d);
        if (!d_member(R, nR, p)) cand[atomicAdd(cnt, 1ull)] = p;
      }
}

// children of refined boxes that are not refined
__global__ __launch_bounds__(TB) void k_leaves(int64_t nR, const uint64_t *__restrict__ R, int d,
                                               uint64_t *__restrict__ out, unsigned long long *__restrict__ cnt) {
  const int64_t i = blockIdx.x * (int64_t)TB + threadIdx.x;
  if (i >= nR) return;
  const uint64_t b = R[i];
  for (int ci = 0; ci < (1 << d); ++ci) {
    const uint64_t c = (b << d) | (uint64_t)ci;
    if (!d_member(R, nR, c)) out[atomicAdd(cnt, 1ull)] = c;
  }
}

// sort keys of the host's leaf order (level, i_0, .., i_{d-1}): the index tuple packed in 60 bits
// (first pass) and the level (second, stable pass)
__global__ __launch_bounds__(TB) void k_tuple_keys(int64_t n, const uint64_t *__restrict__ c, int d,
                                                   uint64_t *__restrict__ tk, uint64_t *__restrict__ lk) {
  const int64_t i = blockIdx.x * (int64_t)TB + threadIdx.x;
  if (i >= n) return;
  int64_t idx[3] = {0, 0, 0};
  d_index(c[i], d, idx);
  const int w = 60 / d;
  uint64_t t = 0;
  for (int k = 0; k < d; ++k) t = (t << w) | (uint64_t)idx[k];
  tk[i] = t;
  lk[i] = (uint64_t)d_level(c[i], d);
}

__global__ __launch_bounds__(TB) void k_gather_kappa(int64_t ne, const int *__restrict__ eid,
                                                     const double *__restrict__ kappa, double *__restrict__ ks) {
  const int64_t i = blockIdx.x * (int64_t)TB + threadIdx.x;
  if (i < ne) ks[i] = kappa[eid[i]];
}

// kappa~ of a leaf: mean over its cluster (sorted order), or over the nearest non-empty ancestor's
__global__ __launch_bounds__(TB) void k_leaf_kappa(int64_t nl, const uint64_t *__restrict__ leaves,
                                                   const uint64_t *__restrict__ code, const double *__restrict__ ks,
                                                   int64_t ne, int d, int D, double *__restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)TB + threadIdx.x;
  if (i >= nl) return;
  uint64_t q = leaves[i];
  while (true) {
    const int sh = d * (D + 1 - d_level(q, d));
    const int64_t s = d_lower(code, ne, q << sh), e = d_lower(code, ne, (q + 1) << sh);
    if (e > s) {
      double sum = 0;
      for (int64_t j = s; j < e; ++j) sum += ks[j];
      out[i] = sum / (double)(e - s);
      return;
    }
    q >>= d;
  }
}

// device buffers of one build, freed on every exit path
struct Bufs {
  std::vector<void *> p;
  template <class T>
  T *get(int64_t n) {
    void *q = nullptr;
    HIPCHECK(hipMalloc(&q, (size_t)std::max<int64_t>(n, 1) * sizeof(T)));
    p.push_back(q);
    return (T *)q;
  }
  ~Bufs() {
    for (void *q : p) (void)hipFree(q);
  }
};

inline int grid(int64_t n) { return (int)std::max<int64_t>(1, (n + TB - 1) / TB); }

// sort keys (and optional values) of length n in place through the out buffers
void sort_keys(Bufs &B, uint64_t *&k, int64_t n, int end_bit, hipStream_t s) {
  if (n <= 1) return;
  uint64_t *ko = B.get<uint64_t>(n);
  size_t tb = 0;
  HIPCHECK(hipcub::DeviceRadixSort::SortKeys(nullptr, tb, k, ko, (int)n, 0, end_bit, s));
  void *tmp = B.get<char>((int64_t)tb);
  HIPCHECK(hipcub::DeviceRadixSort::SortKeys(tmp, tb, k, ko, (int)n, 0, end_bit, s));
  k = ko;
}

// sort and deduplicate; returns the unique count
int64_t sort_unique(Bufs &B, uint64_t *&k, int64_t n, int end_bit, hipStream_t s) {
  if (n == 0) return 0;
  sort_keys(B, k, n, end_bit, s);
  uint64_t *u = B.get<uint64_t>(n);
  int *nsel = B.get<int>(1);
  size_t tb = 0;
  HIPCHECK(hipcub::DeviceSelect::Unique(nullptr, tb, k, u, nsel, (int)n, s));
  void *tmp = B.get<char>((int64_t)tb);
  HIPCHECK(hipcub::DeviceSelect::Unique(tmp, tb, k, u, nsel, (int)n, s));
  int h = 0;
  HIPCHECK(hipMemcpyAsync(&h, nsel, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  k = u;
  return h;
}

uint64_t read_count(unsigned long long *cnt, hipStream_t s) {
  unsigned long long h = 0;
  HIPCHECK(hipMemcpyAsync(&h, cnt, sizeof(h), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  return h;
}

}  // namespace

void build_tree_device(Hierarchy &h, int ordinal) {
  const int d = h.d, D = d == 2 ? 30 : 20, k = d + 1;
  const int n_min = h.opt.n_min > 0 ? h.opt.n_min : (d == 2 ? 3 : 7);
  const int64_t nv = h.nv, ne = h.ne;
  if (ne >= ((int64_t)1 << 31)) throw AsmgError{ASMG_EINVAL, "too many elements for the device tree build"};
  HIPCHECK(hipSetDevice(ordinal));
  Bufs B;  // destroyed after the stream guard: the stream has drained before anything is freed
  hipStream_t s;
  HIPCHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  struct StreamGuard {
    hipStream_t s;
    ~StreamGuard() {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
  } sg{s};
  const int end_bit = d * D + 1;  // marker bit of a level-(D+1) code

  // root box
  double *X = B.get<double>(nv * d);
  HIPCHECK(hipMemcpyAsync(X, h.coords.data(), (size_t)nv * d * 8, hipMemcpyHostToDevice, s));
  const int ge = std::min(grid(nv), 1024);
  double *part = B.get<double>((int64_t)ge * 6);
  hipLaunchKernelGGL(k_extent, dim3(ge), dim3(TB), 0, s, nv, d, (const double *)X, part);
  std::vector<double> hp((size_t)ge * 6);
  HIPCHECK(hipMemcpyAsync(hp.data(), part, hp.size() * 8, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int b = 0; b < ge; ++b)
    for (int q = 0; q < d; ++q) {
      lo[q] = std::min(lo[q], hp[b * 6 + q]);
      hi[q] = std::max(hi[q], hp[b * 6 + 3 + q]);
    }
  h.L = 0;
  for (int q = 0; q < 3; ++q) h.a[q] = 0;
  for (int q = 0; q < d; ++q) {
    h.a[q] = lo[q];
    h.L = std::max(h.L, hi[q] - lo[q]);
  }
  if (!(h.L > 0)) throw AsmgError{ASMG_EINVAL, "mesh has zero extent"};

  // keys and the sorted element codes
  int *E = B.get<int>(ne * k);
  HIPCHECK(hipMemcpyAsync(E, h.elems.data(), (size_t)ne * k * 4, hipMemcpyHostToDevice, s));
  int64_t *keys = B.get<int64_t>(ne * d);
  uint64_t *code = B.get<uint64_t>(ne);
  int *eid = B.get<int>(ne);
  hipLaunchKernelGGL(k_keys, dim3(grid(ne)), dim3(TB), 0, s, ne, d, D, (const double *)X, (const int *)E, h.a[0],
                     h.a[1], h.a[2], h.L, keys, code, eid);
  uint64_t *code_s = B.get<uint64_t>(ne);
  int *eid_s = B.get<int>(ne);
  {
    size_t tb = 0;
    HIPCHECK(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, code, code_s, eid, eid_s, (int)ne, 0, end_bit, s));
    void *tmp = B.get<char>((int64_t)tb);
    HIPCHECK(hipcub::DeviceRadixSort::SortPairs(tmp, tb, code, code_s, eid, eid_s, (int)ne, 0, end_bit, s));
  }
  h.keys.resize((size_t)ne * d);
  HIPCHECK(hipMemcpyAsync(h.keys.data(), keys, (size_t)ne * d * 8, hipMemcpyDeviceToHost, s));

  // R0: level by level until a level has no refined box
  unsigned long long *cnt = B.get<unsigned long long>(1);
  const int64_t cap0 = (int64_t)D * (ne / (n_min + 1)) + 1;
  uint64_t *r0 = B.get<uint64_t>(cap0);
  HIPCHECK(hipMemsetAsync(cnt, 0, sizeof(unsigned long long), s));
  uint64_t nr0 = 0;
  for (int lev = 1; lev <= D; ++lev) {
    hipLaunchKernelGGL(k_r0, dim3(grid(ne)), dim3(TB), 0, s, ne, (const uint64_t *)code_s, d * (D + 1 - lev), n_min,
                       r0, cnt);
    const uint64_t c = read_count(cnt, s);
    if (c == nr0) break;
    nr0 = c;
  }
  int64_t nR = sort_unique(B, r0, (int64_t)nr0, end_bit, s);
  std::vector<uint64_t> hR0((size_t)nR);
  if (nR) HIPCHECK(hipMemcpyAsync(hR0.data(), r0, (size_t)nR * 8, hipMemcpyDeviceToHost, s));

  // closure rounds
  uint64_t *R = r0;
  uint64_t *front = r0;
  int64_t nfront = nR;
  const int noffs = d == 2 ? 4 : 18;
  while (nfront > 0) {
    uint64_t *cand = B.get<uint64_t>(nfront * noffs);
    HIPCHECK(hipMemsetAsync(cnt, 0, sizeof(unsigned long long), s));
    hipLaunchKernelGGL(k_close, dim3(grid(nfront)), dim3(TB), 0, s, nfront, (const uint64_t *)front,
                       (const uint64_t *)R, nR, d, cand, cnt);
    const int64_t nc = (int64_t)read_count(cnt, s);
    const int64_t nnew = sort_unique(B, cand, nc, end_bit, s);
    if (nnew == 0) break;
    uint64_t *merged = B.get<uint64_t>(nR + nnew);
    HIPCHECK(hipMemcpyAsync(merged, R, (size_t)nR * 8, hipMemcpyDeviceToDevice, s));
    HIPCHECK(hipMemcpyAsync(merged + nR, cand, (size_t)nnew * 8, hipMemcpyDeviceToDevice, s));
    nR += nnew;
    sort_keys(B, merged, nR, end_bit, s);
    R = merged;
    front = cand;
    nfront = nnew;
  }

  // leaves
  std::vector<uint64_t> hleaves;
  int64_t nl = 1;
  uint64_t *leaves = B.get<uint64_t>(nR * (1 << d) + 1);
  const uint64_t root = 1;
  if (nR == 0) {
    HIPCHECK(hipMemcpyAsync(leaves, &root, 8, hipMemcpyHostToDevice, s));
  } else {
    HIPCHECK(hipMemsetAsync(cnt, 0, sizeof(unsigned long long), s));
    hipLaunchKernelGGL(k_leaves, dim3(grid(nR)), dim3(TB), 0, s, nR, (const uint64_t *)R, d, leaves, cnt);
    nl = (int64_t)read_count(cnt, s);
    // (level, index tuple) order: stable sort by the tuple, then by the level
    uint64_t *tk = B.get<uint64_t>(nl), *lk = B.get<uint64_t>(nl);
    hipLaunchKernelGGL(k_tuple_keys, dim3(grid(nl)), dim3(TB), 0, s, nl, (const uint64_t *)leaves, d, tk, lk);
    uint64_t *tk2 = B.get<uint64_t>(nl), *l2 = B.get<uint64_t>(nl);
    size_t tb = 0;
    HIPCHECK(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, tk, tk2, leaves, l2, (int)nl, 0, 60, s));
    void *tmp = B.get<char>((int64_t)tb);
    HIPCHECK(hipcub::DeviceRadixSort::SortPairs(tmp, tb, tk, tk2, leaves, l2, (int)nl, 0, 60, s));
    hipLaunchKernelGGL(k_tuple_keys, dim3(grid(nl)), dim3(TB), 0, s, nl, (const uint64_t *)l2, d, tk, lk);
    uint64_t *lk2 = B.get<uint64_t>(nl), *l3 = B.get<uint64_t>(nl);
    tb = 0;
    HIPCHECK(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, lk, lk2, l2, l3, (int)nl, 0, 6, s));
    void *tmp2 = B.get<char>((int64_t)tb);
    HIPCHECK(hipcub::DeviceRadixSort::SortPairs(tmp2, tb, lk, lk2, l2, l3, (int)nl, 0, 6, s));
    leaves = l3;
  }
  // kappa~
  double *kap = B.get<double>(ne);
  HIPCHECK(hipMemcpyAsync(kap, h.kappa.data(), (size_t)ne * 8, hipMemcpyHostToDevice, s));
  double *ks = B.get<double>(ne);
  hipLaunchKernelGGL(k_gather_kappa, dim3(grid(ne)), dim3(TB), 0, s, ne, (const int *)eid_s, (const double *)kap, ks);
  double *lk = B.get<double>(nl);
  hipLaunchKernelGGL(k_leaf_kappa, dim3(grid(nl)), dim3(TB), 0, s, nl, (const uint64_t *)leaves,
                     (const uint64_t *)code_s, (const double *)ks, ne, d, D, lk);
  HIPCHECK(hipGetLastError());

  std::vector<uint64_t> hR((size_t)nR);
  hleaves.resize((size_t)nl);
  std::vector<double> hlk((size_t)nl);
  if (nR) HIPCHECK(hipMemcpyAsync(hR.data(), R, (size_t)nR * 8, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipMemcpyAsync(hleaves.data(), leaves, (size_t)nl * 8, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipMemcpyAsync(hlk.data(), lk, (size_t)nl * 8, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));

  h.R0.clear();
  h.R0.reserve(hR0.size());
  h.R0.insert(hR0.begin(), hR0.end());
  h.R.clear();
  h.R.reserve(hR.size());
  h.R.insert(hR.begin(), hR.end());
  h.leaf_kappa.clear();
  h.leaf_kappa.reserve((size_t)nl);
  for (int64_t i = 0; i < nl; ++i) h.leaf_kappa.emplace(hleaves[i], hlk[i]);
  h.leaves = std::move(hleaves);  // already in the host order: (level, index tuple)
  h.J = 1;
  for (BoxCode b : h.leaves) h.J = std::max(h.J, box_level(b, d));
  if (h.J > 31 || (d == 3 && h.J > 21)) throw AsmgError{ASMG_EINVAL, "tree too deep"};
}

}  // namespace asmg
