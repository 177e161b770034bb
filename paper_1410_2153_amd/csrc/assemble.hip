// Fine-grid matrix assembled on the device (Section 2): A = sum_e kappa_e |tau_e| G_e G_e^T over
// the unknowns (non-Dirichlet vertices), P1 elements in 2-D and 3-D.
//
// The result is bit-identical to the host assembly (assemble_fine_values in setup.cpp):
//   - every product, sum, quotient of the element gradients, the volume and the weight is an
//     explicitly rounded IEEE operation in the host's order (the host compiles this code
//     without contraction);
//   - an entry's contributions are summed from 0 in element order: contributions are generated
//     element-major, sorted by (row, column) with a stable radix sort, and each run of equal
//     keys is summed sequentially;
//   - the pattern is the sorted, deduplicated (row, column) keys, as the host's per-row sort.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
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
constexpr uint64_t NONE = ~(uint64_t)0;  // key of a contribution that touches a Dirichlet vertex

// gradients of the barycentric coordinates (G[a][r] = d lambda_a / d x_r) and |det| of one element,
// with the host's operations and rounding
__device__ double d_element_grads(int d, const double *__restrict__ X, const int *ev, double G[4][3]) {
  double M[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // columns = edges p_k - p_0
  const double *p0 = X + (int64_t)ev[0] * d;
  for (int k = 0; k < d; ++k) {
    const double *pk = X + (int64_t)ev[k + 1] * d;
    for (int r = 0; r < d; ++r) M[r][k] = __dsub_rn(pk[r], p0[r]);
  }
  double det, inv[3][3];
  if (d == 2) {
    det = __dsub_rn(__dmul_rn(M[0][0], M[1][1]), __dmul_rn(M[0][1], M[1][0]));
    inv[0][0] = __ddiv_rn(M[1][1], det);
    inv[0][1] = __ddiv_rn(-M[0][1], det);
    inv[1][0] = __ddiv_rn(-M[1][0], det);
    inv[1][1] = __ddiv_rn(M[0][0], det);
  } else {
    double c[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const int r0 = (j + 1) % 3, r1 = (j + 2) % 3, c0 = (i + 1) % 3, c1 = (i + 2) % 3;
        c[i][j] = __dsub_rn(__dmul_rn(M[r0][c0], M[r1][c1]), __dmul_rn(M[r0][c1], M[r1][c0]));
      }
    det = __dadd_rn(__dadd_rn(__dmul_rn(M[0][0], c[0][0]), __dmul_rn(M[0][1], c[1][0])), __dmul_rn(M[0][2], c[2][0]));
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) inv[i][j] = __ddiv_rn(c[i][j], det);
  }
  for (int k = 0; k < d; ++k)
    for (int r = 0; r < d; ++r) G[k + 1][r] = inv[k][r];
  for (int r = 0; r < d; ++r) {
    double s = 0;
    for (int k = 0; k < d; ++k) s = __dadd_rn(s, inv[k][r]);
    G[0][r] = -s;
  }
  return fabs(det);
}

// (row, column) key and value of every local pair of every element, element-major; flags a
// degenerate element
__global__ __launch_bounds__(TB) void k_contrib(int64_t ne, int d, const double *__restrict__ X,
                                                const int *__restrict__ E, const double *__restrict__ kappa,
                                                const int *__restrict__ dofv, uint64_t *__restrict__ key,
                                                double *__restrict__ val, int *__restrict__ bad) {
  const int64_t e = blockIdx.x * (int64_t)TB + threadIdx.x;
  if (e >= ne) return;
  const int k = d + 1;
  int ev[4];
  for (int a = 0; a < k; ++a) ev[a] = E[e * k + a];
  double G[4][3];
  const double adet = d_element_grads(d, X, ev, G);
  const double det_ok = adet;  // |det| of a valid element is finite and non-zero
  if (!(det_ok != 0.0) || !isfinite(det_ok)) atomicMin(bad, (int)e);
  const double vol = __ddiv_rn(adet, d == 2 ? 2.0 : 6.0);
  const double w = __dmul_rn(kappa[e], vol);
  for (int i = 0; i < k; ++i) {
    const int ui = dofv[ev[i]];
    for (int j = 0; j < k; ++j) {
      const int uj = dofv[ev[j]];
      const int64_t slot = e * k * k + i * k + j;
      if (ui < 0 || uj < 0) {
        key[slot] = NONE;
        val[slot] = 0.0;
        continue;
      }
      double g = 0;
      for (int r = 0; r < d; ++r) g = __dadd_rn(g, __dmul_rn(G[i][r], G[j][r]));
      key[slot] = ((uint64_t)(uint32_t)ui << 32) | (uint32_t)uj;
      val[slot] = __dmul_rn(w, g);
    }
  }
}

// first position of each run of equal keys (NONE excluded)
__global__ __launch_bounds__(TB) void k_heads(int64_t m, const uint64_t *__restrict__ key, int *__restrict__ head) {
  const int64_t i = blockIdx.x * (int64_t)TB + threadIdx.x;
  if (i >= m) return;
  head[i] = key[i] != NONE && (i == 0 || key[i] != key[i - 1]) ? 1 : 0;
}

// entry p (the run starting at i): column, value summed in order, and the row's entry count
__global__ __launch_bounds__(TB) void k_entries(int64_t m, const uint64_t *__restrict__ key,
                                                const double *__restrict__ val, const int *__restrict__ head,
                                                const int *__restrict__ pos, int *__restrict__ ci,
                                                double *__restrict__ v, int *__restrict__ rowcnt) {
  const int64_t i = blockIdx.x * (int64_t)TB + threadIdx.x;
  if (i >= m || !head[i]) return;
  const uint64_t kk = key[i];
  double s = 0.0;
  for (int64_t j = i; j < m && key[j] == kk; ++j) s = __dadd_rn(s, val[j]);
  const int p = pos[i];
  ci[p] = (int)(kk & 0xffffffffu);
  v[p] = s;
  atomicAdd(&rowcnt[(int)(kk >> 32)], 1);
}

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

}  // namespace

void build_fine_device(Hierarchy &h, int ordinal) {
  const int d = h.d, k = d + 1;
  fine_dofs(h);
  const int64_t n = h.n(), ne = h.ne, nv = h.nv, m = ne * k * k;
  if (m >= ((int64_t)1 << 31) || n >= ((int64_t)1 << 31))
    throw AsmgError{ASMG_EINVAL, "mesh too large for the device assembly"};
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

  double *X = B.get<double>(nv * d);
  HIPCHECK(hipMemcpyAsync(X, h.coords.data(), (size_t)nv * d * 8, hipMemcpyHostToDevice, s));
  int *E = B.get<int>(ne * k);
  HIPCHECK(hipMemcpyAsync(E, h.elems.data(), (size_t)ne * k * 4, hipMemcpyHostToDevice, s));
  double *kap = B.get<double>(ne);
  HIPCHECK(hipMemcpyAsync(kap, h.kappa.data(), (size_t)ne * 8, hipMemcpyHostToDevice, s));
  std::vector<int> dofv(h.dof_of_vertex.begin(), h.dof_of_vertex.end());
  int *DV = B.get<int>(nv);
  HIPCHECK(hipMemcpyAsync(DV, dofv.data(), (size_t)nv * 4, hipMemcpyHostToDevice, s));
  int *bad = B.get<int>(1);
  const int big = INT32_MAX;
  HIPCHECK(hipMemcpyAsync(bad, &big, 4, hipMemcpyHostToDevice, s));

  uint64_t *key = B.get<uint64_t>(m), *key_s = B.get<uint64_t>(m);
  double *val = B.get<double>(m), *val_s = B.get<double>(m);
  hipLaunchKernelGGL(k_contrib, dim3(grid(ne)), dim3(TB), 0, s, ne, d, (const double *)X, (const int *)E,
                     (const double *)kap, (const int *)DV, key, val, bad);
  {
    size_t tb = 0;
    HIPCHECK(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, key, key_s, val, val_s, (int)m, 0, 64, s));
    void *tmp = B.get<char>((int64_t)tb);
    HIPCHECK(hipcub::DeviceRadixSort::SortPairs(tmp, tb, key, key_s, val, val_s, (int)m, 0, 64, s));
  }
  int *head = B.get<int>(m), *pos = B.get<int>(m);
  hipLaunchKernelGGL(k_heads, dim3(grid(m)), dim3(TB), 0, s, m, (const uint64_t *)key_s, head);
  {
    size_t tb = 0;
    HIPCHECK(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, head, pos, (int)m, s));
    void *tmp = B.get<char>((int64_t)tb);
    HIPCHECK(hipcub::DeviceScan::ExclusiveSum(tmp, tb, head, pos, (int)m, s));
  }
  int last_pos = 0, last_head = 0, hbad = 0;
  HIPCHECK(hipMemcpyAsync(&last_pos, pos + (m - 1), 4, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipMemcpyAsync(&last_head, head + (m - 1), 4, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  if (hbad != INT32_MAX) throw AsmgError{ASMG_EINVAL, "degenerate element " + std::to_string(hbad)};
  const int64_t nnz = (int64_t)last_pos + last_head;
  int *ci = B.get<int>(nnz);
  double *v = B.get<double>(nnz);
  int *rowcnt = B.get<int>(n);
  HIPCHECK(hipMemsetAsync(rowcnt, 0, (size_t)std::max<int64_t>(n, 1) * 4, s));
  hipLaunchKernelGGL(k_entries, dim3(grid(m)), dim3(TB), 0, s, m, (const uint64_t *)key_s, (const double *)val_s,
                     (const int *)head, (const int *)pos, ci, v, rowcnt);
  HIPCHECK(hipGetLastError());

  Csr &A = h.A;
  A.nrows = A.ncols = n;
  A.ci.resize((size_t)nnz);
  A.v.resize((size_t)nnz);
  std::vector<int> cnt((size_t)n);
  if (nnz) {
    HIPCHECK(hipMemcpyAsync(A.ci.data(), ci, (size_t)nnz * 4, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipMemcpyAsync(A.v.data(), v, (size_t)nnz * 8, hipMemcpyDeviceToHost, s));
  }
  if (n) HIPCHECK(hipMemcpyAsync(cnt.data(), rowcnt, (size_t)n * 4, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  A.rp.assign((size_t)n + 1, 0);
  for (int64_t i = 0; i < n; ++i) A.rp[i + 1] = A.rp[i] + cnt[i];
  if (A.rp[n] != nnz) throw AsmgError{ASMG_EDEVICE, "device assembly: row counts do not add up"};
}

}  // namespace asmg
