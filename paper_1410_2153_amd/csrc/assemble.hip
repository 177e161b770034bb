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

// (row, column) key and value of every local pair of every simplex of a level mesh sigma^(l),
// simplex-major, as assemble_level computes them on the host: integer cofactors of the simplex
// in units of half its box side, the Kuhn coefficient of its box (the first one on fan boxes),
// value = dot / (d! |det|) (times half * unit in 3-D) times kappa~
// Kuhn coefficients of each active box: binary search of its code in the sorted table of all
// boxes' codes (wcode, 6 coefficients per box in wtab)
__global__ __launch_bounds__(TB) void k_box_weights(int64_t nb, const uint64_t *__restrict__ code,
                                                    const uint64_t *__restrict__ wcode, int64_t nw,
                                                    const double *__restrict__ wtab, double *__restrict__ bw,
                                                    int *__restrict__ missing) {
  const int64_t b = blockIdx.x * (int64_t)TB + threadIdx.x;
  if (b >= nb) return;
  const uint64_t c = code[b];
  int64_t lo = 0, hi = nw;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (wcode[mid] < c)
      lo = mid + 1;
    else
      hi = mid;
  }
  if (lo >= nw || wcode[lo] != c) {
    atomicAdd(missing, 1);
    return;
  }
  for (int q = 0; q < 6; ++q) bw[b * 6 + q] = wtab[lo * 6 + q];
}

__global__ __launch_bounds__(TB) void k_level_contrib(int64_t ns, int d, int J, double unit,
                                                      const int64_t *__restrict__ verts, const int64_t *__restrict__ simp,
                                                      const int *__restrict__ sbox, const int8_t *__restrict__ stmpl,
                                                      const uint64_t *__restrict__ bcode, const uint8_t *__restrict__ bfan,
                                                      const double *__restrict__ bw, const uint8_t *__restrict__ kept,
                                                      const int64_t *__restrict__ dofv, uint64_t *__restrict__ key,
                                                      double *__restrict__ val) {
  const int64_t s = blockIdx.x * (int64_t)TB + threadIdx.x;
  if (s >= ns) return;
  const int k = d + 1;
  int u[4];
  const bool in = kept == nullptr || kept[s];
  for (int i = 0; i < k; ++i) u[i] = in ? (int)dofv[simp[s * k + i]] : -1;
  bool any = false;
  for (int i = 0; i < k; ++i) any |= u[i] >= 0;
  if (!any) {
    for (int q = 0; q < k * k; ++q) {
      key[s * k * k + q] = NONE;
      val[s * k * k + q] = 0.0;
    }
    return;
  }
  const int b = sbox[s];
  const int blev = (63 - __clzll((long long)bcode[b])) / d + 1;  // level of the box's code
  const int64_t half = (int64_t)1 << (J - blev);
  const int64_t *v0 = verts + (int64_t)simp[s * k] * d;
  int64_t M[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int c = 0; c < d; ++c) {
    const int64_t *vc = verts + (int64_t)simp[s * k + c + 1] * d;
    for (int r = 0; r < d; ++r) M[r][c] = (vc[r] - v0[r]) / half;
  }
  int64_t a[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  int64_t det;
  if (d == 2) {
    det = M[0][0] * M[1][1] - M[0][1] * M[1][0];
    a[1][0] = M[1][1];
    a[1][1] = -M[0][1];
    a[2][0] = -M[1][0];
    a[2][1] = M[0][0];
  } else {
    det = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
          M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const int r0 = (j + 1) % 3, r1 = (j + 2) % 3, c0 = (i + 1) % 3, c1 = (i + 2) % 3;
        a[i + 1][j] = M[r0][c0] * M[r1][c1] - M[r0][c1] * M[r1][c0];
      }
  }
  for (int r = 0; r < d; ++r) {
    int64_t sum = 0;
    for (int c = 1; c <= d; ++c) sum += a[c][r];
    a[0][r] = -sum;
  }
  const double denom = __dmul_rn(d == 2 ? 2.0 : 6.0, (double)(det < 0 ? -det : det));
  const double kap = bfan[b] ? bw[(int64_t)b * 6] : bw[(int64_t)b * 6 + stmpl[s]];
  const double hu = __dmul_rn((double)half, unit);
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) {
      const int64_t slot = s * k * k + i * k + j;
      if (u[i] < 0 || u[j] < 0) {
        key[slot] = NONE;
        val[slot] = 0.0;
        continue;
      }
      int64_t dot = 0;
      for (int r = 0; r < d; ++r) dot += a[i][r] * a[j][r];
      double v = __ddiv_rn((double)dot, denom);
      if (d == 3) v = __dmul_rn(v, hu);
      v = __dmul_rn(v, kap);
      key[slot] = ((uint64_t)(uint32_t)u[i] << 32) | (uint32_t)u[j];
      val[slot] = v;
    }
}

// box code of level `level` with index tuple idx (the host's box_code: marker bit above the
// interleaved index bits, axis 0 most significant in each bit group)
__device__ __forceinline__ uint64_t d_box_code(int level, const int64_t *idx, int d) {
  uint64_t m = 0;
  const int bits = level - 1;
  for (int b = 0; b < bits; ++b)
    for (int q = 0; q < d; ++q) m |= (uint64_t)((idx[q] >> b) & 1) << (b * d + (d - 1 - q));
  return m | ((uint64_t)1 << (d * bits));
}

// determinant of the edge vectors P[1..d] - P[0] (integer; the caller bounds the coordinates so
// that no intermediate leaves int64)
__device__ __forceinline__ int64_t d_det(int d, const int64_t *const P[4]) {
  int64_t E[3][3];
  for (int c = 0; c < d; ++c)
    for (int r = 0; r < d; ++r) E[r][c] = P[c + 1][r] - P[0][r];
  if (d == 2) return E[0][0] * E[1][1] - E[0][1] * E[1][0];
  return E[0][0] * (E[1][1] * E[2][2] - E[1][2] * E[2][1]) - E[0][1] * (E[1][0] * E[2][2] - E[1][2] * E[2][0]) +
         E[0][2] * (E[1][0] * E[2][1] - E[1][1] * E[2][0]);
}

// row i of P_l (nodal interpolation of level l-1's functions at level l's unknown i): the
// smallest active box of level l-1 holding the vertex, the first of its simplices that contains
// it (exact barycentric coordinates), the nonzero coordinates at level l-1's unknowns, sorted by
// (column, value) as the host does; `bad` gets the row if the point location fails
__global__ __launch_bounds__(TB) void k_iota(int64_t n, int *__restrict__ x) {
  const int64_t i = blockIdx.x * (int64_t)TB + threadIdx.x;
  if (i < n) x[i] = (int)i;
}

__global__ __launch_bounds__(TB) void k_prolong(int n, int d, int J, int level, const int64_t *__restrict__ fverts,
                                                const int64_t *__restrict__ fdof, const int64_t *__restrict__ cverts,
                                                const int64_t *__restrict__ csimp, const uint64_t *__restrict__ ccode,
                                                const int *__restrict__ cidx, int ncb,
                                                const int64_t *__restrict__ cbox_simp, const int64_t *__restrict__ cdofv,
                                                int *__restrict__ pcol, double *__restrict__ pval,
                                                int *__restrict__ pcnt, int *__restrict__ bad) {
  const int i = blockIdx.x * TB + threadIdx.x;
  if (i >= n) return;
  const int k1 = d + 1;
  const int64_t *X = fverts + fdof[i] * d;
  int bi = -1;
  for (int k = 1; k <= level - 1 && bi < 0; ++k) {
    int64_t idx[3];
    const int sh = J - k + 1;
    const int64_t nmax = ((int64_t)1 << (k - 1)) - 1;
    for (int q = 0; q < d; ++q) idx[q] = min(X[q] >> sh, nmax);
    const uint64_t code = d_box_code(k, idx, d);
    int lo = 0, hi = ncb;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (ccode[mid] < code)
        lo = mid + 1;
      else
        hi = mid;
    }
    if (lo < ncb && ccode[lo] == code) bi = cidx[lo];
  }
  pcnt[i] = 0;
  if (bi < 0) {
    atomicMin(bad, i);
    return;
  }
  int64_t sfound = -1;
  int64_t num[4] = {0, 0, 0, 0}, tot = 0;
  for (int64_t sx = cbox_simp[bi]; sx < cbox_simp[bi + 1] && sfound < 0; ++sx) {
    const int64_t *V[4];
    for (int m = 0; m < k1; ++m) V[m] = cverts + (int64_t)csimp[sx * k1 + m] * d;
    int64_t t = d_det(d, V);
    bool inside = true;
    for (int m = 0; m < k1 && inside; ++m) {
      const int64_t *Q[4];
      for (int r = 0; r < k1; ++r) Q[r] = r == m ? X : V[r];
      int64_t nm = d_det(d, Q);
      if (t < 0) nm = -nm;
      if (nm < 0) inside = false;
      num[m] = nm;
    }
    if (inside) {
      sfound = sx;
      tot = t < 0 ? -t : t;
    }
  }
  if (sfound < 0) {
    atomicMin(bad, i);
    return;
  }
  int cols[4];
  double vals[4];
  int c = 0;
  for (int m = 0; m < k1; ++m) {
    const double lam = __ddiv_rn((double)num[m], (double)tot);
    if (lam == 0.0) continue;
    const int j = (int)cdofv[csimp[sfound * k1 + m]];
    if (j < 0) continue;
    // insertion by (column, value)
    int q = c++;
    while (q > 0 && (cols[q - 1] > j || (cols[q - 1] == j && vals[q - 1] > lam))) {
      cols[q] = cols[q - 1];
      vals[q] = vals[q - 1];
      --q;
    }
    cols[q] = j;
    vals[q] = lam;
  }
  // merge equal columns in that order
  int w = 0;
  for (int q = 0; q < c; ++q) {
    if (w > 0 && cols[w - 1] == cols[q]) {
      vals[w - 1] = __dadd_rn(vals[w - 1], vals[q]);
    } else {
      cols[w] = cols[q];
      vals[w] = vals[q];
      ++w;
    }
  }
  for (int q = 0; q < w; ++q) {
    pcol[(int64_t)i * k1 + q] = cols[q];
    pval[(int64_t)i * k1 + q] = vals[q];
  }
  pcnt[i] = w;
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

// A_l on the device, level by level: contributions, stable sort by (row, column), run sums in
// simplex order (the host's order), then the host's rule for the pattern: entries that sum to
// exactly zero off the diagonal (right angles) are dropped.
void assemble_levels_device(Hierarchy &h, int ordinal) {
  const int d = h.d, k = d + 1, J = h.J;
  HIPCHECK(hipSetDevice(ordinal));
  const double unit = std::ldexp(h.L, -h.J);
  Bufs WB;  // destroyed after the stream guard: the stream has drained before it is freed
  hipStream_t s;
  HIPCHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  struct StreamGuard {
    hipStream_t s;
    ~StreamGuard() {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
  } sg{s};
  h.Al.clear();
  // the Kuhn coefficients of every box once, sorted by code (looked up per level on the device)
  std::vector<std::pair<uint64_t, const KuhnW *>> wl;
  wl.reserve(h.kuhn_w.size());
  for (const auto &kv : h.kuhn_w) wl.push_back({(uint64_t)kv.first, &kv.second});
  std::sort(wl.begin(), wl.end(),
            [](const std::pair<uint64_t, const KuhnW *> &x, const std::pair<uint64_t, const KuhnW *> &y) {
              return x.first < y.first;
            });
  const int64_t nw = (int64_t)wl.size();
  std::vector<uint64_t> wcode((size_t)nw);
  std::vector<double> wtab((size_t)nw * 6);
  for (int64_t i = 0; i < nw; ++i) {
    wcode[i] = wl[i].first;
    for (int q = 0; q < 6; ++q) wtab[i * 6 + q] = (*wl[i].second)[q];
  }
  uint64_t *WC = WB.get<uint64_t>(nw);
  double *WT = WB.get<double>(nw * 6);
  int *missing = WB.get<int>(1);
  if (nw) {
    HIPCHECK(hipMemcpyAsync(WC, wcode.data(), (size_t)nw * 8, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(WT, wtab.data(), (size_t)nw * 6 * 8, hipMemcpyHostToDevice, s));
  }
  HIPCHECK(hipMemsetAsync(missing, 0, 4, s));
  // work arrays sized once for the largest level
  int64_t mns = 1, mnb = 1, mnv = 1, mn = 1;
  for (int l = J; l >= h.lc; --l) {
    const LevelMesh &lm = h.meshes.at(l);
    mns = std::max<int64_t>(mns, (int64_t)lm.simp_box.size());
    mnb = std::max<int64_t>(mnb, (int64_t)lm.boxes.size());
    mnv = std::max<int64_t>(mnv, lm.nverts());
    mn = std::max<int64_t>(mn, lm.n());
  }
  const int64_t mm = mns * k * k;
  if (mm >= ((int64_t)1 << 31) || mn >= ((int64_t)1 << 31) || mnv >= ((int64_t)1 << 31))
    throw AsmgError{ASMG_EINVAL, "level too large for the device assembly"};
  int64_t *V = WB.get<int64_t>(mnv * d), *S = WB.get<int64_t>(mns * k), *DV = WB.get<int64_t>(mnv);
  int *SB = WB.get<int>(mns);
  int8_t *ST = WB.get<int8_t>(mns);
  uint8_t *BF = WB.get<uint8_t>(mnb), *KP = WB.get<uint8_t>(mns);
  uint64_t *BCODE = WB.get<uint64_t>(mnb);
  double *BW = WB.get<double>(mnb * 6);
  uint64_t *key = WB.get<uint64_t>(mm), *key_s = WB.get<uint64_t>(mm);
  double *val = WB.get<double>(mm), *val_s = WB.get<double>(mm);
  int *head = WB.get<int>(mm), *pos = WB.get<int>(mm), *ci = WB.get<int>(mm), *rowcnt = WB.get<int>(mn);
  double *v = WB.get<double>(mm);
  size_t tb_sort = 0, tb_scan = 0;
  HIPCHECK(hipcub::DeviceRadixSort::SortPairs(nullptr, tb_sort, key, key_s, val, val_s, (int)mm, 0, 64, s));
  HIPCHECK(hipcub::DeviceScan::ExclusiveSum(nullptr, tb_scan, head, pos, (int)mm, s));
  const size_t tb = std::max(tb_sort, tb_scan);
  void *tmp = WB.get<char>((int64_t)tb);
  for (int l = J; l >= h.lc; --l) {
    const LevelMesh &lm = h.meshes.at(l);
    const int64_t ns = (int64_t)lm.simp_box.size(), nb = (int64_t)lm.boxes.size(), nvl = lm.nverts(),
                  n = lm.n(), m = ns * k * k;
    Csr &A = h.Al[l];
    A.nrows = A.ncols = n;
    if (m == 0 || n == 0) {
      A.rp.assign((size_t)n + 1, 0);
      A.ci.clear();
      A.v.clear();
      continue;
    }
    HIPCHECK(hipMemcpyAsync(V, lm.verts.data(), (size_t)nvl * d * 8, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(S, lm.simp.data(), (size_t)ns * k * 8, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(SB, lm.simp_box.data(), (size_t)ns * 4, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(DV, lm.dof_of_vert.data(), (size_t)nvl * 8, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(ST, lm.simp_tmpl.data(), (size_t)ns, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(BF, lm.fan.data(), (size_t)nb, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(BCODE, lm.boxes.data(), (size_t)nb * 8, hipMemcpyHostToDevice, s));
    if (!lm.kept.empty()) HIPCHECK(hipMemcpyAsync(KP, lm.kept.data(), (size_t)ns, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_box_weights, dim3(grid(nb)), dim3(TB), 0, s, nb, (const uint64_t *)BCODE,
                       (const uint64_t *)WC, nw, (const double *)WT, BW, missing);
    hipLaunchKernelGGL(k_level_contrib, dim3(grid(ns)), dim3(TB), 0, s, ns, d, J, unit, (const int64_t *)V,
                       (const int64_t *)S, (const int *)SB, (const int8_t *)ST, (const uint64_t *)BCODE,
                       (const uint8_t *)BF, (const double *)BW, lm.kept.empty() ? (const uint8_t *)nullptr : KP,
                       (const int64_t *)DV, key, val);
    size_t tbs = tb;
    HIPCHECK(hipcub::DeviceRadixSort::SortPairs(tmp, tbs, key, key_s, val, val_s, (int)m, 0, 64, s));
    hipLaunchKernelGGL(k_heads, dim3(grid(m)), dim3(TB), 0, s, m, (const uint64_t *)key_s, head);
    tbs = tb;
    HIPCHECK(hipcub::DeviceScan::ExclusiveSum(tmp, tbs, head, pos, (int)m, s));
    int last_pos = 0, last_head = 0;
    HIPCHECK(hipMemcpyAsync(&last_pos, pos + (m - 1), 4, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipMemcpyAsync(&last_head, head + (m - 1), 4, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipMemsetAsync(rowcnt, 0, (size_t)n * 4, s));
    hipLaunchKernelGGL(k_entries, dim3(grid(m)), dim3(TB), 0, s, m, (const uint64_t *)key_s, (const double *)val_s,
                       (const int *)head, (const int *)pos, ci, v, rowcnt);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(s));
    const int64_t nnz = (int64_t)last_pos + last_head;
    std::vector<int32_t> hci((size_t)nnz);
    std::vector<double> hv((size_t)nnz);
    std::vector<int> cnt((size_t)n);
    if (nnz) {
      HIPCHECK(hipMemcpyAsync(hci.data(), ci, (size_t)nnz * 4, hipMemcpyDeviceToHost, s));
      HIPCHECK(hipMemcpyAsync(hv.data(), v, (size_t)nnz * 8, hipMemcpyDeviceToHost, s));
    }
    HIPCHECK(hipMemcpyAsync(cnt.data(), rowcnt, (size_t)n * 4, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    // the host's pattern rule: drop entries that are exactly zero off the diagonal
    A.rp.assign((size_t)n + 1, 0);
    A.ci.resize((size_t)nnz);
    A.v.resize((size_t)nnz);
    int64_t p = 0, w = 0;
    for (int64_t i = 0; i < n; ++i) {
      for (int64_t e = p; e < p + cnt[i]; ++e)
        if (hv[e] != 0.0 || hci[e] == i) {
          A.ci[w] = hci[e];
          A.v[w] = hv[e];
          ++w;
        }
      p += cnt[i];
      A.rp[i + 1] = w;
    }
    A.ci.resize((size_t)w);
    A.v.resize((size_t)w);
    if (p != nnz) throw AsmgError{ASMG_EDEVICE, "device level assembly: row counts do not add up"};
  }
  int hmiss = 0;
  HIPCHECK(hipMemcpyAsync(&hmiss, missing, 4, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  if (hmiss) throw AsmgError{ASMG_EDEVICE, "device level assembly: a box without Kuhn coefficients"};
}

// P_l of every level l_c < l <= J on the device; false (nothing built) where the integer
// coordinates are too large for exact int64 determinants (2-D: J > 30, 3-D: J > 19)
bool prolongations_device(Hierarchy &h, int ordinal) {
  const int d = h.d, k1 = d + 1, J = h.J;
  if ((d == 2 && J > 30) || (d == 3 && J > 19)) return false;
  HIPCHECK(hipSetDevice(ordinal));
  hipStream_t s;
  HIPCHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  struct StreamGuard {
    hipStream_t s;
    ~StreamGuard() {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
  } sg{s};
  h.P.clear();
  for (int l = J; l > h.lc; --l) {
    const LevelMesh &fine = h.meshes.at(l), &coarse = h.meshes.at(l - 1);
    const int64_t n = fine.n(), nc = coarse.n(), ncb = (int64_t)coarse.boxes.size();
    Csr &P = h.P[l];
    P.nrows = n;
    P.ncols = nc;
    P.rp.assign((size_t)n + 1, 0);
    P.ci.clear();
    P.v.clear();
    if (n == 0) continue;
    if (n >= ((int64_t)1 << 31) || ncb >= ((int64_t)1 << 31) || coarse.nverts() >= ((int64_t)1 << 31))
      throw AsmgError{ASMG_EINVAL, "level too large for the device prolongation"};
    Bufs B;
    int64_t *FV = B.get<int64_t>(fine.nverts() * d), *FD = B.get<int64_t>(n), *CV = B.get<int64_t>(coarse.nverts() * d);
    int64_t *CBS = B.get<int64_t>(ncb + 1), *CS = B.get<int64_t>((int64_t)coarse.simp.size());
    int64_t *CD = B.get<int64_t>(coarse.nverts());
    uint64_t *CB0 = B.get<uint64_t>(ncb), *CC = B.get<uint64_t>(ncb);
    int *CI0 = B.get<int>(ncb), *CI = B.get<int>(ncb);
    int *PC = B.get<int>(n * k1), *PN = B.get<int>(n), *BAD = B.get<int>(1);
    double *PV = B.get<double>(n * k1);
    HIPCHECK(hipMemcpyAsync(FV, fine.verts.data(), (size_t)fine.nverts() * d * 8, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(FD, fine.dof_vert.data(), (size_t)n * 8, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(CV, coarse.verts.data(), (size_t)coarse.nverts() * d * 8, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(CBS, coarse.box_simp.data(), (size_t)(ncb + 1) * 8, hipMemcpyHostToDevice, s));
    if (!coarse.simp.empty())
      HIPCHECK(hipMemcpyAsync(CS, coarse.simp.data(), coarse.simp.size() * 8, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(CD, coarse.dof_of_vert.data(), (size_t)coarse.nverts() * 8, hipMemcpyHostToDevice, s));
    // the coarse level's active boxes sorted by code, with their indices (radix sort on the device)
    if (ncb) {
      HIPCHECK(hipMemcpyAsync(CB0, coarse.boxes.data(), (size_t)ncb * 8, hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_iota, dim3(grid(ncb)), dim3(TB), 0, s, ncb, CI0);
      size_t tb = 0;
      HIPCHECK(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, CB0, CC, CI0, CI, (int)ncb, 0, 64, s));
      void *tmp = B.get<char>((int64_t)tb);
      HIPCHECK(hipcub::DeviceRadixSort::SortPairs(tmp, tb, CB0, CC, CI0, CI, (int)ncb, 0, 64, s));
    }
    const int big = INT32_MAX;
    HIPCHECK(hipMemcpyAsync(BAD, &big, 4, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_prolong, dim3(grid(n)), dim3(TB), 0, s, (int)n, d, J, l, (const int64_t *)FV,
                       (const int64_t *)FD, (const int64_t *)CV, (const int64_t *)CS, (const uint64_t *)CC,
                       (const int *)CI, (int)ncb, (const int64_t *)CBS, (const int64_t *)CD, PC, PV, PN, BAD);
    HIPCHECK(hipGetLastError());
    std::vector<int> pc((size_t)n * k1), pn((size_t)n);
    std::vector<double> pv((size_t)n * k1);
    int hbad = 0;
    HIPCHECK(hipMemcpyAsync(pc.data(), PC, (size_t)n * k1 * 4, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipMemcpyAsync(pv.data(), PV, (size_t)n * k1 * 8, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipMemcpyAsync(pn.data(), PN, (size_t)n * 4, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipMemcpyAsync(&hbad, BAD, 4, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    if (hbad != INT32_MAX)
      throw AsmgError{ASMG_EINVAL, "prolongation: point location failed at unknown " + std::to_string(hbad)};
    P.ci.reserve((size_t)n * 2);
    P.v.reserve((size_t)n * 2);
    for (int64_t i = 0; i < n; ++i) {
      for (int q = 0; q < pn[i]; ++q) {
        P.ci.push_back(pc[i * k1 + q]);
        P.v.push_back(pv[i * k1 + q]);
      }
      P.rp[i + 1] = (int64_t)P.ci.size();
    }
  }
  return true;
}

}  // namespace asmg
