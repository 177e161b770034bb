// Level meshes sigma^(l) on the device (Section 3.3): the active boxes of level l (the tree's
// boxes of that level and the leaves of coarser levels), in the Morton order of their lower
// corners; each box split by its template: Kuhn simplices, or, where a same-level box sharing a
// facet (3-D: or an edge) is refined, the fan from the box centre over the box's boundary with
// the hanging midpoints (2-D) or the face triangulations (3-D); the vertices numbered by the rank
// of their Morton key; the unknowns the vertices inside the root box.
//
// Identical to make_level_mesh in setup.cpp: every box is handled by one thread that emits its
// simplices in the host's template order (a counting pass sizes the output), the boxes and the
// vertices are ordered by the same keys, and equal vertex keys keep their first position (a
// stable radix sort). Used on the root box (no general domain) while the Morton keys of the
// vertices fit 64 bits ((J+1) d <= 64).
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "common.hpp"
#include "setup.hpp"
#include "trace.hpp"
#include "tree.hpp"

namespace asmg {
namespace {

constexpr int LB = 256;

__device__ __forceinline__ int lv_level(uint64_t c, int d) { return (63 - __clzll((long long)c)) / d + 1; }

__device__ __forceinline__ void lv_index(uint64_t c, int d, int64_t *idx) {
  const int bits = lv_level(c, d) - 1;
  for (int k = 0; k < d; ++k) idx[k] = 0;
  for (int b = 0; b < bits; ++b)
    for (int k = 0; k < d; ++k) idx[k] |= (int64_t)((c >> (b * d + (d - 1 - k))) & 1) << b;
}

__device__ __forceinline__ uint64_t lv_code(int level, const int64_t *idx, int d) {
  uint64_t m = 0;
  const int bits = level - 1;
  for (int b = 0; b < bits; ++b)
    for (int k = 0; k < d; ++k) m |= (uint64_t)((idx[k] >> b) & 1) << (b * d + (d - 1 - k));
  return m | ((uint64_t)1 << (d * bits));
}

// bit b of x moved to bit d*b (the host's spread_bits)
__device__ __forceinline__ uint64_t lv_spread(uint64_t x, int d) {
  if (d == 2) {
    x &= 0xffffffffULL;
    x = (x | (x << 16)) & 0x0000ffff0000ffffULL;
    x = (x | (x << 8)) & 0x00ff00ff00ff00ffULL;
    x = (x | (x << 4)) & 0x0f0f0f0f0f0f0f0fULL;
    x = (x | (x << 2)) & 0x3333333333333333ULL;
    x = (x | (x << 1)) & 0x5555555555555555ULL;
  } else {
    x &= 0x1fffffULL;
    x = (x | (x << 32)) & 0x001f00000000ffffULL;
    x = (x | (x << 16)) & 0x001f0000ff0000ffULL;
    x = (x | (x << 8)) & 0x100f00f00f00f00fULL;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ULL;
    x = (x | (x << 2)) & 0x1249249249249249ULL;
  }
  return x;
}

__device__ __forceinline__ uint64_t lv_morton(const int64_t *X, int d) {
  uint64_t m = 0;
  for (int k = 0; k < d; ++k) m |= lv_spread((uint64_t)X[k], d) << (d - 1 - k);
  return m;
}

// is code c in the sorted refined set R[0, nr)?
__device__ __forceinline__ bool lv_in(const uint64_t *__restrict__ R, int64_t nr, uint64_t c) {
  int64_t lo = 0, hi = nr;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (R[mid] < c)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo < nr && R[lo] == c;
}

// same-level box at offset o, refined
__device__ __forceinline__ bool lv_nbr_refined(const uint64_t *R, int64_t nr, uint64_t b, int d, int ox, int oy,
                                               int oz) {
  int64_t idx[3];
  lv_index(b, d, idx);
  const int lev = lv_level(b, d);
  const int64_t n = (int64_t)1 << (lev - 1);
  const int o[3] = {ox, oy, oz};
  for (int k = 0; k < d; ++k) {
    idx[k] += o[k];
    if (idx[k] < 0 || idx[k] >= n) return false;
  }
  return lv_in(R, nr, lv_code(lev, idx, d));
}

// a box of a coarser level with a refined same-level box sharing a facet (3-D: or an edge)
__device__ bool lv_is_fan(const uint64_t *R, int64_t nr, uint64_t b, int d, int level) {
  if (lv_level(b, d) >= level) return false;
  for (int x = -1; x <= 1; ++x)
    for (int y = -1; y <= 1; ++y)
      for (int z = (d == 3 ? -1 : 0); z <= (d == 3 ? 1 : 0); ++z) {
        const int nz = (x != 0) + (y != 0) + (z != 0);
        if (!(nz == 1 || (d == 3 && nz == 2))) continue;
        if (lv_nbr_refined(R, nr, b, d, x, y, z)) return true;
      }
  return false;
}

// Output of one box's simplices: with `pts` null only counts them.
struct Emit {
  int64_t *pts;   // (d+1) d coordinates per simplex
  int *sbox;
  int8_t *stmpl;
  int64_t at;     // next simplex
  int d, box;
  int t;          // template position within the box
  __device__ void add(const int64_t *v) {
    if (pts) {
      const int n = (d + 1) * d;
      for (int q = 0; q < n; ++q) pts[at * n + q] = v[q];
      sbox[at] = box;
      stmpl[at] = (int8_t)t;
    }
    ++at;
    ++t;
  }
};

__device__ void lv_kuhn(int d, const int64_t *c, int64_t S, Emit &em) {
  const int P2[2][2] = {{0, 1}, {1, 0}};
  const int P3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  const int nperm = d == 2 ? 2 : 6;
  for (int t = 0; t < nperm; ++t) {
    int64_t v[4][3];
    for (int q = 0; q < d; ++q) v[0][q] = c[q];
    for (int m = 0; m < d - 1; ++m) {
      for (int q = 0; q < d; ++q) v[m + 1][q] = v[m][q];
      v[m + 1][d == 2 ? P2[t][m] : P3[t][m]] += S;
    }
    for (int q = 0; q < d; ++q) v[d][q] = c[q] + S;
    int64_t flat[12];
    for (int m = 0; m <= d; ++m)
      for (int q = 0; q < d; ++q) flat[m * d + q] = v[m][q];
    em.add(flat);
  }
}

__device__ void lv_fan2(const uint64_t *R, int64_t nr, uint64_t b, const int64_t *c, int64_t S, Emit &em) {
  const int64_t H = S / 2;
  const int64_t LL[2] = {c[0], c[1]}, LR[2] = {c[0] + S, c[1]}, UR[2] = {c[0] + S, c[1] + S}, UL[2] = {c[0], c[1] + S};
  const int64_t C[2] = {c[0] + H, c[1] + H};
  const int64_t *E[4][2] = {{LL, LR}, {LR, UR}, {UR, UL}, {UL, LL}};
  const int O[4][2] = {{0, -1}, {1, 0}, {0, 1}, {-1, 0}};
  for (int e = 0; e < 4; ++e) {
    const int64_t *v0 = E[e][0], *v1 = E[e][1];
    if (lv_nbr_refined(R, nr, b, 2, O[e][0], O[e][1], 0)) {
      const int64_t m[2] = {(v0[0] + v1[0]) / 2, (v0[1] + v1[1]) / 2};
      const int64_t t1[6] = {v0[0], v0[1], m[0], m[1], C[0], C[1]};
      const int64_t t2[6] = {m[0], m[1], v1[0], v1[1], C[0], C[1]};
      em.add(t1);
      em.add(t2);
    } else {
      const int64_t t1[6] = {v0[0], v0[1], v1[0], v1[1], C[0], C[1]};
      em.add(t1);
    }
  }
}

__device__ void lv_fan3(const uint64_t *R, int64_t nr, uint64_t b, const int64_t *c, int64_t S, Emit &em) {
  const int64_t H = S / 2;
  const int64_t C[3] = {c[0] + H, c[1] + H, c[2] + H};
  for (int ax = 0; ax < 3; ++ax) {
    const int u = ax == 0 ? 1 : 0, v = ax == 2 ? 1 : 2;
    for (int s = 0; s < 2; ++s) {
      int of[3] = {0, 0, 0};
      of[ax] = 2 * s - 1;
      int64_t base[3] = {c[0], c[1], c[2]};
      base[ax] += s * S;
      auto P = [&](int al2, int be2, int64_t *out) {
        for (int q = 0; q < 3; ++q) out[q] = base[q];
        out[u] += al2 * H;
        out[v] += be2 * H;
      };
      auto inR = [&](const int *o) { return lv_nbr_refined(R, nr, b, 3, o[0], o[1], o[2]); };
      const int ea[4][4] = {{0, 0, 2, 0}, {2, 0, 2, 2}, {2, 2, 0, 2}, {0, 2, 0, 0}};
      int ip[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
      ip[0][v] = -1;
      ip[1][u] = 1;
      ip[2][v] = 1;
      ip[3][u] = -1;
      const bool face_refined = inR(of);
      bool mid[4], anymid = false;
      for (int e = 0; e < 4; ++e) {
        const int both[3] = {of[0] + ip[e][0], of[1] + ip[e][1], of[2] + ip[e][2]};
        mid[e] = face_refined || inR(ip[e]) || inR(both);
        anymid = anymid || mid[e];
      }
      auto tri = [&](const int64_t *p, const int64_t *q, const int64_t *r) {
        int64_t flat[12];
        for (int k = 0; k < 3; ++k) {
          flat[k] = p[k];
          flat[3 + k] = q[k];
          flat[6 + k] = r[k];
          flat[9 + k] = C[k];
        }
        em.add(flat);
      };
      if (face_refined) {
        for (int be0 = 0; be0 < 2; ++be0)
          for (int al0 = 0; al0 < 2; ++al0) {
            int64_t p00[3], p10[3], p11[3], p01[3];
            P(al0, be0, p00);
            P(al0 + 1, be0, p10);
            P(al0 + 1, be0 + 1, p11);
            P(al0, be0 + 1, p01);
            tri(p00, p10, p11);
            tri(p00, p01, p11);
          }
      } else if (anymid) {
        int64_t FC[3];
        P(1, 1, FC);
        for (int e = 0; e < 4; ++e) {
          int64_t p0[3], p1[3];
          P(ea[e][0], ea[e][1], p0);
          P(ea[e][2], ea[e][3], p1);
          if (mid[e]) {
            const int64_t pm[3] = {(p0[0] + p1[0]) / 2, (p0[1] + p1[1]) / 2, (p0[2] + p1[2]) / 2};
            tri(p0, pm, FC);
            tri(pm, p1, FC);
          } else {
            tri(p0, p1, FC);
          }
        }
      } else {
        int64_t p00[3], p20[3], p22[3], p02[3];
        P(0, 0, p00);
        P(2, 0, p20);
        P(2, 2, p22);
        P(0, 2, p02);
        tri(p00, p20, p22);
        tri(p00, p02, p22);
      }
    }
  }
}

// one thread per active box (sorted): fan flag and simplex count (pts null), or the simplices
// themselves at offsets soff
__global__ __launch_bounds__(LB) void k_box_simplices(int64_t nb, int d, int J, int level,
                                                      const uint64_t *__restrict__ boxes, const uint64_t *__restrict__ R,
                                                      int64_t nr, const int64_t *__restrict__ soff, uint8_t *__restrict__ fan,
                                                      int64_t *__restrict__ cnt, int64_t *__restrict__ pts,
                                                      int *__restrict__ sbox, int8_t *__restrict__ stmpl) {
  const int64_t i = blockIdx.x * (int64_t)LB + threadIdx.x;
  if (i >= nb) return;
  const uint64_t b = boxes[i];
  int64_t idx[3], cor[3];
  lv_index(b, d, idx);
  const int64_t S = (int64_t)1 << (J - lv_level(b, d) + 1);
  for (int q = 0; q < d; ++q) cor[q] = idx[q] * S;
  const bool f = lv_is_fan(R, nr, b, d, level);
  Emit em{pts, sbox, stmpl, pts ? soff[i] : 0, d, (int)i, 0};
  if (!f)
    lv_kuhn(d, cor, S, em);
  else if (d == 2)
    lv_fan2(R, nr, b, cor, S, em);
  else
    lv_fan3(R, nr, b, cor, S, em);
  if (!pts) {
    fan[i] = f ? 1 : 0;
    cnt[i] = em.at;
  }
}

// Morton key of each box's lower corner
__global__ __launch_bounds__(LB) void k_box_keys(int64_t nb, int d, int J, const uint64_t *__restrict__ boxes,
                                                 uint64_t *__restrict__ key) {
  const int64_t i = blockIdx.x * (int64_t)LB + threadIdx.x;
  if (i >= nb) return;
  int64_t idx[3], cor[3];
  lv_index(boxes[i], d, idx);
  const int sh = J - lv_level(boxes[i], d) + 1;
  for (int q = 0; q < d; ++q) cor[q] = idx[q] << sh;
  key[i] = lv_morton(cor, d);
}

__global__ __launch_bounds__(LB) void k_leaf_flags(int64_t nl, int d, int level, const uint64_t *__restrict__ leaves,
                                                   uint8_t *__restrict__ flag) {
  const int64_t i = blockIdx.x * (int64_t)LB + threadIdx.x;
  if (i < nl) flag[i] = lv_level(leaves[i], d) < level ? 1 : 0;
}

__global__ __launch_bounds__(LB) void k_children(int64_t n, int d, const uint64_t *__restrict__ parents,
                                                 uint64_t *__restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)LB + threadIdx.x;
  if (i >= n) return;
  const int nc = 1 << d;
  out[i] = (parents[i / nc] << d) | (uint64_t)(i % nc);
}

// vertex key and position of every simplex corner
__global__ __launch_bounds__(LB) void k_vertex_keys(int64_t nvtx, int d, const int64_t *__restrict__ pts,
                                                    uint64_t *__restrict__ key, int64_t *__restrict__ pos) {
  const int64_t i = blockIdx.x * (int64_t)LB + threadIdx.x;
  if (i >= nvtx) return;
  key[i] = lv_morton(pts + i * d, d);
  pos[i] = i;
}

__global__ __launch_bounds__(LB) void k_run_heads(int64_t n, const uint64_t *__restrict__ key, int64_t *__restrict__ head) {
  const int64_t i = blockIdx.x * (int64_t)LB + threadIdx.x;
  if (i < n) head[i] = (i == 0 || key[i] != key[i - 1]) ? 1 : 0;
}

// rank of every corner's vertex (inclusive head scan - 1) and the coordinates of each vertex
// from the first corner of its run
__global__ __launch_bounds__(LB) void k_vertex_ranks(int64_t n, int d, const int64_t *__restrict__ pos,
                                                     const int64_t *__restrict__ head,
                                                     const int64_t *__restrict__ incl, const int64_t *__restrict__ pts,
                                                     int64_t *__restrict__ simp, int64_t *__restrict__ verts) {
  const int64_t j = blockIdx.x * (int64_t)LB + threadIdx.x;
  if (j >= n) return;
  const int64_t r = incl[j] - 1, p = pos[j];
  simp[p] = r;
  if (head[j])
    for (int q = 0; q < d; ++q) verts[r * d + q] = pts[p * d + q];
}

// unknowns: the vertices strictly inside the root box
__global__ __launch_bounds__(LB) void k_inside(int64_t nv, int d, int64_t top, const int64_t *__restrict__ verts,
                                               int64_t *__restrict__ in) {
  const int64_t v = blockIdx.x * (int64_t)LB + threadIdx.x;
  if (v >= nv) return;
  bool ok = true;
  for (int q = 0; q < d; ++q) {
    const int64_t x = verts[v * d + q];
    ok = ok && x > 0 && x < top;
  }
  in[v] = ok ? 1 : 0;
}

struct LvBufs {
  std::vector<void *> p;
  template <class T>
  T *get(int64_t n) {
    void *q = nullptr;
    HIPCHECK(hipMalloc(&q, (size_t)std::max<int64_t>(n, 1) * sizeof(T)));
    p.push_back(q);
    return (T *)q;
  }
  ~LvBufs() {
    for (void *q : p) (void)hipFree(q);
  }
};

inline int lgrid(int64_t n) { return (int)std::max<int64_t>(1, (n + LB - 1) / LB); }

template <class F>
void cub_tmp(LvBufs &B, F f) {
  size_t tb = 0;
  HIPCHECK(f(nullptr, tb));
  void *tmp = B.get<char>((int64_t)tb);
  HIPCHECK(f(tmp, tb));
}

LevelMesh device_level_mesh(const Hierarchy &h, int level, const uint64_t *dR, int64_t nr,
                            const std::vector<uint64_t> &Rs, const uint64_t *dleaves, int64_t nl, hipStream_t s) {
  const int d = h.d, J = h.J, k = d + 1;
  LevelMesh lm;
  lm.level = level;
  LvBufs B;
  // active boxes: leaves of coarser levels, the children of the refined boxes of level - 1
  uint8_t *flag = B.get<uint8_t>(nl);
  uint64_t *act = nullptr;
  int64_t na_leaves = 0;
  int64_t *nsel = B.get<int64_t>(1);
  HIPCHECK(hipMemsetAsync(nsel, 0, 8, s));
  hipLaunchKernelGGL(k_leaf_flags, dim3(lgrid(nl)), dim3(LB), 0, s, nl, d, level, dleaves, flag);
  // parents: the refined boxes of level - 1 form one range of the sorted R (codes of a level are
  // contiguous: marker bit above the index bits)
  int64_t p0 = 0, p1 = 0;
  if (level >= 2) {
    const uint64_t lo = (uint64_t)1 << (d * (level - 2)), hi = (uint64_t)1 << (d * (level - 1));
    p0 = std::lower_bound(Rs.begin(), Rs.end(), lo) - Rs.begin();
    p1 = std::lower_bound(Rs.begin(), Rs.end(), hi) - Rs.begin();
  }
  const int64_t nchild = level == 1 ? 1 : (p1 - p0) << d;
  uint64_t *sel = B.get<uint64_t>(nl + nchild);
  cub_tmp(B, [&](void *t, size_t &tb) {
    return hipcub::DeviceSelect::Flagged(t, tb, dleaves, flag, sel, nsel, (int)nl, s);
  });
  HIPCHECK(hipMemcpyAsync(&na_leaves, nsel, 8, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  if (na_leaves < 0 || na_leaves > nl) throw AsmgError{ASMG_EDEVICE, "device level mesh: bad leaf count"};
  const int64_t nb = na_leaves + nchild;
  if (level == 1) {
    const uint64_t root = 1;
    HIPCHECK(hipMemcpyAsync(sel + na_leaves, &root, 8, hipMemcpyHostToDevice, s));
  } else if (nchild) {
    hipLaunchKernelGGL(k_children, dim3(lgrid(nchild)), dim3(LB), 0, s, nchild, d, dR + p0, sel + na_leaves);
  }
  act = sel;
  // Morton order of the lower corners (distinct: the active boxes tile the root box)
  uint64_t *bkey = B.get<uint64_t>(nb), *bkey_s = B.get<uint64_t>(nb), *boxes = B.get<uint64_t>(nb);
  hipLaunchKernelGGL(k_box_keys, dim3(lgrid(nb)), dim3(LB), 0, s, nb, d, J, (const uint64_t *)act, bkey);
  cub_tmp(B, [&](void *t, size_t &tb) {
    return hipcub::DeviceRadixSort::SortPairs(t, tb, bkey, bkey_s, act, boxes, (int)nb, 0, 64, s);
  });
  // templates: counts, offsets, simplices
  uint8_t *fan = B.get<uint8_t>(nb);
  int64_t *cnt = B.get<int64_t>(nb), *soff = B.get<int64_t>(nb + 1);
  hipLaunchKernelGGL(k_box_simplices, dim3(lgrid(nb)), dim3(LB), 0, s, nb, d, J, level, (const uint64_t *)boxes, dR, nr,
                     (const int64_t *)nullptr, fan, cnt, (int64_t *)nullptr, (int *)nullptr, (int8_t *)nullptr);
  HIPCHECK(hipMemsetAsync(soff, 0, 8, s));
  cub_tmp(B, [&](void *t, size_t &tb) { return hipcub::DeviceScan::InclusiveSum(t, tb, cnt, soff + 1, (int)nb, s); });
  int64_t ns = 0;
  HIPCHECK(hipMemcpyAsync(&ns, soff + nb, 8, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  const int64_t nvtx = ns * k;
  if (nvtx >= ((int64_t)1 << 31)) throw AsmgError{ASMG_EINVAL, "level mesh too large for the device build"};
  int64_t *pts = B.get<int64_t>(nvtx * d);
  int *sbox = B.get<int>(ns);
  int8_t *stmpl = B.get<int8_t>(ns);
  hipLaunchKernelGGL(k_box_simplices, dim3(lgrid(nb)), dim3(LB), 0, s, nb, d, J, level, (const uint64_t *)boxes, dR, nr,
                     (const int64_t *)soff, fan, cnt, pts, sbox, stmpl);
  // vertex numbering: rank of the Morton key among the distinct keys
  uint64_t *vkey = B.get<uint64_t>(nvtx), *vkey_s = B.get<uint64_t>(nvtx);
  int64_t *vpos = B.get<int64_t>(nvtx), *vpos_s = B.get<int64_t>(nvtx);
  hipLaunchKernelGGL(k_vertex_keys, dim3(lgrid(nvtx)), dim3(LB), 0, s, nvtx, d, (const int64_t *)pts, vkey, vpos);
  cub_tmp(B, [&](void *t, size_t &tb) {
    return hipcub::DeviceRadixSort::SortPairs(t, tb, vkey, vkey_s, vpos, vpos_s, (int)nvtx, 0, (J + 1) * d, s);
  });
  int64_t *head = B.get<int64_t>(nvtx), *incl = B.get<int64_t>(nvtx);
  hipLaunchKernelGGL(k_run_heads, dim3(lgrid(nvtx)), dim3(LB), 0, s, nvtx, (const uint64_t *)vkey_s, head);
  cub_tmp(B, [&](void *t, size_t &tb) { return hipcub::DeviceScan::InclusiveSum(t, tb, head, incl, (int)nvtx, s); });
  int64_t nv = 0;
  HIPCHECK(hipMemcpyAsync(&nv, incl + (nvtx - 1), 8, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  int64_t *simp = B.get<int64_t>(nvtx), *verts = B.get<int64_t>(nv * d);
  hipLaunchKernelGGL(k_vertex_ranks, dim3(lgrid(nvtx)), dim3(LB), 0, s, nvtx, d, (const int64_t *)vpos_s,
                     (const int64_t *)head, (const int64_t *)incl, (const int64_t *)pts, simp, verts);
  // unknowns
  int64_t *in = B.get<int64_t>(nv);
  hipLaunchKernelGGL(k_inside, dim3(lgrid(nv)), dim3(LB), 0, s, nv, d, (int64_t)1 << J, (const int64_t *)verts, in);
  // back to the host
  lm.boxes.resize((size_t)nb);
  lm.fan.resize((size_t)nb);
  lm.simp.resize((size_t)nvtx);
  lm.simp_box.resize((size_t)ns);
  lm.simp_tmpl.resize((size_t)ns);
  lm.verts.resize((size_t)(nv * d));
  lm.box_simp.resize((size_t)nb + 1);
  std::vector<int64_t> inside((size_t)nv);
  HIPCHECK(hipMemcpyAsync(lm.boxes.data(), boxes, (size_t)nb * 8, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipMemcpyAsync(lm.fan.data(), fan, (size_t)nb, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipMemcpyAsync(lm.simp.data(), simp, (size_t)nvtx * 8, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipMemcpyAsync(lm.simp_box.data(), sbox, (size_t)ns * 4, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipMemcpyAsync(lm.simp_tmpl.data(), stmpl, (size_t)ns, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipMemcpyAsync(lm.verts.data(), verts, (size_t)nv * d * 8, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipMemcpyAsync(lm.box_simp.data(), soff, (size_t)(nb + 1) * 8, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipMemcpyAsync(inside.data(), in, (size_t)nv * 8, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  lm.dof_of_vert.assign((size_t)nv, -1);
  for (int64_t v = 0; v < nv; ++v)
    if (inside[v]) {
      lm.dof_of_vert[v] = (int64_t)lm.dof_vert.size();
      lm.dof_vert.push_back(v);
    }
  return lm;
}

}  // namespace

bool build_level_meshes_device(Hierarchy &h, int ordinal) {
  const int d = h.d, J = h.J;
  if (h.domain || (J + 1) * d > 64) return false;
  HIPCHECK(hipSetDevice(ordinal));
  {
    TraceRange r("asmg::setup::level_means");
    compute_level_means(h);
  }
  TraceRange r("asmg::setup::level_meshes");
  std::vector<uint64_t> Rs(h.R.begin(), h.R.end());
  std::sort(Rs.begin(), Rs.end());
  std::vector<uint64_t> leaves(h.leaves.begin(), h.leaves.end());
  LvBufs B;  // destroyed after the stream guard: the stream has drained before it is freed
  hipStream_t s;
  HIPCHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  struct StreamGuard {
    hipStream_t s;
    ~StreamGuard() {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
  } sg{s};
  uint64_t *dR = B.get<uint64_t>((int64_t)Rs.size()), *dL = B.get<uint64_t>((int64_t)leaves.size());
  if (!Rs.empty()) HIPCHECK(hipMemcpyAsync(dR, Rs.data(), Rs.size() * 8, hipMemcpyHostToDevice, s));
  if (!leaves.empty()) HIPCHECK(hipMemcpyAsync(dL, leaves.data(), leaves.size() * 8, hipMemcpyHostToDevice, s));
  const int Nc = h.opt.coarse_max_dofs > 0 ? h.opt.coarse_max_dofs : 1024;
  h.level_n.assign(J, -1);
  h.meshes.clear();
  h.lc = 1;
  // the box lookup of the host's transfer builder (level J), and of the host's point location
  // where the device prolongation does not apply (every level)
  const bool host_prolong = (d == 2 && J > 30) || (d == 3 && J > 19);
  for (int l = J; l >= 1; --l) {
    LevelMesh lm = device_level_mesh(h, l, dR, (int64_t)Rs.size(), Rs, dL, (int64_t)leaves.size(), s);
    if (l == J || host_prolong) {
      lm.box_index.reserve(lm.boxes.size());
      for (size_t i = 0; i < lm.boxes.size(); ++i) lm.box_index[lm.boxes[i]] = (int32_t)i;
    }
    h.level_n[l - 1] = lm.n();
    const bool bottom = lm.n() <= Nc;
    h.meshes.emplace(l, std::move(lm));
    if (bottom) {
      h.lc = l;
      break;
    }
  }
  return true;
}

}  // namespace asmg
