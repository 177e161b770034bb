// C ABI (include/asmg.h): argument checks, error codes, exports of setup objects.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>
#include <string>
#include <thread>
#include <atomic>
#include <mutex>

#include "../../include/asmg.h"
#include "batch.hpp"
#include "device.hpp"
#include "trace.hpp"
#include "tree.hpp"
#include "setup.hpp"

using namespace asmg;

struct asmg_s {
  Hierarchy h;                                     // single-mesh handle
  Device *dev = nullptr;
  std::vector<std::unique_ptr<Hierarchy>> batch;   // batch handle: one hierarchy per mesh
  BatchDevice *bdev = nullptr;
  bool is_batch() const { return !batch.empty(); }
};

static thread_local std::string g_err;

static int set_err(int code, const std::string &m) {
  g_err = m;
  return code;
}

#define ASMG_TRY(...)                                       \
  try {                                                     \
    __VA_ARGS__                                             \
  } catch (const AsmgError &e) {                            \
    return set_err(e.code, e.msg);                          \
  } catch (const std::bad_alloc &) {                        \
    return set_err(ASMG_ENOMEM, "host allocation failed");  \
  } catch (const std::exception &e) {                       \
    return set_err(ASMG_EDEVICE, e.what());                 \
  }

// --------------------------------------------------------------------------
// exports
// --------------------------------------------------------------------------

template <class T>
static int put(const std::vector<T> &src, void *buf, int64_t *count) {
  if (!buf) {
    *count = (int64_t)src.size();
    return ASMG_OK;
  }
  int64_t m = std::min<int64_t>(*count, (int64_t)src.size());
  std::memcpy(buf, src.data(), (size_t)m * sizeof(T));
  *count = m;
  return ASMG_OK;
}

static std::vector<int64_t> boxes_tuples(const Hierarchy &h, std::vector<BoxCode> v) {
  const int d = h.d;
  std::vector<std::vector<int64_t>> t;
  for (BoxCode b : v) {
    std::vector<int64_t> x(d + 1);
    x[0] = box_level(b, d);
    box_index(b, d, &x[1]);
    t.push_back(x);
  }
  std::sort(t.begin(), t.end());
  std::vector<int64_t> out;
  for (auto &x : t) out.insert(out.end(), x.begin(), x.end());
  return out;
}

static int put_csr(const Csr &A, const std::string &part, void *buf, int64_t *count) {
  if (part == "rowptr") return put(A.rp, buf, count);
  if (part == "col") {
    std::vector<int64_t> c(A.ci.begin(), A.ci.end());
    return put(c, buf, count);
  }
  return put(A.v, buf, count);
}


extern "C" {

const char *asmg_last_error(void) { return g_err.c_str(); }

int asmg_default_options(asmg_options *o) {
  if (!o) return set_err(ASMG_EINVAL, "null options");
  o->n_min = 0;
  o->nu_aux = 2;
  o->nu_fine = 1;
  o->coarse_max_dofs = 1024;
  o->max_iter = 1000;
  o->precision = ASMG_PREC_FP64;
  o->colour_seed = 0;
  o->device = 0;
  o->check_every = 0;
  o->colouring = 2;
  o->smoothing = 0;
  o->domain = 0;
  o->autotune = 1;
  o->nested = 0;
  o->setup_device = 0;
  o->red_blocks = 0;
  o->nb_layers = 0;
  return ASMG_OK;
}

int asmg_setup(int dim, int64_t n_vertices, const double *coords, int64_t n_elements, const int32_t *elems,
               const double *kappa, const uint8_t *dirichlet, const asmg_options *opt, asmg_handle *out) {
  if (!out) return set_err(ASMG_EINVAL, "null output handle");
  *out = nullptr;
  if (dim != 2 && dim != 3) return set_err(ASMG_EINVAL, "dim must be 2 or 3");
  if (n_vertices <= 0 || n_elements <= 0 || !coords || !elems || !kappa)
    return set_err(ASMG_EINVAL, "empty mesh or null array");
  if (n_vertices > INT32_MAX) return set_err(ASMG_EINVAL, "too many vertices");
  asmg_options o;
  asmg_default_options(&o);
  if (opt) o = *opt;
  if (o.nu_aux < 1 || o.nu_fine < 1 || o.max_iter < 1 || o.coarse_max_dofs < 1 || o.coarse_max_dofs > 8192 ||
      (o.precision != ASMG_PREC_FP64 && o.precision != ASMG_PREC_MIXED) || o.n_min < 0 || o.colouring < 0 ||
      o.colouring > 2 || o.smoothing < 0 || o.smoothing > 1 || o.domain < 0 || o.domain > 2 ||
      (o.domain >= 1 && dim != 2) || o.nested < 0 || o.nested > 16 || o.setup_device < 0 || o.setup_device > 1 ||
      (o.setup_device == 1 && o.device < 0) || o.red_blocks < 0 || o.red_blocks > 2048 || o.nb_layers < 0 ||
      o.nb_layers > 16)
    return set_err(ASMG_EINVAL, "invalid options");
  if (o.nb_layers > 0 && o.smoothing != 0)
    return set_err(ASMG_EINVAL, "the near-boundary correction needs whole-level smoothing (smoothing = 0)");
  if (o.nested > 0 && o.smoothing != 0)
    return set_err(ASMG_EINVAL, "the nested iteration needs whole-level smoothing (smoothing = 0)");
  for (int64_t i = 0; i < n_vertices * dim; ++i)
    if (!std::isfinite(coords[i])) return set_err(ASMG_EINVAL, "non-finite coordinate");
  for (int64_t i = 0; i < n_elements * (dim + 1); ++i)
    if (elems[i] < 0 || elems[i] >= n_vertices) return set_err(ASMG_EINVAL, "element vertex id out of range");
  for (int64_t e = 0; e < n_elements; ++e)
    if (!(kappa[e] > 0) || !std::isfinite(kappa[e])) return set_err(ASMG_EINVAL, "kappa must be finite and > 0");
  ASMG_TRY({
    std::unique_ptr<asmg_s> HP(new asmg_s());
    asmg_s *H = HP.get();
    Hierarchy &h = H->h;
    h.d = dim;
    h.nv = n_vertices;
    h.ne = n_elements;
    h.opt = o;
    h.coords.assign(coords, coords + n_vertices * dim);
    h.elems.assign(elems, elems + n_elements * (dim + 1));
    h.kappa.assign(kappa, kappa + n_elements);
    if (dirichlet) h.dirichlet.assign(dirichlet, dirichlet + n_vertices);
    const bool tm = std::getenv("ASMG_SETUP_TIMING") != nullptr;
    auto t0 = std::chrono::steady_clock::now();
    auto lap = [&](const char *what) {
      auto t1 = std::chrono::steady_clock::now();
      const double sec = std::chrono::duration<double>(t1 - t0).count();
      h.setup_seconds.push_back(sec);
      if (tm) std::fprintf(stderr, "[asmg setup] %-12s %8.3f s\n", what, sec);
      t0 = t1;
    };
    TraceRange all("asmg::setup");
    {
      TraceRange r("asmg::setup::fine");
      if (o.setup_device == 1) {
        build_fine_device(h, o.device);
        h.device_stages |= 1;
      } else {
        build_fine(h);
      }
    }
    lap("fine");
    {
      TraceRange r("asmg::setup::tree");
      if (o.setup_device == 1) {
        build_tree_device(h, o.device);
        h.device_stages |= 2;
      } else {
        build_tree(h);
      }
      if (o.domain >= 1) build_domain(h);
    }
    lap("tree");
    {
      TraceRange r("asmg::setup::levels");
      if (o.setup_device == 1) {
        if (build_level_meshes_device(h, o.device))
          h.device_stages |= 4;
        else
          build_level_meshes(h);
        {
          TraceRange r2("asmg::setup::level_matrices");
          assemble_levels_device(h, o.device);
        }
        h.device_stages |= 8;
        bool p_dev = false;
        {
          TraceRange r2("asmg::setup::prolongations");
          p_dev = prolongations_device(h, o.device);
          if (!p_dev) build_level_operators(h, false, true);
        }
        if (p_dev) h.device_stages |= 16;
      } else {
        build_levels(h);
      }
    }
    lap("levels");
    {
      TraceRange r("asmg::setup::transfer");
      if (o.setup_device == 1 && build_transfer_device(h, o.device))
        h.device_stages |= 32;
      else
        build_transfer(h);
    }
    lap("transfer");
    {
      TraceRange r("asmg::setup::colourings");
      if (o.setup_device == 1 && o.colouring == 1) {
        build_colourings_device(h, o.device);
        h.device_stages |= 64;
      } else {
        build_colourings(h);
      }
      build_local_sets(h);
    }
    lap("colourings");
    {
      TraceRange r("asmg::setup::coarse");
      build_coarse(h);
      build_near_boundary(h);
    }
    lap("coarse");
    if (o.device >= 0) {
      TraceRange r("asmg::setup::device_layout");
      H->dev = device_create(h, o.device);
    }
    lap("upload");
    *out = HP.release();
    return ASMG_OK;
  })
}

int asmg_update_coefficient(asmg_handle H, const double *kappa) {
  if (!H || !kappa) return set_err(ASMG_EINVAL, "null argument");
  Hierarchy &h = H->h;
  for (int64_t e = 0; e < h.ne; ++e)
    if (!(kappa[e] > 0) || !std::isfinite(kappa[e])) return set_err(ASMG_EINVAL, "kappa must be finite and > 0");
  ASMG_TRY({
    h.kappa.assign(kappa, kappa + h.ne);
    assemble_fine_values(h);
    assemble_aux_values(h);
    build_coarse(h);
    build_near_boundary(h);
    if (H->dev) device_update_values(H->dev, h);
    return ASMG_OK;
  })
}

int asmg_set_precision(asmg_handle H, int precision) {
  if (!H || (precision != ASMG_PREC_FP64 && precision != ASMG_PREC_MIXED)) return set_err(ASMG_EINVAL, "bad argument");
  H->h.opt.precision = precision;
  if (H->dev) device_set_precision(H->dev, precision);
  if (H->bdev) batch_device_set_precision(H->bdev, precision);
  return ASMG_OK;
}

int asmg_num_dofs(asmg_handle H, int64_t *n) {
  if (!H || !n) return set_err(ASMG_EINVAL, "null argument");
  if (H->is_batch()) {
    int64_t t = 0;
    for (auto &hp : H->batch) t += hp->n();
    *n = t;
    return ASMG_OK;
  }
  *n = H->h.n();
  return ASMG_OK;
}

int asmg_dof_vertex(asmg_handle H, int32_t *map) {
  if (!H || !map) return set_err(ASMG_EINVAL, "null argument");
  for (int64_t i = 0; i < H->h.n(); ++i) map[i] = (int32_t)H->h.dofs[i];
  return ASMG_OK;
}

static int need_dev(asmg_handle H) {
  if (!H) return set_err(ASMG_EINVAL, "null handle");
  if (H->is_batch()) return set_err(ASMG_EINVAL, "batch handle: use the batch entry points");
  if (!H->dev) return set_err(ASMG_EDEVICE, "host-only handle (options.device = -1)");
  return ASMG_OK;
}

// vectors of n = 0 unknowns (every vertex Dirichlet) may be null
static bool bad_vec(asmg_handle H, const void *p) { return !p && H->h.n() > 0; }

int asmg_solve(asmg_handle H, const double *f, double tol, double *u, int *iterations, double *true_rel) {
  if (int r = need_dev(H)) return r;
  if (bad_vec(H, f) || bad_vec(H, u)) return set_err(ASMG_EINVAL, "null vector");
  if (!(tol > 0) || !std::isfinite(tol)) return set_err(ASMG_EINVAL, "tol must be > 0");
  ASMG_TRY({
    int rc = device_solve_host(H->dev, f, tol, u, iterations, true_rel);
    if (rc) set_err(rc, "solve did not converge or broke down");
    return rc;
  })
}

int asmg_solve_device(asmg_handle H, const double *d_f, double tol, double *d_u, int *iterations, double *true_rel,
                      void *stream) {
  if (int r = need_dev(H)) return r;
  if (bad_vec(H, d_f) || bad_vec(H, d_u)) return set_err(ASMG_EINVAL, "null vector");
  if (!(tol > 0) || !std::isfinite(tol)) return set_err(ASMG_EINVAL, "tol must be > 0");
  ASMG_TRY({
    int rc = device_solve(H->dev, d_f, tol, d_u, iterations, true_rel, stream);
    if (rc) set_err(rc, "solve did not converge or broke down");
    return rc;
  })
}

int asmg_solve_device_noalloc(asmg_handle H, const double *d_f, double tol, double *d_u, int *iterations,
                              double *true_rel, void *stream) {
  if (int r = need_dev(H)) return r;
  if (bad_vec(H, d_f) || bad_vec(H, d_u)) return set_err(ASMG_EINVAL, "null vector");
  if (!(tol > 0) || !std::isfinite(tol)) return set_err(ASMG_EINVAL, "tol must be > 0");
  ASMG_TRY({
    int rc = device_solve_noalloc(H->dev, d_f, tol, d_u, iterations, true_rel, stream);
    if (rc) set_err(rc, "solve did not converge or broke down");
    return rc;
  })
}

int asmg_apply_preconditioner_device(asmg_handle H, const double *d_r, double *d_z, int precision, void *stream) {
  if (int r = need_dev(H)) return r;
  if (bad_vec(H, d_r) || bad_vec(H, d_z) || (precision != ASMG_PREC_FP64 && precision != ASMG_PREC_MIXED))
    return set_err(ASMG_EINVAL, "bad argument");
  ASMG_TRY({ return device_apply_B(H->dev, d_r, d_z, precision, stream); })
}

int asmg_set_coefficient_device(asmg_handle H, const double *d_kappa, void *stream) {
  if (int r = need_dev(H)) return r;
  if (!d_kappa) return set_err(ASMG_EINVAL, "null coefficient");
  ASMG_TRY({ return device_set_coefficient(H->dev, H->h, d_kappa, stream); })
}

int asmg_set_log_coefficient_device(asmg_handle H, const double *d_m, void *stream) {
  if (int r = need_dev(H)) return r;
  if (!d_m) return set_err(ASMG_EINVAL, "null log-coefficient");
  ASMG_TRY({ return device_set_log_coefficient(H->dev, H->h, d_m, stream); })
}

int asmg_matvec_device(asmg_handle H, const double *d_x, double *d_y, void *stream) {
  if (int r = need_dev(H)) return r;
  if (bad_vec(H, d_x) || bad_vec(H, d_y)) return set_err(ASMG_EINVAL, "null vector");
  ASMG_TRY({ return device_matvec(H->dev, d_x, d_y, stream); })
}

int asmg_element_gradient_device(asmg_handle H, const double *d_u, const double *d_lam, double *d_g, void *stream) {
  if (int r = need_dev(H)) return r;
  if (bad_vec(H, d_u) || bad_vec(H, d_lam) || !d_g) return set_err(ASMG_EINVAL, "null vector");
  ASMG_TRY({ return device_element_gradient(H->dev, d_u, d_lam, d_g, 1.0, stream); })
}

int asmg_adjoint_gradient_device(asmg_handle H, const double *d_u, const double *d_lam, double *d_g, void *stream) {
  if (int r = need_dev(H)) return r;
  if (bad_vec(H, d_u) || bad_vec(H, d_lam) || !d_g) return set_err(ASMG_EINVAL, "null vector");
  ASMG_TRY({ return device_element_gradient(H->dev, d_u, d_lam, d_g, -1.0, stream); })
}

int asmg_time_kernel(asmg_handle H, int which, int reps, int precision, void *stream, double *ms, double *bytes) {
  if (int r = need_dev(H)) return r;
  if (which < 0 || which > 7 || reps < 1 || !ms || !bytes) return set_err(ASMG_EINVAL, "bad argument");
  ASMG_TRY({ return device_time_kernel(H->dev, which, reps, precision, stream, ms, bytes); })
}


static int check_options(const asmg_options &o) {
  if (o.nu_aux < 1 || o.nu_fine < 1 || o.max_iter < 1 || o.coarse_max_dofs < 1 || o.coarse_max_dofs > 8192 ||
      (o.precision != ASMG_PREC_FP64 && o.precision != ASMG_PREC_MIXED) || o.n_min < 0 || o.colouring < 0 ||
      o.colouring > 2 || o.domain < 0 || o.domain > 1 || o.red_blocks < 0 || o.red_blocks > 2048)
    return set_err(ASMG_EINVAL, "invalid options");
  if (o.smoothing != 0) return set_err(ASMG_EINVAL, "local smoothing is available on single-mesh handles only");
  if (o.nested != 0) return set_err(ASMG_EINVAL, "the nested iteration is available on single-mesh handles only");
  if (o.setup_device != 0) return set_err(ASMG_EINVAL, "the device tree build is available on single-mesh handles only");
  if (o.nb_layers != 0) return set_err(ASMG_EINVAL, "the near-boundary correction is available on single-mesh handles only");
  return ASMG_OK;
}

int asmg_setup_batch(int n_meshes, int dim, const int64_t *vert_off, const double *coords, const int64_t *elem_off,
                     const int32_t *elems, const double *kappa, const asmg_options *opt, asmg_handle *out) {
  if (!out) return set_err(ASMG_EINVAL, "null output handle");
  *out = nullptr;
  if (n_meshes < 1 || (dim != 2 && dim != 3) || !vert_off || !coords || !elem_off || !elems || !kappa)
    return set_err(ASMG_EINVAL, "bad batch arguments");
  if (opt && opt->domain >= 1 && dim != 2) return set_err(ASMG_EINVAL, "general domains are 2-D");
  asmg_options o;
  asmg_default_options(&o);
  if (opt) o = *opt;
  if (int rc = check_options(o)) return rc;
  for (int m = 0; m < n_meshes; ++m) {
    const int64_t nv = vert_off[m + 1] - vert_off[m], ne = elem_off[m + 1] - elem_off[m];
    if (nv <= 0 || ne <= 0) return set_err(ASMG_EINVAL, "empty mesh in batch");
    for (int64_t i = vert_off[m] * dim; i < vert_off[m + 1] * dim; ++i)
      if (!std::isfinite(coords[i])) return set_err(ASMG_EINVAL, "non-finite coordinate");
    for (int64_t i = elem_off[m] * (dim + 1); i < elem_off[m + 1] * (dim + 1); ++i)
      if (elems[i] < 0 || elems[i] >= nv) return set_err(ASMG_EINVAL, "element vertex id out of range");
    for (int64_t e = elem_off[m]; e < elem_off[m + 1]; ++e)
      if (!(kappa[e] > 0) || !std::isfinite(kappa[e])) return set_err(ASMG_EINVAL, "kappa must be finite and > 0");
  }
  ASMG_TRY({
    std::unique_ptr<asmg_s> HP(new asmg_s());
    HP->batch.resize(n_meshes);
    // largest meshes first, so that the last ones to finish are small
    std::vector<int> order(n_meshes);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      return elem_off[a + 1] - elem_off[a] > elem_off[b + 1] - elem_off[b];
    });
    std::atomic<int> next{0};
    std::vector<AsmgError> errs;
    std::mutex mu;
    auto work = [&]() {
      while (true) {
        const int i = next.fetch_add(1);
        if (i >= n_meshes) return;
        const int m = order[i];
        try {
          auto h = std::make_unique<Hierarchy>();
          h->d = dim;
          h->nv = vert_off[m + 1] - vert_off[m];
          h->ne = elem_off[m + 1] - elem_off[m];
          h->opt = o;
          h->threads = 1;  // the meshes themselves run on parallel threads
          h->coords.assign(coords + vert_off[m] * dim, coords + vert_off[m + 1] * dim);
          h->elems.assign(elems + elem_off[m] * (dim + 1), elems + elem_off[m + 1] * (dim + 1));
          h->kappa.assign(kappa + elem_off[m], kappa + elem_off[m + 1]);
          build_fine(*h);
          build_tree(*h);
          if (o.domain >= 1) build_domain(*h);
          build_levels(*h);
          build_transfer(*h);
          build_colourings(*h);
          build_coarse(*h);
          HP->batch[m] = std::move(h);
        } catch (const AsmgError &e) {
          std::lock_guard<std::mutex> g(mu);
          errs.push_back(AsmgError{e.code, "mesh " + std::to_string(m) + ": " + e.msg});
        } catch (const std::bad_alloc &) {
          std::lock_guard<std::mutex> g(mu);
          errs.push_back(AsmgError{ASMG_ENOMEM, "host allocation failed"});
        }
      }
    };
    const bool tm = std::getenv("ASMG_SETUP_TIMING") != nullptr;
    auto t0 = std::chrono::steady_clock::now();
    const int nt = std::max(1, std::min<int>(n_meshes, (int)std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t) th.emplace_back(work);
    for (auto &t : th) t.join();
    if (!errs.empty()) throw errs.front();
    auto t1 = std::chrono::steady_clock::now();
    if (tm)
      std::fprintf(stderr, "[asmg batch setup] meshes (%d threads) %8.3f s\n", nt,
                   std::chrono::duration<double>(t1 - t0).count());
    HP->h.d = dim;
    HP->h.opt = o;
    if (o.device >= 0) HP->bdev = batch_device_create(HP->batch, o.device);
    if (tm)
      std::fprintf(stderr, "[asmg batch setup] device layout %8.3f s\n",
                   std::chrono::duration<double>(std::chrono::steady_clock::now() - t1).count());
    *out = HP.release();
    return ASMG_OK;
  })
}

int asmg_solve_batch_device(asmg_handle H, int n_rhs, const double *d_F, double tol, double *d_U, int *iterations,
                            double *true_rel, void *stream) {
  if (!H || !H->is_batch()) return set_err(ASMG_EINVAL, "not a batch handle");
  if (!H->bdev) return set_err(ASMG_EDEVICE, "host-only handle (options.device = -1)");
  if (!d_F || !d_U || (n_rhs != 1 && n_rhs != 2 && n_rhs != 4)) return set_err(ASMG_EINVAL, "bad argument");
  if (!(tol > 0) || !std::isfinite(tol)) return set_err(ASMG_EINVAL, "tol must be > 0");
  ASMG_TRY({
    int rc = batch_device_solve(H->bdev, n_rhs, d_F, tol, d_U, iterations, true_rel, stream);
    if (rc) set_err(rc, "a system did not converge or broke down");
    return rc;
  })
}

int asmg_time_batch(asmg_handle H, int n_rhs, int reps, int precision, void *stream, double *ms, double *bytes) {
  if (!H || !H->is_batch() || !H->bdev) return set_err(ASMG_EINVAL, "not a device batch handle");
  if ((n_rhs != 1 && n_rhs != 2 && n_rhs != 4) || reps < 1 || !ms || !bytes) return set_err(ASMG_EINVAL, "bad argument");
  ASMG_TRY({ return batch_device_time(H->bdev, n_rhs, reps, precision, stream, ms, bytes); })
}

int asmg_time_batch_kernel(asmg_handle H, int which, int n_rhs, int reps, int precision, void *stream, double *ms,
                           double *bytes) {
  if (!H || !H->is_batch() || !H->bdev) return set_err(ASMG_EINVAL, "not a device batch handle");
  if (which < 0 || which > 1 || (n_rhs != 1 && n_rhs != 2 && n_rhs != 4) || reps < 1 || !ms || !bytes ||
      (precision != ASMG_PREC_FP64 && precision != ASMG_PREC_MIXED))
    return set_err(ASMG_EINVAL, "bad argument");
  ASMG_TRY({ return batch_device_time_kernel(H->bdev, which, n_rhs, reps, precision, stream, ms, bytes); })
}

void asmg_destroy(asmg_handle H) {
  if (!H) return;
  if (H->dev) device_destroy(H->dev);
  if (H->bdev) batch_device_destroy(H->bdev);
  delete H;
}

int asmg_export(asmg_handle H, const char *name_c, int level, void *buf, int64_t *count) {
  if (!H || !name_c || !count) return set_err(ASMG_EINVAL, "null argument");
  Hierarchy &h = H->h;
  const std::string name(name_c);
  ASMG_TRY({
    if (H->is_batch()) {
      if (name == "batch_shapes") {  // level = NR + 8 * precision
        if (!H->bdev) return set_err(ASMG_EINVAL, "host-only batch handle");
        return put(batch_tuned_shapes(H->bdev, level % 8, level / 8), buf, count);
      }
      if (name == "batch_tune_times") {  // level = NR + 8 * precision
        if (!H->bdev) return set_err(ASMG_EINVAL, "host-only batch handle");
        return put(batch_tune_times(H->bdev, level % 8, level / 8), buf, count);
      }
      if (name == "batch_n" || name == "batch_J" || name == "batch_lc") {
        std::vector<int64_t> v;
        for (auto &hp : H->batch) v.push_back(name == "batch_n" ? hp->n() : name == "batch_J" ? hp->J : hp->lc);
        return put(v, buf, count);
      }
      return set_err(ASMG_EINVAL, "batch handle exports: batch_n, batch_J, batch_lc, batch_shapes, batch_tune_times");
    }
    if (name == "info") {
      std::vector<int64_t> v(16, 0);
      v[0] = h.d;
      v[1] = h.n();
      v[2] = h.J;
      v[3] = h.lc;
      v[4] = h.J - h.lc + 1;
      v[5] = h.A.nnz();
      v[6] = h.Pi.nnz();
      v[7] = (int64_t)h.R.size();
      v[8] = (int64_t)h.leaves.size();
      v[9] = h.colour_fine.empty() ? 0 : *std::max_element(h.colour_fine.begin(), h.colour_fine.end()) + 1;
      v[10] = h.ne;
      v[11] = h.nv;
      return put(v, buf, count);
    }
    if (name == "refined") return put(boxes_tuples(h, std::vector<BoxCode>(h.R.begin(), h.R.end())), buf, count);
    if (name == "leaves") return put(boxes_tuples(h, h.leaves), buf, count);
    if (name == "keys") return put(h.keys, buf, count);
    if (name == "leaf_kappa") {  // kappa~ per leaf, in the order of "leaves"
      std::vector<double> v;
      for (BoxCode b : h.leaves) v.push_back(h.leaf_kappa.at(b));
      return put(v, buf, count);
    }
    if (name == "setup_seconds") return put(h.setup_seconds, buf, count);
    if (name == "device_stages") return put(std::vector<int64_t>{h.device_stages}, buf, count);
    if (name == "level_n") {
      std::vector<int64_t> v(h.J);
      for (int l = 1; l <= h.J; ++l) v[l - 1] = level_mesh(h, l).n();
      return put(v, buf, count);
    }
    if (name == "colour_fine") {
      std::vector<int64_t> c(h.colour_fine.begin(), h.colour_fine.end());
      return put(c, buf, count);
    }
    if (name.rfind("level_", 0) == 0 || name == "colour_aux" || name == "local_set" || name.rfind("Al_", 0) == 0 ||
        name.rfind("P_", 0) == 0) {
      if (level < 1 || level > h.J) return set_err(ASMG_EINVAL, "level out of range");
    }
    if (name == "level_verts") return put(level_mesh(h, level).verts, buf, count);
    if (name == "level_simp") return put(level_mesh(h, level).simp, buf, count);
    if (name == "level_dofs") return put(level_mesh(h, level).dof_vert, buf, count);
    if (name == "level_kept") {
      const LevelMesh &lm = level_mesh(h, level);
      std::vector<int64_t> k(lm.simp_box.size(), 1);
      if (!lm.kept.empty())
        for (size_t i = 0; i < k.size(); ++i) k[i] = lm.kept[i];
      return put(k, buf, count);
    }
    if (name == "nb_set") {  // level: the near-boundary set, ascending unknown ids
      auto it = h.nb.find(level);
      std::vector<int64_t> v;
      if (it != h.nb.end()) {
        v = it->second.J;
        std::sort(v.begin(), v.end());
      }
      return put(v, buf, count);
    }
    if (name == "nb_info") {  // level: |J|, dense (1) or decomposed (0), interior size, pieces
      auto it = h.nb.find(level);
      std::vector<int64_t> v(4, 0);
      if (it != h.nb.end()) {
        v[0] = (int64_t)it->second.J.size();
        v[1] = it->second.dense ? 1 : 0;
        v[2] = it->second.nI;
        v[3] = it->second.poff.empty() ? 0 : (int64_t)it->second.poff.size() - 1;
      }
      return put(v, buf, count);
    }
    if (name == "coarse_inv") return put(h.coarse_inv, buf, count);
    if (name == "solve_stats") {
      if (!H->dev) return set_err(ASMG_EINVAL, "host-only handle");
      std::vector<int64_t> v = {device_last_iterations(H->dev), device_restarts(H->dev)};
      return put(v, buf, count);
    }
    if (name == "tune_times") {  // level = precision
      if (!H->dev) return set_err(ASMG_EINVAL, "host-only handle");
      return put(device_tune_times(H->dev, level), buf, count);
    }
    if (name == "tuned_shapes") {  // level = precision
      if (!H->dev) return set_err(ASMG_EINVAL, "host-only handle");
      return put(device_tuned_shapes(H->dev, level), buf, count);
    }
    if (name == "local_set") {
      auto it = h.local_set.find(level);
      if (it == h.local_set.end()) return set_err(ASMG_EINVAL, "no smoothed level there");
      std::vector<int64_t> c(it->second.begin(), it->second.end());
      return put(c, buf, count);
    }
    if (name == "colour_aux") {
      auto it = h.colour_aux.find(level);
      if (it == h.colour_aux.end()) return set_err(ASMG_EINVAL, "no colouring on that level");
      std::vector<int64_t> c(it->second.begin(), it->second.end());
      return put(c, buf, count);
    }
    auto us = name.find('_');
    if (us != std::string::npos) {
      const std::string mat = name.substr(0, us), part = name.substr(us + 1);
      if (part == "rowptr" || part == "col" || part == "val") {
        if (mat == "A") return put_csr(h.A, part, buf, count);
        if (mat == "Pi") return put_csr(h.Pi, part, buf, count);
        if (mat == "Al") {
          auto it = h.Al.find(level);
          if (it == h.Al.end()) return set_err(ASMG_EINVAL, "no A_l on that level");
          return put_csr(it->second, part, buf, count);
        }
        if (mat == "P") {
          auto it = h.P.find(level);
          if (it == h.P.end()) return set_err(ASMG_EINVAL, "no P_l on that level");
          return put_csr(it->second, part, buf, count);
        }
      }
    }
    return set_err(ASMG_EINVAL, "unknown export name: " + name);
  })
}

}  // extern "C"
