// Device side of the solver: uploaded hierarchy, kernels and the PCG driver (device.hip).
#pragma once

#include <vector>

#include <cstdint>

#include "setup.hpp"

namespace asmg {

struct Device;

// Upload the hierarchy (internal colour-major numbering) to device `ordinal`.
Device *device_create(Hierarchy &h, int ordinal);
// Re-upload matrix values after a coefficient update (patterns unchanged).
void device_update_values(Device *dv, Hierarchy &h);
void device_destroy(Device *dv);
void device_set_precision(Device *dv, int precision);

int device_solve(Device *dv, const double *d_f, double tol, double *d_u, int *iters, double *true_rel, void *stream);
// as device_solve, with the control block and reduction partials in the library's static
// per-device scratch: no allocation of any kind
int device_solve_noalloc(Device *dv, const double *d_f, double tol, double *d_u, int *iters, double *true_rel,
                         void *stream);
int device_apply_B(Device *dv, const double *d_r, double *d_z, int precision, void *stream);
int device_set_coefficient(Device *dv, Hierarchy &h, const double *d_kappa, void *stream);
// kappa = exp(m) on the device, then the refresh of device_set_coefficient
int device_set_log_coefficient(Device *dv, Hierarchy &h, const double *d_m, void *stream);
// restarts from the true residual in the last solve
int device_restarts(const Device *dv);
int device_last_iterations(const Device *dv);
int device_matvec(Device *dv, const double *d_x, double *d_y, void *stream);
int device_element_gradient(Device *dv, const double *d_u, const double *d_lam, double *d_g, double scale,
                            void *stream);
int device_time_kernel(Device *dv, int which, int reps, int precision, void *stream, double *ms, double *bytes);
// launch shapes picked by the autotuner for a precision: (threads per block, XCD order, kernel
// variant) per slice-kernel launch site, flattened (empty before the first solve in that precision)
std::vector<int64_t> device_tuned_shapes(Device *dv, int precision);
// the autotuner's best time (ms) of every candidate shape at every launch site, site-major
// (kNumShapes values per site; -1 where a candidate was not timed)
std::vector<double> device_tune_times(Device *dv, int precision);
// host-pointer solve through device staging buffers
int device_solve_host(Device *dv, const double *f, double tol, double *u, int *iters, double *true_rel);

}  // namespace asmg
