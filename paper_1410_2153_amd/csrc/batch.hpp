// Batched engine (batch.hip): many meshes x up to 4 right-hand sides per launch sequence.
#pragma once

#include <cstdint>
#include <memory>
#include <vector>

#include "setup.hpp"

namespace asmg {

struct BatchDevice;

BatchDevice *batch_device_create(std::vector<std::unique_ptr<Hierarchy>> &H, int ordinal);
void batch_device_destroy(BatchDevice *dv);
void batch_device_set_precision(BatchDevice *dv, int precision);
int batch_device_solve(BatchDevice *dv, int n_rhs, const double *d_F, double tol, double *d_U, int *iters,
                       double *true_rel, void *stream);
int batch_device_time(BatchDevice *dv, int n_rhs, int reps, int precision, void *stream, double *ms, double *bytes);
// which 0: one B_co application as a hipGraph, median over `reps` replays, with its algorithmic
// bytes; which 1: every Gauss-Seidel colour pass inside `reps` applications timed per launch,
// mean ms and mean algorithmic bytes per launch
int batch_device_time_kernel(BatchDevice *dv, int which, int n_rhs, int reps, int precision, void *stream, double *ms,
                             double *bytes);
int64_t batch_n_total(BatchDevice *dv);
// launch shapes picked by the autotuner for (NR, precision): threads per block, XCD order and
// kernel variant of every slice-kernel launch site, flattened triples (empty before the first solve)
std::vector<int64_t> batch_tuned_shapes(BatchDevice *dv, int nr, int precision);
// the autotuner's best time (ms) of every candidate at every launch site, site-major (-1 = not timed)
std::vector<double> batch_tune_times(BatchDevice *dv, int nr, int precision);

}  // namespace asmg
