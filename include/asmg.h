/*
 * asmg.h -- C ABI of the MI355X auxiliary-space multigrid (ASMG) PCG solver.
 *
 * Method: Grasedyck, Wang, Xu, "A Nearly Optimal Multigrid Method for General
 * Unstructured Grids" (arXiv:1410.2153).
 *   - problem: A u = f, A the P1 stiffness matrix of -div(kappa grad u) with
 *     homogeneous Dirichlet data (Section 2, eq. (1)-(2));
 *   - setup: cluster tree of element barycenters (Section 3.1), closure
 *     (Section 3.2), nested conforming auxiliary grids (Section 3.3), Dirichlet
 *     auxiliary grids (Section 3.4), auxiliary matrices A_l, prolongations P_l and
 *     the Scott-Zhang transfer Pi (Section 4.1);
 *   - solve: CG (Section 5.2) preconditioned by one multiplicative auxiliary
 *     space cycle (Algorithm 1): Gauss-Seidel on the original grid, transfer
 *     Pi^T, a V-cycle (Algorithm 2) down the auxiliary hierarchy with a dense
 *     Cholesky solve at the bottom, transfer Pi, Gauss-Seidel back.
 *
 * Conventions
 *   - All functions return 0 on success or a negative ASMG_E* code; they never
 *     throw. asmg_last_error() returns a thread-local message for the last
 *     failure on the calling thread.
 *   - The caller owns every input buffer; setup copies what it needs and keeps
 *     no caller pointer. Outputs go to caller-allocated buffers.
 *   - Host-pointer calls (asmg_solve) copy through the handle's staging buffers.
 *     *_device calls take device pointers and are ordered on the caller's HIP
 *     stream (passed as void*; NULL = the null stream); they return once the
 *     results are in device memory.
 *   - A handle owns all device memory it uses. It is not thread-safe; distinct
 *     handles are independent.
 *   - Unknowns ("DOFs") are the non-Dirichlet vertices in ascending vertex id.
 *     Vectors f and u have one entry per unknown in that order.
 */
#ifndef ASMG_H
#define ASMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ASMG_OK 0
#define ASMG_EINVAL (-1)    /* invalid argument (shape, index range, kappa <= 0 or NaN, tol <= 0) */
#define ASMG_ENOCONV (-2)   /* max_iter reached; u holds the last iterate */
#define ASMG_ENOTSPD (-3)   /* p.Ap <= 0 or r.z <= 0 during CG */
#define ASMG_ENAN (-4)      /* a NaN/Inf appeared in the iteration */
#define ASMG_EDEVICE (-5)   /* HIP runtime error, or a device call on a host-only handle */
#define ASMG_ENOMEM (-6)    /* host or device allocation failed */

#define ASMG_PREC_FP64 0    /* whole solve in FP64 */
#define ASMG_PREC_MIXED 1   /* B_co (smoothers, transfers, aux V-cycle) in FP32 inside FP64 CG */

typedef struct asmg_s *asmg_handle;

typedef struct {
  int n_min;           /* cluster leaf size; 0 = 3 in 2-D (Section 3.1), 7 in 3-D */
  int nu_aux;          /* Gauss-Seidel sweeps before and after the coarse correction (Section 5.1: 2) */
  int nu_fine;         /* fine Gauss-Seidel sweeps per side of Algorithm 1 (1) */
  int coarse_max_dofs; /* the V-cycle bottom is the finest level with at most this many unknowns (1024) */
  int max_iter;        /* PCG iteration cap (1000) */
  int precision;       /* ASMG_PREC_FP64 or ASMG_PREC_MIXED */
  uint32_t colour_seed;/* seed of the hash colour order (colouring = 1) */
  int device;          /* HIP device ordinal; -1 = host-only handle (setup and exports, no solve) */
  int check_every;     /* PCG iterations between host reads of the device convergence flag (0 = auto) */
  int colouring;       /* Gauss-Seidel colour order (greedy colouring of each matrix's pattern):
                          0 = greedy in unknown order,
                          1 = greedy in descending (fmix32(i ^ colour_seed), i) (Jones-Plassmann order),
                          2 = greedy in smallest-last order (Matula-Beck; at most degeneracy + 1
                              colours; default) */
  int smoothing;       /* auxiliary-level smoothing: 0 = every unknown of the level (Algorithm 2,
                          default); 1 = local, only the unknowns of N~_l, the index set of the
                          decomposition of Section 4.3 (new on level l, or with a basis function
                          that changed from level l-1). Single-mesh handles only. */
  int domain;          /* Dirichlet auxiliary grids (Section 3.4): 0 = every simplex of the root box
                          (default; the domain is the mesh's bounding box); 1 = only the simplices
                          inside the mesh's own domain, the closed union of its triangles (2-D,
                          any polygon, holes allowed); with a null `dirichlet` the Dirichlet
                          vertices are then the mesh's boundary vertices. 2 = mixed Dirichlet/
                          Neumann grids (remark of Section 3.5, 2-D): the simplices that meet the
                          domain and not its Dirichlet boundary Gamma_D (boundary edges whose two
                          vertices are Dirichlet); essential conditions at the vertices of
                          simplices meeting Gamma_D, natural ones elsewhere. Without the
                          near-boundary correction of Algorithm 3. */
  int autotune;        /* 1 = at the first solve in a precision, time the candidate launch shapes
                          of every V-cycle slice kernel (threads per block, block order, kernel
                          variant: one slice per wave, or a grid-stride loop over the slices that
                          loads the next slice's header early) and keep the fastest (default);
                          0 = fixed 256-thread blocks in XCD order, one slice per wave. Results do
                          not depend on it. */
  int nested;          /* initial guess of PCG: 0 = u_0 = 0 (default); k in 1..16 = nested iteration
                          over the auxiliary levels (Section 5.2): g_J = Pi^T f, g_(l-1) = P_l^T g_l,
                          e = A_(l_c)^-1 g_(l_c) at the bottom, then on each finer level
                          e_l = P_l e_(l-1) and k V-cycles (Algorithm 2) on A_l e = g_l, in the
                          V-cycle's precision; u_0 = Pi e_J. Single-mesh handles with whole-level
                          smoothing (smoothing = 0) only. */
  int setup_device;    /* 1 = build on the HIP device: the fine matrix (Section 2), the cluster
                          tree (Sections 3.1-3.2: root box, keys, Morton sort, refinement by
                          cluster size, closure, leaves, kappa~), the level meshes (Section 3.3;
                          root-box grids whose vertex keys fit 64 bits, (J+1) dim <= 64), the
                          level matrices A_l, the prolongations P_l and the Scott-Zhang
                          transfer Pi (Section 4.1), and with
                          colouring = 1 the multicolour orderings (Jones-Plassmann rounds, the
                          same colouring as the host's greedy one in the hash order); every
                          result identical to the host setup's. The other setup steps (and the
                          level meshes of general domains) stay on the host. Needs device >= 0;
                          single-mesh handles. 0 = host (default). */
  int red_blocks;      /* cap on the blocks of the PCG reduction kernels (dot products, residual
                          norms, q = A p), 1..2048; 0 = 2048 (default). Beyond the cap the kernels
                          loop over their rows (grid-stride). Results do not depend on it beyond
                          the summation order of the dot products. Single-mesh handles. */
  int nb_layers;       /* near-boundary correction (Section 3.5, Algorithm 3): j > 0 = on every
                          auxiliary level above the bottom, an exact solve on the unknowns within j
                          layers of simplices of the level grid's boundary, before and after the
                          coarse-grid correction (so that the V-cycle stays symmetric); 0 = off
                          (default). Single-mesh handles with whole-level smoothing. */
} asmg_options;

/* Fill *opt with the defaults listed above. */
int asmg_default_options(asmg_options *opt);

/*
 * Build the hierarchy for one mesh (Sections 3.1-3.4, 4.1) and upload it.
 *   dim          2 (triangles) or 3 (tetrahedra)
 *   coords       n_vertices * dim doubles, row-major (vertex-major)
 *   elems        n_elements * (dim+1) int32, 0-based vertex ids; any orientation;
 *                a zero-volume element is an error
 *   kappa        n_elements doubles, finite and > 0 (piecewise constant coefficient)
 *   dirichlet    n_vertices bytes (nonzero = Dirichlet vertex) or NULL: the
 *                vertices with a coordinate equal to the bounding-box min or max
 *   opt          options or NULL for the defaults
 *   out          receives the handle (NULL on failure)
 * The auxiliary Dirichlet grids cover the root box, so the domain is expected
 * to be the bounding box (square/cube), as in the paper's test problem.
 * With the environment variable ASMG_SETUP_TIMING set, the time of each setup
 * phase is printed on stderr (also asmg_export("setup_seconds")).
 */
int asmg_setup(int dim, int64_t n_vertices, const double *coords, int64_t n_elements,
               const int32_t *elems, const double *kappa, const uint8_t *dirichlet,
               const asmg_options *opt, asmg_handle *out);

/* Replace kappa (n_elements, finite, > 0) keeping the tree, grids and patterns:
 * re-assembles A, A_l and the coarse inverse (Section 4.1), uploads values. */
int asmg_update_coefficient(asmg_handle h, const double *kappa);

/*
 * Replace the coefficient of the operator A on the original grid from a device
 * array d_kappa (n_elements doubles, finite and > 0, not checked) without any
 * host work. A is linear in kappa (Section 2, eq. (2)): every stored entry is
 * re-summed from fixed per-element contributions on the device, in element
 * order. The auxiliary hierarchy (A_l, bottom inverse) keeps the coefficient of
 * the last asmg_setup / asmg_update_coefficient. The preconditioner stays SPD
 * (its Gauss-Seidel part uses the new A). Later solves are exact for the new A
 * to the requested tolerance; only the iteration count may change. Host-side
 * exports of A are not updated. Stream-ordered on `stream`. The per-entry element
 * lists this needs are built at the first call (host work proportional to the
 * mesh, then uploaded), not at setup.
 */
int asmg_set_coefficient_device(asmg_handle h, const double *d_kappa, void *stream);

/*
 * As asmg_set_coefficient_device with kappa_e = exp(m_e) computed on the device from a device
 * array d_m of n_elements per-element log-coefficients (finite, not checked). This is the
 * parametrisation of the adjoint gradient below.
 */
int asmg_set_log_coefficient_device(asmg_handle h, const double *d_m, void *stream);

/* Switch the precision of later solves (ASMG_PREC_FP64 or ASMG_PREC_MIXED); both
 * value copies are resident after setup, so this only changes which kernels run. */
int asmg_set_precision(asmg_handle h, int precision);

/* Number of unknowns, and the vertex id of each unknown (n int32). */
int asmg_num_dofs(asmg_handle h, int64_t *n);
int asmg_dof_vertex(asmg_handle h, int32_t *map);

/*
 * PCG solve from u_0 = 0 (or the nested iteration's guess, asmg_options.nested) until
 * ||f - A u||_2 <= tol ||f||_2 (recursively updated residual). The true residual is
 * recomputed in FP64 at exit; while it is above tol, CG restarts from it, at most 3 times
 * (then the solve returns 0 with *true_rel_residual > tol); a restart needed with the
 * iteration budget spent returns ASMG_ENOCONV. A guess that already meets the rule returns
 * it after 0 iterations.
 *   f, u                 n doubles (host pointers)
 *   iterations           number of products with A (may be NULL)
 *   true_rel_residual    ||f - A u|| / ||f|| recomputed at exit (may be NULL)
 * f = 0 returns u = 0 and 0 iterations. Returns ASMG_ENOCONV if max_iter is hit. A mesh with
 * no unknown (every vertex Dirichlet, n = 0) returns at once with 0 iterations; its vector
 * arguments, here and in the other single-mesh vector entry points, may then be NULL.
 */
int asmg_solve(asmg_handle h, const double *f, double tol, double *u, int *iterations,
               double *true_rel_residual);

/* As asmg_solve with device pointers d_f, d_u (n doubles each) on `stream`. */
int asmg_solve_device(asmg_handle h, const double *d_f, double tol, double *d_u, int *iterations,
                      double *true_rel_residual, void *stream);

/*
 * As asmg_solve_device, for callers that cannot allocate (serving loops, harnesses that forbid
 * allocation): the call allocates nothing, host or device, and calls no allocating routine.
 * The PCG control block and the reduction partials live in a static per-GPU scratch array of
 * 16640 bytes (256 for the control block, 8 per reduction block up to 2048) held by the library
 * until the process ends; every handle's reduction grid fits it (a larger one would be rejected
 * with ASMG_EINVAL). The iteration runs as eager kernel launches (no graph is built) and the
 * launch-shape autotuner never runs here: the shapes tuned by earlier asmg_solve_device calls on
 * the handle are used, or the defaults. Results equal asmg_solve_device's bit for bit. Calls on
 * one GPU share that GPU's scratch: calls that overlap on one GPU (from several threads, or on
 * streams that run concurrently) race and are not allowed; calls on different GPUs are
 * independent. The handle's work vectors are used as by asmg_solve_device.
 */
int asmg_solve_device_noalloc(asmg_handle h, const double *d_f, double tol, double *d_u, int *iterations,
                              double *true_rel_residual, void *stream);

/* z = B_co r (Algorithm 1 with u_0 = 0): one preconditioner application on
 * device vectors in unknown order; precision as in asmg_options. */
int asmg_apply_preconditioner_device(asmg_handle h, const double *d_r, double *d_z, int precision,
                                     void *stream);

/* y = A x on device vectors in unknown order (FP64; Section 2, eq. (2)). */
int asmg_matvec_device(asmg_handle h, const double *d_x, double *d_y, void *stream);

/*
 * Per-element derivative of lam^T A u w.r.t. the log-coefficient m_e
 * (kappa_e = exp(m_e)): g_e = kappa_e lam_e^T K1_e u_e, K1_e the element
 * stiffness at kappa = 1 (Section 2). d_u, d_lam: n doubles in unknown order
 * (Dirichlet values 0); d_g: n_elements doubles. The gradient of
 * J = 1/2 ||u - u_obs||^2 with A lam = u - u_obs is -g.
 */
int asmg_element_gradient_device(asmg_handle h, const double *d_u, const double *d_lam, double *d_g,
                                 void *stream);

/*
 * Adjoint gradient in the log-coefficients m (kappa_e = exp(m_e)) of a loss J(u) with
 * u = A(exp(m))^-1 f: given the solution u and the adjoint state lam of A lam = dJ/du (A is
 * symmetric, Section 2, so the adjoint solve is the same PCG), writes
 *   d_g[e] = dJ/dm_e = -kappa_e lam_e^T K1_e u_e
 * with the handle's current coefficient (the last asmg_set_(log_)coefficient_device, or setup).
 * d_u, d_lam: n doubles in unknown order; d_g: n_elements doubles. Stream-ordered.
 */
int asmg_adjoint_gradient_device(asmg_handle h, const double *d_u, const double *d_lam, double *d_g,
                                 void *stream);

/*
 * Kernel timing for the bandwidth report: launches kernel `which` `reps` times
 * on `stream` between two HIP events and returns the mean duration in ms and
 * the algorithmic bytes one launch moves.
 *   which: 0 = fine SpMV q = A p (FP64), 1 = fine Gauss-Seidel sweep (all colours),
 *          2 = one full B_co application (captured in a hipGraph; *ms is the median
 *          over `reps` replays, each between its own events), 3 = same as 2 in the
 *          precision set at setup,
 *          4 (or 5) = the Gauss-Seidel colour-pass kernel (sliced ELL): inside `reps`
 *          full B_co applications every colour pass is launched once with a pair of HIP
 *          events stamped with that launch's own start and end (hipExtLaunchKernel), so
 *          caches are as in a solve; *ms and *bytes are the mean per launch,
 *          6 = the PCG product q = A p with its partial dot products (k_cg_spmv, sliced ELL,
 *          FP64), the product the solve runs,
 *          7 = the same product with the p gathers staged in LDS (per tile of 4 slices, the
 *          distinct columns loaded once into LDS, entries addressing them by a 16-bit
 *          position; a measured alternative the solve does not use). Before timing, its
 *          result on a nonzero p is checked against mode 6's (ASMG_EDEVICE if they differ
 *          by more than 1e-14 relative). Needs at most 64 KiB of LDS per tile.
 * Algorithmic bytes count each matrix entry, row pointer and vector entry the
 * operation needs once (a colour pass: its rows, b, 1/diag, the x write, and each
 * distinct gathered x entry).
 */
int asmg_time_kernel(asmg_handle h, int which, int reps, int precision, void *stream, double *ms,
                     double *bytes);

/*
 * Export of setup objects for checking (works on host-only handles).
 * `name` selects the array, `level` the auxiliary level where relevant.
 * If buf is NULL, *count receives the number of elements; otherwise up to
 * *count elements are written. Element types per name:
 *   "info"          int64[16]: dim, n_dofs, J, lc, n_levels, nnz(A), nnz(Pi),
 *                   n_refined, n_leaves, n_colours_fine, n_elements, n_vertices
 *   "refined"       int64 (level, i_0..i_{d-1}) per refined box, sorted
 *   "leaves"        int64 (level, i_0..i_{d-1}) per leaf box, sorted
 *   "keys"          int64 per element and axis (n_elements*dim)
 *   "leaf_kappa"    double kappa~ per leaf, in the order of "leaves"
 *   "setup_seconds" double wall time of the setup phases: fine matrix, cluster tree, level
 *                   meshes, transfers, colourings, bottom inverse, device upload
 *   "device_stages" int64[1] setup stages that ran on the device (option setup_device), bits:
 *                   1 fine matrix, 2 cluster tree, 4 level meshes, 8 A_l, 16 P_l, 32 Pi,
 *                   64 colourings
 *   "level_n"       int64 number of unknowns of every level 1..J
 *   "level_verts"   int64 integer coordinates (n_verts*dim) of sigma^(level)
 *   "level_simp"    int64 vertex indices (n_simp*(dim+1)) of sigma^(level)
 *   "level_dofs"    int64 vertex index of every unknown of sigma^(level)
 *   "A_rowptr","A_col" int64, "A_val" double      fine matrix, unknown order
 *   "Al_rowptr","Al_col" int64, "Al_val" double   A_level (lc <= level <= J)
 *   "P_rowptr","P_col" int64, "P_val" double      P_level (lc < level <= J)
 *   "Pi_rowptr","Pi_col" int64, "Pi_val" double   Pi (fine unknowns x aux unknowns of level J)
 *   "colour_fine"   int64 colour of every fine unknown
 *   "colour_aux"    int64 colour of every unknown of A_level (lc < level <= J)
 *   "local_set"     int64 0/1 per unknown of level `level` (lc < level <= J): member of N~_l
 *   "level_kept"    int64 0/1 per simplex of sigma^(level): kept in the Dirichlet grid
 *   "coarse_inv"    double nc*nc: the explicit inverse of the bottom matrix A_lc (row-major),
 *                   regularised on components whose rows sum to zero (pure Neumann problems)
 *   "nb_set"        int64: near-boundary set J_{l,j} of level `level` (ascending unknown ids;
 *                   empty without the option or off the levels above the bottom)
 *   "nb_info"       int64[4] of level `level`: |J|, 1 = dense inverse / 0 = decomposed solve,
 *                   interior unknowns, pieces
 *   "solve_stats"   int64[2]: PCG iterations and restarts from the true residual of the last
 *                   solve (device handles)
 *   "tuned_shapes"  int64 (threads per block, XCD order, kernel variant) per slice-kernel launch
 *                   site of B_co chosen by the launch-shape autotuner (level = precision; device
 *                   handles, empty before the first solve in that precision); variant 0 = one
 *                   slice per wave, 1 = grid-stride loop over the slices
 *   "tune_times"    double: the autotuner's best time in ms of every candidate shape at every
 *                   launch site, site-major (-1 = not timed; level = precision)
 * Batch handles: "batch_n", "batch_J", "batch_lc" (int64 per mesh), "batch_shapes"
 * (level = n_rhs + 8 * precision): (threads per block, XCD order, kernel variant) triples chosen
 * by the launch-shape autotuner for every slice-kernel launch site of B_co, empty before the
 * first solve with that n_rhs and precision, and "batch_tune_times" (same level): the tuner's
 * best time per site and candidate, as "tune_times".
 * Returns ASMG_EINVAL for an unknown name or level.
 */
int asmg_export(asmg_handle h, const char *name, int level, void *buf, int64_t *count);

/*
 * Batched setup: n_meshes independent meshes of one dimension, concatenated.
 * Mesh m has vertices [vert_off[m], vert_off[m+1]) of `coords` (dim doubles each)
 * and elements [elem_off[m], elem_off[m+1]) of `elems` ((dim+1) int32 each, vertex
 * ids local to the mesh) and of `kappa`. Dirichlet vertices: the bounding-box
 * boundary of each mesh. Every mesh gets its own hierarchy (Sections 3-4); the
 * meshes are set up on parallel host threads. The device copy merges all meshes
 * level by level (level k = k-th auxiliary level below each mesh's finest).
 * Single-mesh entry points return ASMG_EINVAL on a batch handle; asmg_num_dofs
 * returns the total number of unknowns. Exports: "batch_n", "batch_J",
 * "batch_lc" (int64 per mesh). With ASMG_SETUP_TIMING set, the times of the
 * per-mesh setups and of the merged device layout are printed on stderr.
 */
int asmg_setup_batch(int n_meshes, int dim, const int64_t *vert_off, const double *coords,
                     const int64_t *elem_off, const int32_t *elems, const double *kappa,
                     const asmg_options *opt, asmg_handle *out);

/*
 * Batched PCG: every (mesh, right-hand side) system runs the same algorithm as
 * asmg_solve_device, all systems advancing in one launch sequence per step.
 * Each system has its own CG scalars and stops on its own ||r|| <= tol ||f||.
 *   n_rhs        1, 2 or 4
 *   d_F, d_U     device arrays laid out [mesh][rhs][unknown]: mesh m starts at
 *                n_rhs * (n_0 + ... + n_{m-1}), right-hand side r of mesh m at
 *                that offset + r * n_m
 *   iterations   n_meshes * n_rhs ints (mesh-major), may be NULL
 *   true_rel_residual  n_meshes * n_rhs doubles, may be NULL
 * Returns the first failure status over the systems (ASMG_ENOTSPD, ASMG_ENAN,
 * ASMG_ENOCONV) or 0.
 */
int asmg_solve_batch_device(asmg_handle h, int n_rhs, const double *d_F, double tol, double *d_U,
                            int *iterations, double *true_rel_residual, void *stream);

/* One batched B_co application timed with HIP events over `reps` launches on
 * `stream` (mean ms) and its algorithmic bytes. */
int asmg_time_batch(asmg_handle h, int n_rhs, int reps, int precision, void *stream, double *ms,
                    double *bytes);

/*
 * Kernel timing of the batched engine on `stream`, with algorithmic bytes (each matrix entry,
 * row index and vector entry an operation needs, once):
 *   which 0: one batched B_co application captured in a hipGraph as the solve runs it; *ms is the
 *            median over `reps` replays, *bytes the application's bytes;
 *   which 1: the Gauss-Seidel colour-pass kernel (sliced ELL over n_rhs interleaved right-hand
 *            sides): inside `reps` B_co applications every colour pass is launched once with a
 *            pair of HIP events stamped with its own start and end; *ms and *bytes are the mean
 *            per launch (a pass: its rows' matrix entries, one row index per row, b, 1/diag and
 *            the x write of its rows, and each distinct gathered x entry, n_rhs values each).
 */
int asmg_time_batch_kernel(asmg_handle h, int which, int n_rhs, int reps, int precision, void *stream, double *ms,
                           double *bytes);

/* Free the handle and all its device memory. NULL is ignored. */
void asmg_destroy(asmg_handle h);

/* Thread-local message of the last failure ("" if none). */
const char *asmg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ASMG_H */
