/*
 * mace.h -- C ABI of the MI355X partial-update MACE CT reconstruction library.
 *
 * The library computes the MAP image
 *     x* = argmin_x  sum_k 1/2 ||y_k - A_k x||^2_{Lambda_k} + h(x)
 * (Sec. II-A, eq. (MAPest) and eq. (global_obj)) by partial-update multi-agent
 * consensus equilibrium: the views are split into N agents (view subsets J_i,
 * Sec. II-A), each agent applies one ICD pass as a partial proximal update of
 *     f_i(x) = sum_{k in J_i} 1/2 ||y_k - A_k x||^2_{Lambda_k} + h(x)/N
 * (eq. (local_obj), eq. (prox_F), Algorithm 2), and the agents are tied
 * together by the consensus average G (eq. (G_operators)) and the Mann
 * iteration w <- rho (2F - I)(2G - I) w + (1 - rho) w (eq. (Mann), Algorithm 1).
 * The returned image is the mean of the agents' w (Algorithm 1, "Solution").
 *
 * Conventions
 *   - Image: nx * ny pixels, raster order s = i * nx + j (row i, column j).
 *   - Sinogram rows: r = view * n_channels + channel (view-major).
 *   - A is given in compressed sparse columns (one column per pixel), with
 *     any sparsity pattern.  Columns with at most two nonzeros per view, on
 *     adjacent channels (true whenever the channel spacing is at least the
 *     pixel width over sqrt(2), e.g. 1 mm pixels and 1 mm channels), and at
 *     most 128 views per agent fit the compact device records; any other
 *     matrix takes the general records (mace_opts.format).
 *   - Units are the caller's (e.g. A in mm, x in 1/mm).
 *   - Every int-returning call returns MACE_OK (0), a negative error code, or
 *     a positive warning; mace_last_error() describes the last failure of the
 *     calling thread.
 *   - All host pointers are read only during the call and stay owned by the
 *     caller; outputs go to caller buffers.  A mace_system owns its device
 *     memory until mace_free_system().  Calls on one mace_system must not
 *     overlap (the system holds the scan workspaces and runs every solve on
 *     one private stream); calls on different systems may run on different
 *     host threads at the same time (the library serializes its graph
 *     captures with its allocations internally).
 *   - Device-pointer variants (suffix _dev) take device addresses and a HIP
 *     stream (hipStream_t passed as void*, NULL = default stream); they
 *     wait for the work already queued on that stream, run on the system's
 *     own stream, and return after it has finished.
 */
#ifndef MACE_H
#define MACE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MACE_OK 0
#define MACE_E_ARG (-1)       /* invalid argument */
#define MACE_E_MATRIX (-2)    /* malformed or unsupported system matrix */
#define MACE_E_PARTITION (-3) /* view_to_agent is not a partition */
#define MACE_E_NOMEM (-4)     /* device or host memory exhausted */
#define MACE_E_HIP (-5)       /* HIP runtime error */
#define MACE_E_NONFINITE (-6) /* the iteration produced a non-finite residual */
#define MACE_E_CANCELLED (-7) /* a served scan was cancelled */
#define MACE_W_MAXITER 1      /* max_iters reached before tol; x_out written */

typedef struct mace_system mace_system;

typedef struct {
  int32_t nx, ny;       /* image size in pixels */
  int32_t n_views;      /* number of views N_theta */
  int32_t n_channels;   /* channels per view N_D */
} mace_geom;

/* Prior h(x) = sum over unordered 8-neighbour pairs {s,r} of b_sr rho(x_s-x_r),
 * b_sr = b_edge for edge neighbours and b_diag for diagonal ones, free image
 * boundary.  kind 0: rho(d) = d^2 / (2 sigma_x^2).  kind 1 (q-GGMRF):
 * rho(d) = |d|^p / (p sigma_x^p) / (1 + (|d| / (T sigma_x))^(p-q)), which the
 * GPU path supports for p = 2 and 1 <= q <= 2 (the ICD step uses the
 * potential's symmetric quadratic majoriser, curvature rho'(d)/d, which is
 * finite at d = 0 only for p = 2).  b_edge = b_diag = 0 selects the defaults
 * 1/(4 + 2 sqrt 2) and 1/(4 sqrt 2 + 4), which sum to 1 over the 8 neighbours. */
typedef struct {
  int32_t kind;
  double sigma_x, p, q, T;
  double b_edge, b_diag;
} mace_prior;

/* Execution options (NULL = all defaults). */
typedef struct {
  int32_t precision;      /* 0: A values FP32 (default); 1: FP16 with a per
                             (agent, pixel) FP32 scale */
  int32_t sv_size;        /* super-voxel side S in pixels: 4, 8, 16 or 32
                             (16 and 32: general format); 0 = 8 for
                             images of at least 256 x 256 pixels, else 4;
                             -1 = autotuned with rows_per_agent (see
                             mace_autotune) */
  int32_t rows_per_agent; /* concurrent super-voxels per agent; 0 = automatic
                             (about 8192 rows in total over the agents, and
                             at least a quarter of one colour's super-voxels,
                             but at most half of them -- a quarter below 256
                             per colour); 1 = sequential (one super-voxel of
                             an agent at a time: the visiting order of
                             mace_visit_order) */
  int32_t fp32_tail_iters;/* with precision 1 (> 0: the FP32 values are
                             kept too): a scan switches to the FP32 values
                             when it first meets tol with the FP16 ones, or
                             this many iterations before max_iters, which
                             ever comes first; theta2 and e = y - A X_i are
                             rebuilt with the FP32 values at the switch, and
                             the scan then runs until it meets tol again (or
                             max_iters).  Applies to mace_solve,
                             mace_solve_batch and served scans. */
  int64_t hbm_budget_bytes; /* 0 = no limit */
  int32_t refresh_every;  /* recompute e = y - A X_i every this many Mann
                             iterations to stop FP32 drift (0 = never) */
  int32_t format;         /* device record format of the matrix: 0 = the
                             compact format when the matrix and options
                             allow it, else the general one; 1 = compact
                             (sv_size 4 or 8, at most 128 views per agent,
                             at most two nonzeros per column and view, on
                             adjacent channels; FP32 or FP16 values);
                             2 = general (any sparsity pattern and view
                             count, sv_size 4, 8, 16 or 32, FP32 values) */
} mace_opts;

typedef struct {
  int32_t iters;    /* Mann iterations run */
  double residual;  /* last r_k = ||X^{k+1} - G w^k|| / ||w^k|| (FP64) */
  double equits;    /* sweeps * iters: agent-voxel updates / (N * n) */
  int32_t status;   /* MACE_OK, MACE_W_MAXITER or MACE_E_NONFINITE */
  double sweep_ms;  /* with timing on: time of the ICD sweep launches (HIP events) */
  int32_t sweep_launches; /* number of sweep launches timed */
  double iter_ms;   /* with timing on: time of all Mann iterations (HIP events) */
  int32_t fp32_tail_iters; /* precision 1 with an FP32 tail: iterations run
                              with the FP32 values after the switch */
} mace_info;

/*
 * Load (once per scanner geometry) the precomputed sparse system matrix and
 * split its views into n_agents view subsets (Sec. I: the matrix is
 * precomputed because the geometry is fixed; Sec. II-A: the partition).
 *   col_ptr[nx*ny + 1] (int64, col_ptr[0] = 0, non-decreasing),
 *   row_idx[nnz] (ascending and distinct within a column, < n_views*n_channels),
 *   val[nnz] (finite).
 *   view_to_agent[n_views]: agent of each view (NULL = interleaved, view k ->
 *   agent k mod n_agents); every agent must own at least one view (more than
 *   128 views per agent take the general records).
 * The matrix is copied and repacked on the device; *out receives the handle.
 * A super-voxel's band (its channels in every view of the agent) is staged in
 * LDS, one row of 16 lanes per (agent, super-voxel) task: workgroups hold 16,
 * 8 or 4 rows, whichever keeps the most rows of a CU's 160 KiB resident (the
 * general records go down to 2 or 1); MACE_E_ARG if even the smallest
 * workgroup does not fit 160 KiB (a smaller sv_size or more agents help).
 * Errors: MACE_E_ARG, MACE_E_MATRIX, MACE_E_PARTITION, MACE_E_NOMEM, MACE_E_HIP.
 */
int mace_load_system(const mace_geom* geom, const int64_t* col_ptr, const int32_t* row_idx,
                     const float* val, int32_t n_agents, const int32_t* view_to_agent,
                     const mace_opts* opts, mace_system** out);

/*
 * Partial-update MACE (Algorithm 1) with `sweeps` ICD passes per partial
 * update (Algorithm 2).  y and lambda: [n_views * n_channels] measurements and
 * diagonal inverse-variance weights (host).  rho in (0,1) (eq. (Mann)),
 * sigma > 0 (eq. (prox_F)).  w_init: [n_agents * nx * ny] initial w (NULL =
 * 0; the fixed point does not depend on it).  Stops after max_iters Mann
 * iterations or when r_k < tol (tol <= 0: never); x_out[nx*ny] receives the
 * consensus image mean_i w_i.  info (optional) receives the statistics.
 * Returns MACE_OK, MACE_W_MAXITER (tol > 0 not reached), MACE_E_NONFINITE
 * (the iteration diverged: its state or residual is not finite, with or
 * without tol; x_out then holds non-finite values), or another error.
 * max_iters = 0 runs no iteration: x_out = mean_i w_init (0 without it),
 * info->iters = 0 and residual 0, and MACE_W_MAXITER if tol > 0.
 */
int mace_solve(mace_system* sys, const float* y, const float* lambda, const mace_prior* prior,
               double rho, double sigma, int32_t sweeps, int32_t max_iters, double tol,
               const float* w_init, float* x_out, mace_info* info);

/*
 * Resume a solve from a checkpoint.  The state Algorithm 1 carries from one
 * Mann iteration to the next is (w, X): the agents' Mann variables and the
 * agents' partial-update states X_i, which each ICD pass starts from.
 * mace_get_state returns both after a solve; mace_solve_resume continues
 * from w0 = w, X0 = X ([n_agents * nx * ny] each, host), rebuilding every
 * agent's error sinogram e = y - A X_i, for up to max_iters further
 * iterations.  Resuming a run after k iterations reproduces the uninterrupted
 * run to FP32 rounding (the rebuilt e differs from the carried one in the
 * summation order only).  Other arguments, results and errors as mace_solve.
 */
int mace_solve_resume(mace_system* sys, const float* y, const float* lambda,
                      const mace_prior* prior, double rho, double sigma, int32_t sweeps,
                      int32_t max_iters, double tol, const float* w0, const float* X0,
                      float* x_out, mace_info* info);

/*
 * Volume reconstruction: nz slices of nx x ny pixels, each measured by the
 * system's 2-D matrix A (parallel beam: every ray lies in one slice), with
 * the 3-D prior that adds to the 8 in-plane cliques of every slice the axial
 * cliques between voxel (z, s) and (z + 1, s) with weight b_axial:
 *   h(x) = sum_z h_2D(x_z) + sum_{z,s} b_axial rho(x_{z,s} - x_{z+1,s})
 * (the MAP cost of eq. (global_obj) over the stacked volume, its prior split
 * as h / N among the agents as in eq. (local_obj)).  Each agent holds its
 * views of every slice.  Partial-update MACE (Algorithm 1, Algorithm 2) runs
 * over the nz * nx * ny voxels: the consensus, the Mann update and the
 * residual r_k are those of the stacked vectors, and all slices stop
 * together when r_k < tol.  The agents visit the super-voxels of one colour
 * in the even slices, then in the odd slices (the axial neighbours a voxel
 * reads do not change while its slice sweeps).
 * y, lambda: host, float[nz][n_views * n_channels] (slice z's sinogram in
 *   global row order); x_out: host, float[nz][nx * ny].
 * 1 <= nz <= 128; b_axial >= 0 (0: independent slices).  Either record
 * format; the system must hold FP32 matrix values (precision 0), else
 * MACE_E_ARG; other arguments, results and errors as mace_solve
 * (info->residual is the stacked r_k).  The slices occupy scan slots 0 ..
 * nz - 1: mace_get_slot_state(sys, z, ...) returns slice z's (w, X).
 */
int mace_solve_volume(mace_system* sys, int32_t nz, const float* y, const float* lambda,
                      const mace_prior* prior, double b_axial, double rho, double sigma,
                      int32_t sweeps, int32_t max_iters, double tol, float* x_out,
                      mace_info* info);

/*
 * Super-voxel groups of a volume (SV-ICD's multi-slice super-voxels, Sec. IV:
 * the slices of a group are swept together per super-voxel): with slices = G
 * > 1, mace_solve_volume takes the slices in groups of G consecutive ones;
 * one row of the sweep takes a super-voxel of one agent through the G slices
 * of its group in turn (slice z sees slice z - 1's new values of the same
 * pass), and the even / odd groups sweep in separate launches, so a group's
 * axial neighbours in the next group hold still while it runs.  G = 1
 * (default) is the even / odd slice scheme.  The fixed point does not depend
 * on G (only the visiting order changes).  slices in [1, 128]; applies to
 * later mace_solve_volume calls.
 */
int mace_set_slice_group(mace_system* sys, int32_t slices);

/*
 * Partial-update MACE with a plug-and-play prior (Algorithm 3, Sec. III):
 * the agents apply partial updates of the proximal maps of their data terms
 * alone (beta = 0, no prior), F_i(v; sqrt(N) sigma) (eq. (FG_PnP)), and the
 * consensus operator is G_H(w) = H(mean_i w_i) for every agent, with the
 * Mann iteration of eq. (Mann_PnP).  The denoiser H here is h_passes
 * applications of the 3x3 binomial smoother (1/4, 1/2, 1/4 along rows, then
 * along columns, zero outside the image): symmetric with its spectrum in
 * (0, 1), hence firmly non-expansive (the case of the lemma of Sec. III that
 * makes T_H non-expansive), and the proximal
 * map of x^T (H^-1 - I) x / 2, so the fixed point is the minimiser of
 * f(x) + x^T (H^-1 - I) x / (2 sigma^2) (Theorem 3).  w starts at 0; x_out
 * [nx*ny] receives x* = H(mean_i w_i).  The residual and stopping test are
 * those of mace_solve with G_H in place of G.  h_passes in [1, 64].
 * With no prior term in the agents, many concurrent super-voxels per agent
 * leave the agents' states jittering about the fixed point: at 512x512 with
 * 16 agents the automatic 512 rows per agent hold r near 4e-4 while x
 * converges (NRMSE 1.3e-5 against the converged image after 600
 * iterations); 32 rows per agent reach r < 1e-6.  For tol below 1e-3, load
 * the system with fewer rows per agent.
 * Errors: as mace_solve.
 */
int mace_solve_pnp(mace_system* sys, const float* y, const float* lambda, double rho,
                   double sigma, int32_t sweeps, int32_t max_iters, double tol, int32_t h_passes,
                   float* x_out, mace_info* info);

/* Device-pointer variant of mace_solve (all arrays in device memory). */
int mace_solve_dev(mace_system* sys, const float* y, const float* lambda,
                   const mace_prior* prior, double rho, double sigma, int32_t sweeps,
                   int32_t max_iters, double tol, const float* w_init, float* x_out,
                   mace_info* info, void* stream);

/*
 * For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation): mace_solve_dev
 * with the scan's working state (error sinogram, weights, agent images, Mann
 * state, theta2, residual partials, slot descriptor) in a static workspace
 * of mace_noalloc_capacity() bytes (16 MiB) per GPU, held from the first
 * load on that GPU until the process ends.  The call allocates no device or
 * pinned memory and creates no stream, event or graph; the system's
 * matrix, schedule and the workspace's address were set up by
 * mace_load_system.  Same arguments, results and errors as mace_solve_dev
 * (y, lambda, w_init, x_out in device memory); it runs the same kernels
 * eagerly on `stream` (NULL = default stream), after the work already queued
 * there, and returns after they have finished.  A system whose scan state
 * does not fit the workspace (e.g. 256x256 with 8 agents and 360 views
 * fits; 512x512 with 16 agents does not) is rejected with MACE_E_NOMEM
 * before any launch.  Every call on a GPU uses that GPU's one workspace, and
 * each call clears what must start at zero: calls that overlap in time on
 * one GPU (from several host threads or streams) race and must not be
 * made.
 */
int mace_solve_dev_noalloc(mace_system* sys, const float* y, const float* lambda,
                           const mace_prior* prior, double rho, double sigma, int32_t sweeps,
                           int32_t max_iters, double tol, const float* w_init, float* x_out,
                           mace_info* info, void* stream);

/* Bytes of the static workspace of mace_solve_dev_noalloc on each GPU. */
int64_t mace_noalloc_capacity(void);

/*
 * Batched partial-update MACE: n_scans independent scans of this geometry
 * (e.g. the slices of a volume, or requests of a reconstruction service)
 * advance together, one Mann iteration of every scan per round of kernel
 * launches, all scans sharing the one device copy of the matrix (Sec. I: the
 * precomputed matrix is the large, reused operand).  Each scan stops on its
 * own: when its residual falls below tol it is switched off while the others
 * continue.  y[i], lambda[i]: [n_views * n_channels] of scan i; x_out[i]:
 * [nx*ny]; info (optional): array of n_scans records.  1 <= n_scans <= 128.
 * With rows_per_agent = 1 every scan follows exactly the iterates mace_solve
 * computes for it alone.  With the automatic rows_per_agent the concurrent
 * super-voxels per (scan, agent) are divided by n_scans, so the total
 * concurrency stays about the same and the scans walk the super-voxels in
 * step (sharing the matrix reads); the scans then reach the same fixed
 * points by different iterates.  Returns the worst status over the scans.
 */
int mace_solve_batch(mace_system* sys, int32_t n_scans, const float* const* y,
                     const float* const* lambda, const mace_prior* prior, double rho,
                     double sigma, int32_t sweeps, int32_t max_iters, double tol,
                     float* const* x_out, mace_info* info);

/* Device-pointer variant of mace_solve_batch (every y/lambda/x_out array in
 * device memory; the pointer arrays themselves on the host). */
int mace_solve_batch_dev(mace_system* sys, int32_t n_scans, const float* const* y,
                         const float* const* lambda, const mace_prior* prior, double rho,
                         double sigma, int32_t sweeps, int32_t max_iters, double tol,
                         float* const* x_out, mace_info* info, void* stream);

/*
 * Partial proximal update of one agent (Algorithm 2 applied `sweeps` times):
 * starting from x_init, ICD passes on f_i(z) + ||z - v||^2/(2 sigma^2)
 * (eq. (prox_F)); with many sweeps this approaches F_i(v).  All image arrays
 * have nx*ny entries (host).
 */
int mace_prox(mace_system* sys, int32_t agent, const float* y, const float* lambda,
              const mace_prior* prior, double sigma, const float* v, const float* x_init,
              int32_t sweeps, float* x_out);

/*
 * Pixel visiting order of one ICD pass (int64[nx*ny]): super-voxel colour
 * phases, the super-voxels of a phase in schedule order, raster order inside a
 * super-voxel.  With rows_per_agent = 1 every agent visits pixels exactly in
 * this order.
 */
int mace_visit_order(const mace_system* sys, int64_t* order);

/* Stacked agent states of the last solve (of the first scan of the last
 * batch), device layout [N][nx*ny], copied to host: w and X (either may be
 * NULL). */
int mace_get_state(const mace_system* sys, float* w, float* X);

/* As mace_get_state for scan slot `slot` of the last batch or volume solve
 * (slice z of a volume is slot z).  MACE_E_ARG if the slot holds no state. */
int mace_get_slot_state(const mace_system* sys, int32_t slot, float* w, float* X);

/* Error sinogram e = y - A X_i of the last solve, every row from its own
 * agent's state, copied to host in global row order (float[n_views*n_channels]). */
int mace_get_error_sinogram(const mace_system* sys, float* e);

/*
 * Scale of every ICD coordinate step, gamma in (0, 1]: z_s += gamma * alpha_s.
 * Default: 1 when the system runs the sequential schedule (rows_per_agent =
 * 1, or an image too small for more), else 0.5 -- also for batches and
 * served scans that share the rows and fall back to one row per (scan,
 * agent), because the colour-phase visiting order is not raster order.  gamma = 1 is Algorithm 2's exact coordinate minimisation
 * (of the prior's quadratic majoriser); gamma < 1 under-relaxes the partial
 * update.  A pixel is left unchanged exactly when its coordinate derivative
 * vanishes for any gamma, so the fixed points -- and, by Theorem 1, the MAP
 * solution -- do not depend on it (the argument of Lemma B.1); it changes
 * the iterates and their stability when many super-voxels of an agent are
 * updated at once.  Applies to later mace_solve / mace_prox calls.
 */
int mace_set_relaxation(mace_system* sys, double gamma);

/* Precision-path setting of a system loaded with precision 1: the FP32
 * tail (see mace_opts.fp32_tail_iters) of later solves; 0 runs FP16
 * throughout.  A positive value needs the FP32 values, which a system holds
 * when it was loaded with fp32_tail_iters > 0.  Errors: MACE_E_ARG. */
int mace_set_fp32_tail(mace_system* sys, int32_t iters);

/* Enable (1) or disable (0) HIP-event timing of the solve's kernels; the
 * figures land in mace_info.sweep_ms / sweep_launches / iter_ms. */
int mace_set_timing(mace_system* sys, int32_t enable);

/* The configuration a loaded system runs with: precision, the super-voxel
 * side in use, the rows per agent in use (the automatic value resolved),
 * fp32_tail_iters and refresh_every. */
int mace_get_config(const mace_system* sys, mace_opts* out);

/* Bytes of repacked system matrix held on the device. */
int64_t mace_system_bytes(const mace_system* sys);

/* Device bytes of one scan's state (w, X, e, Lambda, y, theta2 of every agent,
 * residual partials): what a batch slot or an admitted served scan holds. */
int64_t mace_scan_bytes(const mace_system* sys);

/* One candidate configuration measured by mace_autotune. */
typedef struct {
  int32_t sv_size, rows_per_agent;
  double ms_per_iter;  /* HIP-event time of one Mann iteration */
  double residual;     /* r_k after the timed iterations */
  int32_t status;      /* MACE_OK or MACE_E_NONFINITE */
  int32_t format;      /* record format of the candidate (1 compact, 2 general) */
} mace_tune_result;

/*
 * Autotuner of the launch configuration for one geometry: for super-voxel
 * side S in {4, 8, 16, 32} (those whose band fits in LDS; 16 and 32 in the
 * general records, FP32 values only; only base->sv_size if it is set) and
 * rows_per_agent in {P/4, P/2, P} below the automatic P (only
 * base->rows_per_agent if it is set), loads the system, solves a synthetic
 * scan (uniform 0.02/mm image, 1e4 photons, q-GGMRF prior) for `iters` timed
 * Mann iterations and keeps the fastest time per iteration among candidates
 * whose residual is within 1.5x of the best.  All candidates have the same
 * fixed point (the MAP image), so they are compared at equal accuracy.
 * *best = *base with sv_size, rows_per_agent and format chosen; results
 * (optional, up to max_results) receive every candidate, *n_results their
 * number.  Results are cached per geometry, matrix, partition and precision
 * for the life of the process.  mace_load_system with sv_size = -1 calls it.
 * Errors: as mace_load_system, MACE_E_NONFINITE if no candidate stays finite.
 */
int mace_autotune(const mace_geom* geom, const int64_t* col_ptr, const int32_t* row_idx,
                  const float* val, int32_t n_agents, const int32_t* view_to_agent,
                  const mace_opts* base, int32_t iters, mace_opts* best, double* best_ms_per_iter,
                  mace_tune_result* results, int32_t max_results, int32_t* n_results);

/*
 * Host-only dry run of mace_load_system for the same arguments: builds the
 * device tables and the super-voxel schedules in host memory and checks every
 * index the kernels form from them (band rows, record rows, task ids, LDS
 * size), without using a device.  *lds_bytes (optional) receives the LDS a
 * workgroup of the main kernel needs in a 2-D solve (for the rows per
 * workgroup chosen: 16, 8 or 4; 2 or 1 for general records with very wide
 * bands).  Same error codes as mace_load_system.
 */
int mace_check_layout(const mace_geom* geom, const int64_t* col_ptr, const int32_t* row_idx,
                      const float* val, int32_t n_agents, const int32_t* view_to_agent,
                      const mace_opts* opts, int64_t* lds_bytes);

/*
 * Reconstruction service (continuous batching).  A server drives the given
 * systems (one per scanner geometry; each may appear once, must outlive the
 * server and must not be used by other calls while the server exists).
 * Scans are submitted at any time; a worker thread per system admits them
 * oldest first into scan slots while the device memory of the admitted scans'
 * state (w, X, e, Lambda, y, theta2 per agent: mace_server_stats reports the
 * bytes) stays within hbm_budget_bytes (0 = no limit); a scan whose state
 * alone exceeds the budget fails with MACE_E_NOMEM, and one that does not fit
 * yet waits, holding back later scans so that it is not starved.  Every Mann
 * iteration (Algorithm 1) runs over all admitted scans of a system that share
 * (prior, rho, sigma, sweeps) in one round of launches; each scan stops on its
 * own when r_k < tol or after max_iters iterations, and a waiting scan takes
 * the free slot at the next iteration.  The systems' iterations run on their
 * own streams and overlap on the GPU.  A scan's result does not depend on the
 * other scans in flight beyond the iterates (the fixed point is the same).
 */
typedef struct mace_server mace_server;

typedef struct {
  int64_t submitted, completed, queued;
  int32_t in_flight, max_in_flight;    /* scans admitted and not finished */
  int64_t bytes_in_use, peak_bytes;    /* device bytes of admitted scans' state */
} mace_server_counters;

/* Starts the worker threads.  Errors: MACE_E_ARG. */
int mace_server_create(mace_system* const* systems, int32_t n_systems, int64_t hbm_budget_bytes,
                       mace_server** out);

/* Queues one scan of systems[system_idx] (y, lambda: host, copied before the
 * call returns); *ticket identifies it.  max_iters >= 1; tol >= 0 (0: run
 * max_iters iterations).  Errors: MACE_E_ARG, or the server's failure code. */
int mace_server_submit(mace_server* srv, int32_t system_idx, const float* y, const float* lambda,
                       const mace_prior* prior, double rho, double sigma, int32_t sweeps,
                       double tol, int32_t max_iters, int64_t* ticket);

/* Blocks until the scan has finished; x_out[nx*ny] (may be NULL) receives its
 * image, info its statistics, *latency_s the time from submit to finish.  A
 * ticket can be waited for once.  Returns the scan's status (MACE_OK,
 * MACE_W_MAXITER, or an error such as MACE_E_NOMEM / MACE_E_NONFINITE). */
int mace_server_wait(mace_server* srv, int64_t ticket, float* x_out, mace_info* info,
                     double* latency_s);

/* Cancels a submitted scan: one still waiting for admission leaves the queue
 * at once; one in flight is released, with its slot and memory, after the
 * Mann iteration running now.  Its mace_server_wait then returns
 * MACE_E_CANCELLED without an image.  A scan that has finished already is
 * left as it is (MACE_OK).  Errors: MACE_E_ARG (unknown ticket). */
int mace_server_cancel(mace_server* srv, int64_t ticket);

/* Counters of the server; returns MACE_OK or the server's failure code. */
int mace_server_stats(mace_server* srv, mace_server_counters* out);

/* Finishes the scans in flight, drops the waiting ones, stops the workers. */
void mace_server_destroy(mace_server* srv);

void mace_free_system(mace_system* sys);
const char* mace_last_error(void);

/* Testing hook (not part of the method): the after-th next device
 * allocation of the library in this process (0 = the very next one) fails as
 * if the device were out of memory; after < 0 switches the hook off.  It
 * fires once.  Used to check that a call which fails on memory leaves its
 * system usable: the next call allocates again (or fails cleanly) and never
 * launches a kernel on a buffer that was not allocated. */
int mace_test_fail_alloc(int32_t after);

#ifdef __cplusplus
}
#endif
#endif /* MACE_H */
