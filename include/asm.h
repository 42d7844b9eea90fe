/*
 * asm.h - C ABI of the MI355X Schwarz-preconditioned GMRES solver for 3x3
 * block Jacobians (Jackson, Taroni, Ponting, "A Two-Level Variant of
 * Additive Schwarz Preconditioning for Use in Reservoir Simulation",
 * arXiv:1401.7227).
 *
 * The linear problem is the one of Section 2: r = b - A x with b = R (the
 * non-linear residual) and A = -J (J the Jacobian of eq. (1.2)), so the
 * solution x is the Newton update of eq. (1.1).  Unknowns are grouped per
 * grid cell into 3-vectors (p, So, Sg) and A is stored with dense 3x3
 * blocks (Section 1).
 *
 * Conventions for every call:
 *  - Pointers named *_dev are device pointers (HBM of the current HIP
 *    device); pointers named *_host are host pointers.  The caller owns
 *    them; the library never frees or retains them past the call.
 *  - Cell c = (ix*ny + iy)*nz + iz (z fastest); unknown 3c + v.
 *  - BSR: row_ptr[nb+1], col_idx[nnzb] (strictly increasing per row,
 *    diagonal block present), vals[9*nnzb] with each 3x3 block row-major.
 *  - Work is ordered on the given stream; calls that return host results
 *    synchronise that stream before returning.
 *  - Errors are returned as asm_status, never thrown; asm_last_error()
 *    gives a thread-local message for the last failing call.  A host
 *    allocation failure inside the library returns ASM_ERR_OOM, any other
 *    internal C++ exception ASM_ERR_INVALID ("internal error: ...").
 *  - A handle must not be used from two threads at once.  Handles hold
 *    device memory until destroyed.
 */
#ifndef ASM_MI355X_H
#define ASM_MI355X_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ASM_OK = 0,
  ASM_NOT_CONVERGED = 1,        /* warning: x holds the last iterate        */
  ASM_ERR_INVALID = -1,         /* bad argument, shape or BSR structure     */
  ASM_ERR_OOM = -2,             /* device or host allocation failed         */
  ASM_ERR_SINGULAR_PIVOT = -3,  /* a 3x3 ILU pivot is singular/non-finite   */
  ASM_ERR_NONFINITE = -4,       /* NaN/Inf in A, b or x0                    */
  ASM_ERR_HIP = -5              /* a HIP runtime call failed                */
} asm_status;

typedef struct asm_system_s *asm_system;   /* device copy of A, own layout */
typedef struct asm_precond_s *asm_precond; /* partition, maps, factors     */

typedef struct {
  int32_t nx, ny, nz;
} asm_grid;

/* Preconditioner kinds and combinations. */
enum { ASM_KIND_NONE = 0, ASM_KIND_CLASSICAL = 1, ASM_KIND_TWO_LEVEL = 2 };
enum { ASM_COMBINE_ADDITIVE = 0, ASM_COMBINE_RESTRICTED = 1 };
enum { ASM_PREC_FP64 = 0, ASM_PREC_FP32 = 1 };
/* Outside cells of the two-level form (the variants of Section 5). */
enum { ASM_FIELD_NEAR_FAR = 0, ASM_FIELD_NEAR = 1, ASM_FIELD_FAR = 2 };
/* Global coarse-grid correction (Section 3). */
enum { ASM_COARSE_NONE = 0, ASM_COARSE_ADDITIVE = 1, ASM_COARSE_TWO_STAGE = 2 };
#define ASM_COARSE_MAX_UNKNOWNS 8192
/* Local solver: block ILU(0) (Section 2, Section 6) or exact (Section 5:
 * Gaussian elimination; here a dense inverse of each A_i). */
enum { ASM_LOCAL_ILU0 = 0, ASM_LOCAL_EXACT = 1 };
#define ASM_EXACT_MAX_UNKNOWNS 6144

/*
 * asm_create_system - take a device copy of A (Section 2's A = -J).
 *   grid       : host; nx*ny*nz must equal nb.
 *   nb, nnzb   : block rows and stored blocks.
 *   row_ptr_dev, col_idx_dev, vals_dev : device BSR arrays (see above);
 *                copied, the caller may free them after return.
 *   Validates the structure (INVALID) and finiteness (NONFINITE); one
 *   device-to-host copy of the pattern is made for the host-side setup.
 *   out        : host; receives the handle.
 */
asm_status asm_create_system(const asm_grid *grid, int32_t nb, int64_t nnzb,
                             const int32_t *row_ptr_dev, const int32_t *col_idx_dev,
                             const double *vals_dev, hipStream_t stream, asm_system *out);

/* New values on the same pattern (the next Newton iteration, Section 4:
 * matrices are re-lumped once per non-linear iteration).  vals_dev as in
 * asm_create_system.  Preconditioners built on the system must then be
 * refreshed with asm_refactor. */
asm_status asm_update_values(asm_system sys, const double *vals_dev, hipStream_t stream);

/* y = A x (device vectors of 3*nb doubles), with the system's SpMV
 * launch shape (see asm_tuning; every shape sums in the same order). */
asm_status asm_spmv(asm_system sys, const double *x_dev, double *y_dev, hipStream_t stream);

/*
 * Preconditioner options.
 *   kind      NONE (B = I), CLASSICAL (eq. (3.3)-(3.4): A_i = R_i A R_i^T
 *             with R_i restricting to the overlapping subdomain), or
 *             TWO_LEVEL (Section 4, eq. (4.1): outside cells are lumped by
 *             summation into near-field boxes on face-neighbour subdomains
 *             and far-field boxes elsewhere; Appendix B, eq. (B.3)).
 *   combine   ADDITIVE (eq. (3.3): overlapping contributions summed) or
 *             RESTRICTED (eq. (4.2): each cell keeps its owner's value; the
 *             coarse part of every local solution is discarded).
 *   sx, sy    subdomains along x and y; each spans all of z.  Balanced
 *             split: the first (n mod s) parts get one extra column.
 *   overlap   algebraic overlap: cells within this graph distance of a
 *             subdomain in A's (symmetrised) block graph.
 *   near, far coarsening boxes (cells per box along x, y, z), two-level only.
 *   precision FP64, or FP32: factors of fine rows stored and applied in
 *             single precision, coarse rows kept in double; the outer GMRES
 *             stays double.
 *   field     two-level only (Section 5 compares the three): NEAR_FAR
 *             (default), NEAR (near field only: outside cells of
 *             non-neighbouring subdomains are dropped) or FAR (far field only:
 *             every outside cell is lumped into far boxes).
 *   coarse    global coarse-grid correction with boxes of coarse_box cells:
 *             R_C sums the cells of each box of a global box grid (per
 *             unknown), A_C = R_C A R_C^T (eq. (3.6)) is inverted exactly
 *             (dense, on the device; at most ASM_COARSE_MAX_UNKNOWNS = 3 x
 *             boxes, INVALID beyond) and B_C^-1 = R_C^T A_C^-1 R_C is
 *             ADDITIVE: added to the Schwarz part (eq. (3.5)), or
 *             TWO_STAGE: applied to the residual the Schwarz part leaves,
 *             B^-1 = B_AS^-1 + B_C^-1 (I - A B_AS^-1) (eq. (3.8)).  Not
 *             available in asm_solve_batch or the server (INVALID).
 *   local     ILU0 (default), or EXACT: every A_i is inverted densely on
 *             the device (Gauss-Jordan with partial pivoting, FP64 whatever
 *             the precision option) and applied as a dense product; for
 *             small subdomains only: 3 x rows of A_i at most
 *             ASM_EXACT_MAX_UNKNOWNS and all inverses together at most
 *             8 GiB (INVALID beyond).  Not available in asm_solve_batch or
 *             the server (INVALID).
 * Default local solver: block ILU(0) with 3x3 pivots inverted directly
 * (Section 2; Section 6 names ILU as the approximate local solve).
 */
typedef struct {
  int32_t kind;
  int32_t combine;
  int32_t sx, sy;
  int32_t overlap;
  int32_t near_box[3];
  int32_t far_box[3];
  int32_t precision;
  int32_t field;
  int32_t coarse;
  int32_t coarse_box[3];
  int32_t local;
} asm_precond_opts;

/* Builds the partition, overlap, coarse maps, extended patterns and level
 * schedules on the host, then assembles and factorises every A_i on the
 * device.  A singular pivot returns ASM_ERR_SINGULAR_PIVOT naming the
 * subdomain and block row.  out: host; receives the handle. */
asm_status asm_setup_precond(asm_system sys, const asm_precond_opts *opts, hipStream_t stream,
                             asm_precond *out);

/* Numeric re-assembly and re-factorisation after asm_update_values. */
asm_status asm_refactor(asm_precond pc, hipStream_t stream);

/*
 * asm_precond_clone - the preconditioner of `sys` built on the plan of `src`.
 * Section 4 re-lumps the coarse matrices once per non-linear iteration on a
 * fixed decomposition: everything that depends only on the grid, the block
 * pattern and the options (partition, overlap, coarse maps, level schedules,
 * sweep layout) is computed once.  sys must have the same grid and block
 * pattern as src's system (INVALID otherwise).  The clone shares that
 * pattern-only state with src (it stays alive until every handle sharing it
 * is destroyed; src may be destroyed first) and gets its own assembled
 * matrices and factors, computed on the device from sys's values, exactly
 * as asm_setup_precond would compute them.  out: host; receives the handle.
 */
asm_status asm_precond_clone(asm_precond src, asm_system sys, hipStream_t stream, asm_precond *out);

/* z = B^-1 r (device vectors of 3*nb doubles). */
asm_status asm_precond_apply(asm_precond pc, const double *r_dev, double *z_dev, hipStream_t stream);

/* Sizes of the preconditioner (host struct). */
typedef struct {
  int32_t nsub;
  int64_t ext_rows;      /* sum over subdomains of rows of A_i           */
  int64_t coarse_rows;   /* of which lumped (coarse) rows                */
  int64_t factor_blocks; /* stored 3x3 blocks of all factors             */
  int64_t fine_row_blocks; /* of which in fine rows (single precision   */
                           /* when precision is FP32)                    */
  int32_t max_levels;    /* longest forward or backward level schedule   */
  int64_t device_bytes;  /* device memory held by the preconditioner     */
  int64_t sweep_steps;   /* forward + backward sweep steps, all subdomains */
  int64_t reloaded_rows; /* rows whose values are reloaded from global
                            memory (no on-chip slot) during a sweep      */
  int64_t split_rows;    /* rows (counted once per sweep) whose sum is
                            computed in pieces over several sweep steps:
                            too many entries for one record, or too many
                            reloaded inputs for the reload slots          */
} asm_precond_stats;
asm_status asm_precond_get_stats(asm_precond pc, asm_precond_stats *stats_host);

/* Copies subdomain s's local matrix and factors to host buffers, in the
 * local ordering (fine cells ascending, then near boxes, then far boxes):
 *   rp_host[n+1], ci_host[nnz], a_host[9*nnz] (assembled A_i),
 *   f_host[9*nnz] (ILU(0): L below the diagonal, U above, D^-1 on it),
 *   label_host[nb] (row of A_i each cell maps to, -1 if none).
 * Any pointer may be NULL.  Query n and nnz first with all buffers NULL. */
asm_status asm_precond_export_sub(asm_precond pc, int32_t s, int32_t *n, int32_t *nnz,
                                  int32_t *rp_host, int32_t *ci_host, double *a_host,
                                  double *f_host, int32_t *label_host);

/* Restarted right-preconditioned GMRES(restart) (Section 2 names GMRES as
 * the accelerator).  One iteration is one Arnoldi step.  Stops when the
 * true residual satisfies ||b - A x|| <= rtol ||b||, or at max_iters
 * (ASM_NOT_CONVERGED, x holds the last iterate).  fixed_iters > 0 runs
 * exactly that many steps without convergence tests. */
typedef struct {
  int32_t restart;     /* default 30, at most 32 */
  double rtol;         /* default 1e-6 */
  int32_t max_iters;   /* default 10000 */
  int32_t fixed_iters; /* 0 = off */
} asm_solve_opts;

typedef struct {
  int32_t iters, cycles;
  double rel_res_true, rel_res_est;
} asm_solve_info;

/* b_dev: device, 3*nb doubles.  x_dev: device, in: x0, out: solution.
 * opts, info: host.  Synchronises the stream before returning. */
asm_status asm_solve(asm_system sys, asm_precond pc, const double *b_dev, double *x_dev,
                     const asm_solve_opts *opts, hipStream_t stream, asm_solve_info *info);

/*
 * asm_solve_noalloc - asm_solve for callers that cannot allocate memory:
 * code around HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  The same restarted GMRES with the same arithmetic and results
 * as asm_solve, but every Krylov work array (basis, work vectors, partial
 * sums, published Hessenberg columns) lives in one fixed device array of the
 * library, ASM_NOALLOC_SCRATCH_BYTES per device, reserved when the library's
 * code is loaded on a device and held until the process ends; host-side
 * state is on the caller's stack.  The call makes no device or pinned-host
 * allocation (asm_solve allocates the system's workspace on its first call).
 * Limits: 8 * ((restart+1)*3*nb + 3*3*nb) bytes plus about 360 KiB must fit
 * the array (at restart 30 about 240,000 unknowns, 80,000 cells); larger
 * systems return ASM_ERR_INVALID.  The host reads each step's column
 * synchronously (no step queued ahead), so it is somewhat slower than
 * asm_solve.  Every call on a device shares that device's array: calls that
 * overlap on one device (two host threads, or two streams) race and must not
 * be made.  sys and pc must already exist (their setup allocates).
 */
#define ASM_NOALLOC_SCRATCH_BYTES (64 << 20)
asm_status asm_solve_noalloc(asm_system sys, asm_precond pc, const double *b_dev, double *x_dev,
                             const asm_solve_opts *opts, hipStream_t stream, asm_solve_info *info);

/* The same solve as asm_solve, with every restart cycle run as one HIP
 * graph: the m Arnoldi steps, the Givens rotations (computed on the device),
 * the triangular solve, the correction x += B^-1 V_k y and the true residual.
 * A cycle's end (residual estimate at the tolerance, breakdown, or the step
 * limit the host writes before each cycle) sets a device flag on which the
 * later steps' kernels return at once, so the host synchronises once per
 * cycle instead of reading every step.  The graph is captured on the first
 * cycle and kept by the system for later calls with the same preconditioner,
 * b, x and restart length (capturing again otherwise); it runs on a stream of
 * the library's own, after the work already queued on `stream`.  Results
 * equal asm_solve's up to rounding (the rotations are computed on the
 * device).  Preconditioners with ILU(0) local solves and no global coarse
 * grid (or none) only: others give ASM_ERR_INVALID.  The host thread does no
 * per-step work; on one MI355X this is not faster than asm_solve, whose host
 * loop keeps one step queued ahead of the device (the steps after a cycle's
 * end still launch, then return). */
asm_status asm_solve_graph(asm_system sys, asm_precond pc, const double *b_dev, double *x_dev,
                           const asm_solve_opts *opts, hipStream_t stream, asm_solve_info *info);

/* Solves `count` independent systems together: systems[i] x[i] = b[i] with
 * preconds[i] (built on systems[i]), all with the same options.  Every
 * kernel launch serves all systems still iterating (one sweep launch covers
 * the subdomains of all of them, and so on), so many small systems fill the
 * GPU; each system's arithmetic is exactly that of asm_solve, so every x[i]
 * and infos[i] equal what asm_solve returns for that system alone.
 * systems, preconds, b, x: host arrays of `count` handles / device vector
 * pointers (each 3*nb_i doubles; x[i] in: x0, out: solution); a system may
 * appear only once.  infos, status: host arrays of `count` (status[i] is
 * ASM_OK or ASM_NOT_CONVERGED).  Returns ASM_OK if all converged,
 * ASM_NOT_CONVERGED if any did not, or an error (nothing solved).  Uses the
 * systems' own workspaces; synchronises the stream before returning. */
asm_status asm_solve_batch(int32_t count, const asm_system *systems, const asm_precond *preconds,
                           const double *const *b_dev, double *const *x_dev, const asm_solve_opts *opts,
                           hipStream_t stream, asm_solve_info *infos, int32_t *status);

/*
 * Request server.  A request is the sequence of linear solves of one
 * simulation on one grid: Section 2's Newton iteration (eq. (1.1)) solves
 * A x = b once per non-linear iteration, with new values on the same block
 * pattern, and Section 4 re-lumps the coarse matrices for each of them on
 * the same decomposition.  The server keeps many requests in flight on one
 * device:
 *  - admission: queued requests are admitted in submission order while the
 *    device memory they are expected to hold fits hbm_budget_bytes (0 = no
 *    limit) and fewer than max_active solves are in flight; the first
 *    request that does not fit stops admission (no overtaking), except that
 *    a request is always admitted when no other request is running;
 *  - plans: the pattern-only part of the preconditioner (asm_setup_precond's
 *    host planning) is built once per grid, pattern and options and cached;
 *    every request gets a clone of it (asm_precond_clone) with its own
 *    factors.  Cached plans no request uses are dropped, least recently used
 *    first, when the budget needs their memory;
 *  - execution: the solves of all admitted requests iterate together, as
 *    asm_solve_batch runs them (one launch per kernel serves all), and a new
 *    solve joins between restart cycles.  After solve k of a request its
 *    system takes the values vals_dev[k+1] and its preconditioner is
 *    refactored (asm_update_values, asm_refactor) before solve k+1 joins.
 *    Every solve's arithmetic is that of asm_solve on the same system and
 *    preconditioner options, whatever else is in flight.
 * One server drives one stream from one host thread.
 */
#define ASM_SERVER_MAX_SOLVES 8
#define ASM_SERVER_MAX_ACTIVE 1024
typedef struct asm_server_s *asm_server;
typedef struct {
  asm_solve_opts solve;      /* for every solve; see asm_solve                    */
  int64_t hbm_budget_bytes;  /* device bytes for requests and cached plans, 0 = no limit */
  int32_t max_active;        /* solves in flight at once, 1..ASM_SERVER_MAX_ACTIVE */
} asm_server_opts;

/* A request; the server copies this descriptor.  Every device buffer it
 * names belongs to the caller and must stay valid until the request's
 * completion is returned. */
typedef struct {
  int64_t tag;                      /* caller's id, returned on completion          */
  asm_grid grid;                    /* as asm_create_system                          */
  int32_t nb;
  int64_t nnzb;
  const int32_t *row_ptr_dev;       /* BSR pattern (device)                          */
  const int32_t *col_idx_dev;
  asm_precond_opts precond;         /* kind CLASSICAL or TWO_LEVEL                   */
  int32_t nsolves;                  /* 1..ASM_SERVER_MAX_SOLVES                       */
  const double *vals_dev[ASM_SERVER_MAX_SOLVES];  /* values of solve k (device)   */
  const double *b_dev[ASM_SERVER_MAX_SOLVES];     /* right-hand side of solve k     */
  double *x_dev[ASM_SERVER_MAX_SOLVES];           /* in: x0, out: solution k        */
} asm_request;

typedef struct {
  int64_t tag;
  int32_t status;        /* ASM_OK; ASM_NOT_CONVERGED if any solve stopped at
                            max_iters; or the error of a setup, refactor or
                            input check (later solves are not run)            */
  int32_t solves;        /* solves finished                                    */
  int32_t iters;         /* Arnoldi steps over all solves                      */
  int32_t plan_cached;   /* 1 if the plan was in the cache at admission        */
  double rel_res_true;   /* of the last solve                                  */
} asm_completion;

typedef struct {
  int32_t queued, running, iterating, completed_unread, cached_plans;
  int64_t bytes_in_use;  /* device bytes of running requests and cached plans */
  int64_t plan_builds, plan_hits;
} asm_server_state;

asm_status asm_server_create(const asm_server_opts *opts, hipStream_t stream, asm_server *out);
/* Queues a request (no device work).  Its tag must differ from the tags of
 * all live requests (queued, running, or completed but not yet returned by
 * asm_server_poll): ASM_ERR_INVALID otherwise.  A tag is free again once
 * its completion has been returned. */
asm_status asm_server_submit(asm_server srv, const asm_request *req);
/* One scheduling round: admission, one restart cycle of every solve in
 * flight, then up to `max` completions (oldest first) into done_host;
 * *ndone receives their number.  Synchronises the stream.  An error return
 * (device failure) leaves the server unusable except for destroy. */
asm_status asm_server_poll(asm_server srv, int32_t max, asm_completion *done_host, int32_t *ndone);
asm_status asm_server_get_state(asm_server srv, asm_server_state *state_host);
/* Frees every request still queued or running (their results are lost)
 * and every cached plan. */
void asm_server_destroy(asm_server srv);

/* Kernel-phase timing of asm_solve (HIP events on the solve stream).
 * asm_profile_enable(sys, phase_mask): bit k of phase_mask times phase k
 * (0 = off, 0xff = all): inside asm_solve every launch of a timed phase
 * is bracketed by events, which add a little time per launch, so time
 * only what is needed.  asm_profile_read returns the launch counts and
 * accumulated device milliseconds since the last reset. */
enum {
  ASM_PHASE_ILU_APPLY = 0,  /* forward/backward sweeps (one kernel launch)   */
  ASM_PHASE_LUMP = 1,       /* restriction: lumped coarse sums, subdomain
                               right-hand sides in sweep order             */
  ASM_PHASE_COMBINE = 2,    /* additive combination                           */
  ASM_PHASE_SPMV = 3,       /* w = A z                                        */
  ASM_PHASE_DOTS = 4,       /* Gram-Schmidt projections V^T w and ||w||       */
  ASM_PHASE_UPDATE = 5,     /* w - V h and its norm                           */
  ASM_PHASE_RESIDUAL = 6,   /* b - A x and its norm                           */
  ASM_PHASE_OTHER = 7,      /* reductions, solution update                    */
  ASM_NPHASE = 8
};
typedef struct {
  int64_t launches[ASM_NPHASE];
  double ms[ASM_NPHASE];
} asm_profile;
asm_status asm_profile_enable(asm_system sys, int32_t phase_mask);
asm_status asm_profile_read(asm_system sys, asm_profile *out_host, int32_t reset);

/* Launch-shape tuning of a system's Krylov kernels (no passage of the
 * paper: a choice of this implementation).  Two runtime choices:
 *   spmv_rows   block rows per thread of the SpMV w = A z: 1, 2 or 4.  The
 *               same sums in the same order whatever the choice.
 *   red_blocks  partial-sum blocks of the Gram-Schmidt kernels (V^T w and
 *               w - V h with its norm): 512, 1024, 2048 or 4096.  The
 *               choice fixes the order of the dot products' sums, so it
 *               changes results in the last bits (not beyond the rounding
 *               bound of a dot product).
 * The first asm_solve, asm_solve_graph or asm_solve_batch on an untuned
 * system times every candidate on the system's own matrix and work arrays
 * (HIP events, a few milliseconds for a 1M-cell system) and keeps the
 * fastest; a candidate replaces the default (1 row, 1024 blocks) only when
 * it is at least 3% faster.  The choice is cached per process, device,
 * size class (block rows rounded up to a power of two) and restart length:
 * later systems of the same class take it without timing (source
 * ASM_TUNE_CACHED), so one process makes one choice per class.  The
 * environment variable ASM_TUNE=0 turns timing off (defaults are used);
 * asm_tuning_set fixes a choice (for reproducible summation orders across
 * processes).  asm_solve_noalloc never times: it uses the system's current
 * choice.  A batch uses each system's choice, so batched and single solves
 * stay identical. */
enum {
  ASM_TUNE_DEFAULT = 0,  /* not tuned: default choice                      */
  ASM_TUNE_TIMED = 1,    /* timed on this system                           */
  ASM_TUNE_CACHED = 2,   /* taken from an earlier system of its size class */
  ASM_TUNE_SET = 3       /* fixed by asm_tuning_set                        */
};
typedef struct {
  int32_t spmv_rows;     /* 1, 2 or 4                                      */
  int32_t red_blocks;    /* 512, 1024, 2048 or 4096                        */
  int32_t source;        /* ASM_TUNE_*                                     */
  int32_t restart;       /* restart length the Krylov timing used          */
  double spmv_us[3];     /* one SpMV with 1, 2, 4 rows per thread (timed
                            choices; else 0)                               */
  double krylov_us[4];   /* Gram-Schmidt kernels per Arnoldi step, mean over
                            a restart cycle (1 .. restart columns), with
                            512, 1024, 2048, 4096 blocks                   */
} asm_tuning;
/* The system's current choice and the timings it was made from. */
asm_status asm_tuning_get(asm_system sys, asm_tuning *out_host);
/* Fixes the choice (source becomes ASM_TUNE_SET; timings are cleared).
 * spmv_rows = red_blocks = 0 returns the system to untuned: the next solve
 * times again, bypassing the cache.  INVALID for any other value outside
 * the lists above. */
asm_status asm_tuning_set(asm_system sys, int32_t spmv_rows, int32_t red_blocks);

/* Order of the systems in the launches of asm_solve_batch (a choice of
 * this implementation; results do not depend on it):
 *   ASM_BATCH_ORDER_SUBMITTED      as passed;
 *   ASM_BATCH_ORDER_LARGEST_FIRST  systems with more block rows first, so a
 *                                  launch's workgroups for the small
 *                                  systems fill in at its end;
 *   ASM_BATCH_ORDER_TUNE           (default) the first batch of a size class
 *                                  (device, count and total block rows, each
 *                                  rounded up to a power of two) runs its
 *                                  first restart cycle in the submitted
 *                                  order and its second largest first, timed
 *                                  on the host per block row and Arnoldi
 *                                  step; the second order is kept, for the
 *                                  rest of that batch and for later batches
 *                                  of the class, only if at least 3% faster.
 *                                  ASM_TUNE=0 keeps the submitted order.
 * asm_batch_order_set sets the process-wide choice (INVALID for other
 * values); asm_batch_tuning_last reports what the calling thread's last
 * asm_solve_batch used (source: ASM_TUNE_*; the timings of the two orders,
 * nanoseconds per block row and step, where they were timed, else the
 * cached ones or 0). */
enum {
  ASM_BATCH_ORDER_TUNE = -1,
  ASM_BATCH_ORDER_SUBMITTED = 0,
  ASM_BATCH_ORDER_LARGEST_FIRST = 1
};
typedef struct {
  int32_t order;
  int32_t source;
  double ns_per_row_step[2]; /* submitted, largest first */
} asm_batch_tuning;
asm_status asm_batch_order_set(int32_t order);
asm_status asm_batch_tuning_last(asm_batch_tuning *out_host);

/* Device-memory hooks, for callers whose framework owns device memory (a
 * caching allocator): with hooks set, every device array a handle keeps
 * (matrix, factors, plans, Krylov work arrays) comes from
 * alloc(bytes, device, ctx), which returns NULL on failure (the call then
 * fails with ASM_ERR_OOM) and a pointer aligned to 256 bytes, and goes back
 * through free_fn(ptr, bytes, device, ctx) when the handle is destroyed
 * (after a device synchronisation, so no kernel still uses it).  A handle
 * keeps the hooks that were set when it was created.  Both NULL: hipMalloc
 * and hipFree (the default).  The small per-call tables of batched and
 * served solves, the pinned host buffers and the no-allocation solve's
 * fixed array do not use the hooks.  INVALID if only one is NULL. */
typedef void *(*asm_alloc_fn)(size_t bytes, int32_t device, void *ctx);
typedef void (*asm_free_fn)(void *ptr, size_t bytes, int32_t device, void *ctx);
asm_status asm_set_allocator(asm_alloc_fn alloc, asm_free_fn free_fn, void *ctx);

/* Frees a handle and its device memory.  A system's preconditioners are
 * destroyed before the system. */
void asm_destroy_precond(asm_precond pc);
void asm_destroy_system(asm_system sys);

/* Thread-local message of the last failing call on this thread. */
const char *asm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ASM_MI355X_H */
