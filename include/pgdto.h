/*
 * pgdto.h - C ABI of the MI355X (gfx950) projection library for PGD-TO
 * (projected gradient descent for topology optimization, arXiv 2511.13905).
 *
 * What it computes.  Every entry point solves the projection subproblem of the
 * paper: given a point y (the paper's rho~, the gradient step of Alg. 3), the
 * box [lo, hi] (the paper's [l, u]) and m linearized constraint rows
 * A x <= b (rows a_j = grad g_j(rho_t), Sec. 3.2, eq. (linearized)),
 *
 *     x = argmin 1/2 ||x - y||^2 + (1/(2 kappa)) ||s||^2
 *         s.t. lo <= x <= hi,  A x - s <= b,  s >= 0,          kappa = 2/C
 *
 * (the regularized projection, eq. (regularized_projection); kappa = 0, i.e.
 * C = INFINITY, is eq. (linearized) itself).  By Theorems 1 and 2 the answer is
 * x = clip(y - A^T lam, lo, hi) for the unique multiplier lam >= 0 (lam is the
 * paper's -y) with h(lam) <= 0 and lam_j h_j(lam) = 0, where
 * h_j(lam) = a_j.x(lam) - b_j - kappa lam_j (Appendix A.2, eq. (h)).
 * Rows flagged in pgdto_problem.eq_mask are equalities a_j.x = b_j (Sec. 3.2,
 * the note on equality constraints): always active, lam_j of either sign.
 * A negative C asks for the automatic penalty of Appendix A.2.
 *
 *   PGDTO_SINGLE       one dense row: Algorithm 1 (dual bracket search).
 *   PGDTO_INDEPENDENT  m rows on disjoint contiguous element ranges
 *                      (Sec. 3.2.2): one bracket search per block, all blocks
 *                      in one launch.
 *   PGDTO_COUPLED      m <= PGDTO_MAX_M dense rows: Algorithm 2 (Stage 1
 *                      single-active searches, then semismooth Newton with a
 *                      line search, Appendix A.2).  Up to 8 rows every
 *                      route and dtype; 9 to 64 rows (the Jacobian sums
 *                      A D A^T of eq. reg_jacobian on the matrix cores, the
 *                      Stage-1 candidate check in float64 on the matrix
 *                      cores, a workgroup-parallel float64 LDL^T of the
 *                      active block): float32 projections through
 *                      pgdto_project / pgdto_project_async only; other
 *                      routes (Algorithm 3 steps, batches, serving,
 *                      pgdto_project_noalloc) return PGDTO_ERR_ARG
 *                      (pgdto_project_noalloc: PGDTO_ERR_SCRATCH).  The
 *                      context allocates a 4.6 MiB workspace for it at
 *                      its first such call.
 *
 * pgdto_pgd_step additionally performs one iteration body of Algorithm 3:
 * step size (eq. final_alpha with the fallback rule), conjugate direction
 * (eq. CG), rho~ = rho_t + omega alpha_t d_t, projection, stop test.
 *
 * Memory.  Pointers named "device" are HIP device memory (or memory the GPU
 * can read), owned by the caller, 16-byte aligned.  Rows of A start on 16-byte
 * boundaries: lda (in elements) must be >= n and lda * sizeof(T) a multiple of
 * 16.  Outputs must not alias inputs except where stated.  The library never
 * frees or retains caller buffers after a call returns (batch calls: until
 * the request's poll returns PGDTO_OK or an error).
 *
 * Errors.  Every function returns a pgdto_status.  Argument errors are found
 * on the host before anything is launched (PGDTO_ERR_ARG).  Numerical
 * outcomes are reported in pgdto_result.outcome, never as a status.  No C++
 * exception crosses this interface.
 *
 * Threads.  A context serializes its work on the stream it is called with;
 * calls on one context must not overlap (use one context per stream).
 * Batch submit/poll are thread-safe.
 */
#ifndef PGDTO_H
#define PGDTO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PGDTO_VERSION 8      /* 2: eq_mask, automatic C, pgdto_result.kappa; 3: lambda0, 5 tune shapes;
                                4: pgdto_result.lambda_err, x_err; 5: pgdto_project_noalloc;
                                6: pgdto_project_batch_async, pgdto_pgd_step_batch_async;
                                7: pgdto_params.compact, pgdto_pgd_args.work, autotune save/load;
                                8: pgdto_result.dist2, pgdto_kappa_path */
#define PGDTO_MAX_M 64       /* coupled rows */
#define PGDTO_MAX_BLOCKS 64  /* independent blocks */

typedef enum {
  PGDTO_OK = 0,
  PGDTO_PENDING = 1,           /* batch: request admitted, not finished    */
  PGDTO_QUEUED = 2,            /* batch: request waiting for admission     */
  PGDTO_ERR_ARG = -1,          /* invalid argument (nothing was launched)  */
  PGDTO_ERR_HIP = -2,          /* HIP runtime error                        */
  PGDTO_ERR_NOMEM = -3,        /* device or host allocation failed         */
  PGDTO_ERR_UNKNOWN_TICKET = -4,
  PGDTO_ERR_TIMEOUT = -5,      /* a device-side wait ran past its bound    */
  PGDTO_ERR_BUSY = -6,         /* batch: queue full                        */
  PGDTO_ERR_CANCELLED = -7,    /* batch: destroyed before the request ran  */
  PGDTO_ERR_SCRATCH = -8       /* pgdto_project_noalloc: the problem needs
                                  more workspace than the static array holds */
} pgdto_status;

typedef enum {
  PGDTO_CONVERGED = 0,   /* multiplier found to tolerance                       */
  PGDTO_INACTIVE = 1,    /* lam = 0: x = clip(y) (Alg. 1 first branch)          */
  PGDTO_INFEASIBLE = 2,  /* a row cannot hold on the box; kappa = 0: x is the
                            saturated point, kappa > 0: positive slack          */
  PGDTO_MAXITER = 3,     /* iteration limit reached; x is the last iterate      */
  PGDTO_NONFINITE = 4    /* NaN/Inf in y or A; x is clip(y) and meaningless     */
} pgdto_outcome;

typedef enum { PGDTO_F32 = 0, PGDTO_F64 = 1 } pgdto_dtype;
typedef enum { PGDTO_SINGLE = 0, PGDTO_INDEPENDENT = 1, PGDTO_COUPLED = 2 } pgdto_kind;

/* 1-D dual search rule (Alg. 1 and Stage 1 of Alg. 2).
 * BISECT: the printed midpoint rule.  NEWTON (default): the same bracket,
 * but each pass also evaluates Newton points from both bracket ends of the
 * piecewise-linear dual function (its slope sum_free a_i^2 + kappa comes
 * out of the same pass), which reaches the exact root in a few passes.     */
typedef enum { PGDTO_SEARCH_NEWTON = 0, PGDTO_SEARCH_BISECT = 1 } pgdto_search;

/* Complementarity function of the semismooth Newton stage.
 * PAPER: Phi_j = max(h_j, 0) + sign(max(-h_j, 0)) y_j as printed (eq. phi).
 * CONTINUOUS (default): Phi_j = max(h_j, -c_j lam_j), c_j = (J_h)_jj; same
 * roots, continuous at h_j = 0 (the printed form jumps there, which stalls
 * the line search once h is at rounding level).                           */
typedef enum { PGDTO_NCP_CONTINUOUS = 0, PGDTO_NCP_PAPER = 1 } pgdto_ncp;

typedef enum { PGDTO_CG_PR_PLUS = 0, PGDTO_CG_FR = 1, PGDTO_CG_NONE = 2 } pgdto_cg_rule;

typedef struct {
  int32_t kind;                 /* pgdto_kind                                   */
  int32_t dtype;                /* pgdto_dtype of y, A and x                    */
  int64_t n;                    /* elements, n >= 1                             */
  int32_t m;                    /* rows (SINGLE: 1; INDEPENDENT: blocks)        */
  const void* y;                /* device [n]: point to project (rho~)          */
  const void* A;                /* device: SINGLE/COUPLED [m][lda] row-major;
                                   INDEPENDENT [n], coefficient of element i in
                                   the row of the block that owns it            */
  int64_t lda;                  /* SINGLE/COUPLED row stride (elements)         */
  const int64_t* block_offsets; /* host [m+1], INDEPENDENT only:
                                   0 = o_0 < o_1 < ... < o_m = n               */
  const double* b;              /* host [m]: right-hand sides of A x <= b       */
  double lo, hi;                /* box, finite, lo < hi                         */
  double C;                     /* penalty; kappa = 2/C; INFINITY: kappa = 0.
                                   C < 0: automatic, C = 2 max_j bp_j / tau with
                                   tau = -C (the bound on constraint violation
                                   of the regularized projection, Appendix A.2):
                                   kappa = tau / max_j bp_j, bp_j the largest
                                   breakpoint (y_i - bound_i)/a_ji of row j;
                                   kappa = 0 when no breakpoint is positive     */
  void* x;                      /* device [n] output; must not alias y or A    */
  uint32_t* free_mask;          /* optional device [(n+31)/32]: bit i set when
                                   lo <= (y - A^T lam)_i <= hi; NULL to skip    */
  uint64_t eq_mask;             /* bit j set: row / block j is an equality
                                   a_j.x = b_j (Sec. 3.2, the note on equality
                                   constraints: always active, multiplier of
                                   either sign, lambda[j] < 0 when the row is
                                   raised to its target); 0: all A x <= b.
                                   Bits at or above m: PGDTO_ERR_ARG           */
  const double* lambda0;        /* optional host [m]: warm start, e.g. the
                                   multipliers of the previous Algorithm 3
                                   iteration; NULL: cold start.  Finite, >= 0
                                   for inequality rows (else PGDTO_ERR_ARG).
                                   Changes the search path, not the problem:
                                   1-D rows evaluate lambda0[j] in the first
                                   search pass, beside the cold first trial,
                                   when it lies inside the bracket (0, largest
                                   breakpoint) and ignore it otherwise;
                                   COUPLED starts the Newton iteration at
                                   lambda0 instead of Stage 1                 */
} pgdto_problem;

typedef struct {
  double tol_b;          /* bracket width at which a 1-D search stops (absolute,
                            dual units; paper default 1e-8, Sec. 3.5)        */
  double tol_n;          /* residual tolerance relative to each row's scale
                            sigma_j = sum_i |a_ji| max(|lo|,|hi|); default
                            1e-12 (the paper's 1e-6 is absolute)             */
  int32_t max_search;    /* passes of one 1-D search (default 64)            */
  int32_t max_newton;    /* Newton iterations (default 50)                   */
  int32_t max_ls;        /* line-search trials per iteration (default 12)    */
  int32_t search;        /* pgdto_search                                     */
  int32_t ncp;           /* pgdto_ncp                                        */
  int32_t stage1;        /* COUPLED: 1 = run Stage 1 (default), 0 = skip      */
  double c1, c2;         /* Armijo / curvature constants (1e-4, 0.9)         */
  int32_t compact;       /* 1-D searches: 1 = free-set compaction
                            (Sec. 4.2.1, the remark that saturated variables
                            add nothing to the Jacobian): once a row's bracket
                            lies within 25% of its upper end, each whole tile
                            folds the elements whose state (below / inside /
                            above the box) is the same at both bracket ends
                            into three sums and later passes stream only the
                            other elements' (y, a) pairs, kept in scratch:
                            x for a projection, pgdto_pgd_args.work for an
                            Algorithm 3 step (no compaction without it);
                            0 (default) = every pass streams every element.
                            Results agree to rounding; every route
                            (one-instance, batch, served) gives the same
                            bits for one setting.  A separate kernel
                            instantiation, so the default keeps its
                            registers                                        */
} pgdto_params;

typedef struct {
  int32_t outcome;       /* pgdto_outcome, worst over rows/blocks            */
  int32_t path;          /* 0 box only, 1 bracket search, 2 Stage-1 exit,
                            3 Newton                                         */
  int32_t passes;        /* streaming passes over y and A (incl. final)      */
  int32_t iters_search;  /* 1-D search passes (max over rows/blocks)         */
  int32_t iters_newton;  /* Newton iterations                                */
  int32_t iters_ls;      /* line-search trials (Newton passes)               */
  int32_t m;             /* rows / blocks                                    */
  int32_t error;         /* 0, or PGDTO_ERR_TIMEOUT if a device wait expired */
  int64_t n_free;        /* elements with lo <= z_i <= hi                    */
  double lambda[PGDTO_MAX_BLOCKS];  /* multipliers (>= 0; equality rows: any sign) */
  double resid[PGDTO_MAX_BLOCKS];   /* a_j.x - b_j with x as stored          */
  double slack[PGDTO_MAX_BLOCKS];   /* kappa lam_j (eq. s_y_robust)          */
  int32_t row_outcome[PGDTO_MAX_BLOCKS];
  double res_inf;        /* max_j scaled KKT residual of x as stored:
                            |h_j| / sigma_j for rows with lambda_j != 0 and
                            equality rows, max(h_j, 0) / sigma_j otherwise,
                            h_j = a_j.x - b_j - kappa lambda_j, sigma_j =
                            sum_i |a_ji| max(|lo|, |hi|)                   */
  double lambda_width;   /* width of the final bracket of the 1-D searches
                            (max over rows; a root of the computed dual
                            function lies in it), 0 when no search ran      */
  double kappa;          /* regularization used: 2/C, or the automatic value */
  /* Stated error of the result against the exact solution of the problem
   * as given (Theorems 1 and 2: x and lambda are unique when kappa > 0).
   * lambda_err[j]: 2 |h_j| / slope_j at the last evaluated point of a 1-D
   * search (capped by its bracket width), or 2 |Delta_j| for the Newton
   * step that the float64 factor of (A D A^T + kappa I) on the active rows
   * gives at the returned multipliers, plus 16 float64 rounding units of
   * |lambda_j| and of sigma_j / slope_j; INFINITY when the slope is zero (a
   * flat stretch of the dual, kappa = 0: lambda is not unique there, x is).
   * x_err: sum_j max_i |a_ji| lambda_err[j] (max over blocks for
   * independent blocks) plus half a unit in the last place of the stream
   * dtype at max(|lo|, |hi|): a bound on max_i |x_i - x*_i|. */
  double lambda_err[PGDTO_MAX_BLOCKS];
  double x_err;
  int64_t n_compact;     /* 1-D searches: elements the free-set compaction kept
                            for the later passes (summed over rows / blocks;
                            see pgdto_params.compact); -1 when none ran      */
  int32_t passes_compacted;  /* search passes that streamed only the kept
                            elements (max over rows / blocks)                */
  int32_t reserved;
  double dist2;          /* ||x - y||_2^2 of x as stored: the distance the
                            projection moved the point (y = rho~ for a step) */
} pgdto_result;

typedef struct {
  pgdto_problem proj;    /* A = grad g(rho_t); proj.y and proj.b are ignored
                            (formed on the device); proj.x receives rho_{t+1} */
  const void* rho;       /* device [n] rho_t                                  */
  const void* rho_prev;  /* device [n] rho_{t-1} (ignored at t = 0)           */
  const void* grad;      /* device [n] grad f(rho_t)                          */
  const void* grad_prev; /* device [n] grad f(rho_{t-1}) (ignored at t = 0)   */
  void* dir;             /* device [n]: in d_{t-1}, out d_t (in place)        */
  const double* g;       /* host [m] g_j(rho_t)                               */
  const double* G;       /* host [m] bounds G_j                               */
  int64_t t;             /* iteration index                                   */
  int32_t t_warmup;      /* 50                                                */
  int32_t cg_rule;       /* pgdto_cg_rule                                     */
  double alpha_max;      /* 1e2                                               */
  double alpha_fallback; /* 0.2                                               */
  double omega;          /* 1.0                                               */
  double eps_alpha;      /* 1e-6                                              */
  double tol_viol;       /* tol_N of the fallback rule (1e-6)                 */
  double tol;            /* stop test ||rho_{t+1}-rho_t|| / ||rho_{t+1}||     */
  void* work;            /* optional device [n] of the stream dtype: scratch
                            for the free-set compaction (see pgdto_params.
                            compact); NULL: none.  May be the caller's
                            rho_prev or grad_prev buffer (they are read only
                            in the first pass); must not overlap x, dir, rho
                            or grad                                          */
} pgdto_pgd_args;

typedef struct {
  double alpha, beta;    /* step size and conjugate coefficient used          */
  double rel_change;     /* ||rho_{t+1} - rho_t||_2 / ||rho_{t+1}||_2         */
  int32_t used_fallback; /* 1 if alpha = min(alpha_max, alpha_fb/||grad||_inf)*/
  int32_t converged;     /* rel_change <= tol                                 */
  pgdto_result proj;     /* the projection's result (x = rho_{t+1})           */
} pgdto_pgd_out;

typedef struct pgdto_ctx pgdto_ctx;
typedef struct pgdto_batch pgdto_batch;

/* Defaults listed above (paper Sec. 3.5 where the paper fixes them). */
void pgdto_params_default(pgdto_params* p);
void pgdto_pgd_args_default(pgdto_pgd_args* a);

/* Create a context on HIP device `device`: allocates the fixed workspace
 * (per-tile partial sums, barrier words, result staging) once. */
int pgdto_ctx_create(int device, pgdto_ctx** out);
int pgdto_ctx_destroy(pgdto_ctx* ctx);

/* Grid autotuner (also on when the environment variable PGDTO_AUTOTUNE is
 * set at creation).  enable > 0: the first blocking pgdto_project of each
 * shape class (kind, dtype, m, tile count) times the launch at all
 * co-resident workgroups and at 1/2, 1/4, 1/8 of them on the caller's stream
 * and keeps the fastest for the class (later calls of the class, async and
 * pgd_step included, use it); 0: stop tuning, keep choices; < 0: stop and
 * forget.  Results do not depend on the choice (bitwise).  Returns the
 * previous setting or PGDTO_ERR_ARG. */
int pgdto_ctx_autotune(pgdto_ctx* ctx, int enable);
/* Persist the autotuner's choices across processes: save writes every shape
 * class tuned on this context to the text file `path` (a header with the
 * library version and the device's architecture and compute-unit count,
 * then one "class grid" line each) and returns how many; load adds the
 * choices of such a file to the context and returns how many (0 when the
 * file was written for another device or library version).  PGDTO_ERR_ARG
 * for a file that cannot be opened. */
int pgdto_ctx_autotune_save(pgdto_ctx* ctx, const char* path);
int pgdto_ctx_autotune_load(pgdto_ctx* ctx, const char* path);
/* Three more environment variables read at context creation, for studies
 * of the launch (results do not depend on any of them, bitwise):
 *   PGDTO_GRID=k       one-instance launches use at most k workgroups (the
 *                      size of a server slot, traced in isolation);
 *   PGDTO_DOOR_WAIT=t  the kernel's arrival door waits at most t ticks of the
 *                      100 MHz clock for the whole grid before it closes
 *                      (default 3000 = 30 us; 0 closes it at the first
 *                      arrival, so that fewer workgroups take part);
 *   PGDTO_REDUCE_WG0=1 one-instance launches reduce each pass's tile partials
 *                      in workgroup 0 alone, which publishes the totals with
 *                      a go word (the form of launches of more than 256
 *                      workgroups), instead of in every workgroup. */
/* Workgroups and tiles of the context's last launch. */
int pgdto_ctx_last_launch(pgdto_ctx* ctx, int32_t* grid, int32_t* tiles);

/* Project (Alg. 1 / Alg. 2).  Enqueues one launch on `stream` and waits
 * for it; *out is filled on return.  params may be NULL. */
int pgdto_project(pgdto_ctx* ctx, const pgdto_problem* prob, const pgdto_params* params,
                  pgdto_result* out, void* stream);

/* Same, without waiting: the result struct is written to `result_dev`
 * (device memory, sizeof(pgdto_result) bytes, caller-owned) when the launch
 * completes in stream order.  Host arrays (b, block_offsets) are read before
 * the call returns.  The call enqueues exactly one kernel launch (no copy or
 * memset), so it may be captured into a HIP graph: every replay runs as a
 * new launch (the kernel takes its barrier epochs from a device-side
 * counter of the context), with the b and offsets of the captured call.
 * Launches on one context must not overlap in time (one stream, or ordered
 * streams). */
int pgdto_project_async(pgdto_ctx* ctx, const pgdto_problem* prob, const pgdto_params* params,
                        pgdto_result* result_dev, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * projection of pgdto_project_async with no context.  Its workspace
 * (per-tile partial sums, barrier and arrival-door words;
 * PGDTO_NOALLOC_SCRATCH_BYTES) is a static array of the library in device
 * memory, one copy per GPU, held until the process ends.  The call allocates
 * nothing: no hipMalloc, hipFree or allocating library routine.  It runs on
 * the calling thread's current HIP device; `stream` must belong to it.  The
 * first call on a device looks up that device's copy of the array and clears
 * it with one small kernel on `stream` (enqueued before the solve); every
 * later call enqueues the solve kernel only, like pgdto_project_async.  The
 * result struct is written to `result_dev` (device memory, caller-owned);
 * params may be NULL.  Every call on one GPU shares that GPU's array, which
 * keeps the last call's contents: calls that overlap in time on one GPU race
 * (issue them on one stream, or order their streams).  The array holds the
 * tile table of every problem the ABI accepts (at most 704 tiles of at most
 * 112 partial values); a problem beyond it returns PGDTO_ERR_SCRATCH before
 * anything is launched.  Argument errors: PGDTO_ERR_ARG, as for
 * pgdto_project_async. */
#define PGDTO_NOALLOC_SCRATCH_BYTES 1466752
int pgdto_project_noalloc(const pgdto_problem* prob, const pgdto_params* params, pgdto_result* result_dev,
                          void* stream);

/* kappa-continuation (Appendix A.2, the closing remark on choosing C: for
 * an infeasible subproblem C trades constraint violation against the
 * distance the projection moves the point).  Solves prob at each penalty
 * C_values[0..count-1] (count 1..64; each > 0 or INFINITY, or < 0 for the
 * automatic choice with tolerance -C), in that order, each solve
 * warm-started from the previous point's multipliers (the first from
 * prob->lambda0 when given), and fills points[i] (host memory).  prob->x
 * holds the last point's x on return.  tau > 0 also states each point's
 * worst violation against that tolerance (0: not stated).  Blocking; one
 * launch per point.  PGDTO_ERR_ARG for an invalid problem or list. */
typedef struct {
  double C, kappa;                         /* penalty asked for and kappa used     */
  double dist;                             /* ||x - y||_2 of x as stored           */
  double max_violation;                    /* max_j violation[j]                   */
  double violation_over_tau;               /* max_violation / tau (0 if tau = 0)   */
  int32_t outcome, passes;
  double lambda[PGDTO_MAX_BLOCKS];         /* multipliers                          */
  double slack[PGDTO_MAX_BLOCKS];          /* kappa lambda_j: the violation the
                                              regularized problem allows (eq. s_y_robust) */
  double violation[PGDTO_MAX_BLOCKS];      /* max(0, a_j.x - b_j) (equality rows:
                                              |a_j.x - b_j|) of x as stored        */
} pgdto_path_point;
int pgdto_kappa_path(pgdto_ctx* ctx, const pgdto_problem* prob, const pgdto_params* params, const double* C_values,
                     int count, double tau, pgdto_path_point* points, void* stream);

/* One body of Algorithm 3 (step size, direction, rho~, projection, stop test),
 * one launch; waits and fills *out.  The _async form writes the
 * pgdto_pgd_out to device memory and, like pgdto_project_async, enqueues a
 * single kernel launch that may be captured into a HIP graph and replayed. */
int pgdto_pgd_step(pgdto_ctx* ctx, const pgdto_pgd_args* args, const pgdto_params* params,
                   pgdto_pgd_out* out, void* stream);
int pgdto_pgd_step_async(pgdto_ctx* ctx, const pgdto_pgd_args* args, const pgdto_params* params,
                         pgdto_pgd_out* out_dev, void* stream);

/* Batching: `count` (1..256) float32 instances solved by ONE persistent
 * cooperative launch on `stream`, the GPU split into `slots` slots of equal
 * workgroup ranges (0: min(count, 16)); slot s solves instances s, s + slots,
 * ... in order, each with the solver of a one-instance launch on its own
 * workgroups, so every instance's result is bitwise that of pgdto_project
 * (pgdto_pgd_step) on the same problem.  Results go to results_dev[i]
 * (device memory, caller-owned, written when the launch completes in stream
 * order).  Instances must not share output buffers (x, free_mask, dir).
 * Host arrays are read before the call returns.  The context keeps the
 * per-slot workspace (grown on the first call that needs more slots: that
 * call synchronises the device and allocates) and BATCH_RING = 4 pinned
 * descriptor areas used in turn (a call waits for the launch four calls back
 * before it rewrites that area).  Not for HIP graph capture: the kernel reads
 * descriptors the host writes per call.  PGDTO_ERR_ARG for a float64
 * instance, count out of range or any invalid instance (nothing launched). */
int pgdto_project_batch_async(pgdto_ctx* ctx, const pgdto_problem* probs, int count, const pgdto_params* params,
                              pgdto_result* results_dev, int slots, void* stream);
/* The same for Algorithm 3 steps (pgdto_pgd_step_async per instance). */
int pgdto_pgd_step_batch_async(pgdto_ctx* ctx, const pgdto_pgd_args* args, int count, const pgdto_params* params,
                               pgdto_pgd_out* outs_dev, int slots, void* stream);

/* Serving: continuous batching of projection and Algorithm 3 requests.
 *
 * max_slots != 1 selects the persistent executor: one long-running
 * cooperative launch whose workgroups form max_slots slots; each slot solves
 * one request at a time and claims the next published request as soon as it
 * finishes, so requests that arrive while others run are admitted as slots
 * and budget free up, and requests of different sizes overlap on the device.
 * Results are bitwise those of pgdto_project on the same problem.  The
 * launch holds the GPU while requests are outstanding and ends a few ms
 * after the last one; other launches on the device wait meanwhile.  The
 * persistent executor takes float32 streams only (a float64 request fails
 * with PGDTO_ERR_ARG).  max_slots == 1 selects the plain one-at-a-time path:
 * FIFO, one full-GPU launch per request (any dtype). */
typedef struct {
  size_t hbm_budget_bytes;   /* admission limit on the summed footprint of the
                                requests in flight (0: 90% of free memory)    */
  int32_t max_slots;         /* 1: plain path; 0: 8 slots; else slot count   */
  int32_t wg_per_slot;       /* workgroups per slot (0: all that fit / slots) */
  int32_t queue_capacity;    /* pending requests (0: 65536)                   */
  int32_t slots_only;        /* persistent executor: non-zero sends a lone
                                request to a slot too (default: a lone request
                                with nothing else on the device runs as one
                                full-GPU launch; same bits either way)        */
} pgdto_batch_cfg;

int pgdto_batch_create(pgdto_ctx* ctx, const pgdto_batch_cfg* cfg, pgdto_batch** out);
/* Non-blocking.  The problem's device buffers must hold their data when
 * this is called (the executor may start on them at once, in no stream
 * order: finish the work that writes y and A first) and stay valid until
 * poll returns PGDTO_OK or an error for this ticket.  free_mask need not be
 * cleared by the caller.  Host arrays are copied. */
int pgdto_batch_submit(pgdto_batch* b, const pgdto_problem* prob, const pgdto_params* params,
                       uint64_t* ticket);
/* An Algorithm 3 step (as pgdto_pgd_step) as a served request: the same
 * contract as pgdto_batch_submit for its device buffers (rho_t, rho_{t-1},
 * grad, grad_{t-1}, d: read; d and x: written; all ready at submit and kept
 * valid until the ticket retires); g, G, block offsets and lambda0 are copied.  Poll it
 * with pgdto_batch_poll_pgd (pgdto_batch_poll returns its projection part). */
int pgdto_batch_submit_pgd(pgdto_batch* b, const pgdto_pgd_args* args, const pgdto_params* params,
                           uint64_t* ticket);
/* PGDTO_QUEUED / PGDTO_PENDING / PGDTO_OK (result copied, ticket retired) /
 * error.  Thread-safe. */
int pgdto_batch_poll(pgdto_batch* b, uint64_t ticket, pgdto_result* out);
/* Blocks until the ticket finishes (or errors). */
int pgdto_batch_wait(pgdto_batch* b, uint64_t ticket, pgdto_result* out);
/* pgdto_batch_poll (wait == 0) or pgdto_batch_wait (wait != 0) that also
 * returns, when the ticket retires, times[0..2] = submitted, admitted to the
 * device, completion seen, in ns on the host's monotonic clock. */
int pgdto_batch_poll_timed(pgdto_batch* b, uint64_t ticket, pgdto_result* out, int64_t* times, int wait);
/* pgdto_batch_poll_timed for any ticket, returning the whole Algorithm 3
 * output (a projection ticket fills out->proj only).  times may be NULL. */
int pgdto_batch_poll_pgd(pgdto_batch* b, uint64_t ticket, pgdto_pgd_out* out, int64_t* times, int wait);
/* Executor shape: slots and workgroups per slot (0, 0 on the plain path). */
int pgdto_batch_shape(pgdto_batch* b, int32_t* slots, int32_t* wg_per_slot);
/* Shape autotuner for the persistent executor (blocks per instance).  Runs
 * `count` float32 requests, taken round-robin from samples[0..nsamples-1]
 * (distinct instances, so that inputs are not all served from cache), all
 * submitted at once, through executors of PGDTO_TUNE_SHAPES candidate
 * shapes: 4, 8, 16, 32, 64 slots, each with the co-resident workgroups split
 * evenly; every shape runs twice and its faster run counts.  Writes the
 * fastest shape to *slots, *wg_per_slot (for pgdto_batch_cfg.max_slots and
 * wg_per_slot) and, when times_ms is not NULL, the wall time of each
 * candidate (first submit to last completion, ms; INFINITY for a shape the
 * device cannot hold) to times_ms[0..PGDTO_TUNE_SHAPES-1].  Blocking.  The
 * samples follow the pgdto_batch_submit contract for their buffers; their x
 * is written (by several requests at once, with the same values) and their
 * free_mask is ignored.  PGDTO_ERR_ARG for a bad argument or a float64
 * sample; otherwise the first error of a request. */
#define PGDTO_TUNE_SHAPES 5
int pgdto_batch_autotune(pgdto_ctx* ctx, const pgdto_problem* samples, int nsamples,
                         const pgdto_params* params, int count, int32_t* slots, int32_t* wg_per_slot,
                         float* times_ms);
/* Statistics: admitted, completed, queued, in flight, peak footprint. */
int pgdto_batch_stats(pgdto_batch* b, int64_t* admitted, int64_t* completed, int64_t* queued,
                      int64_t* in_flight, int64_t* peak_bytes);
/* Cancels queued requests, waits for in-flight ones, releases resources. */
int pgdto_batch_destroy(pgdto_batch* b);

/* Host-only validation of a projection request: the checks pgdto_project,
 * pgdto_project_async and pgdto_batch_submit make before anything is
 * launched (kinds, sizes, alignment of the device pointers, box, C,
 * eq_mask, lambda0, block offsets, params; params may be NULL for the
 * defaults).  No
 * device memory is read and no device is needed.  PGDTO_OK or
 * PGDTO_ERR_ARG. */
int pgdto_problem_check(const pgdto_problem* prob, const pgdto_params* params);
const char* pgdto_status_string(int status);
int pgdto_version(void);

/* Tracing: when the environment variable PGDTO_TRACE is set (non-zero) at
 * context creation, every launch records, per streaming pass, eight 64-bit
 * values on the device's 100 MHz clock: workgroup 0's (phase << 56 | pass
 * start), element loop done, all flags seen, totals reduced, synchronisation
 * left, control done; the last workgroup's loop done and totals seen (these
 * two only in launches of more than 256 workgroups, where workgroup 0 reduces
 * the pass alone and the others wait for its totals).  This
 * copies up to max_records records (8 values each) of the last launch to host
 * memory `out` and clears them; returns the number of records copied
 * (0 when tracing is off) or a negative status.  With max_records < 0 it
 * instead copies the per-workgroup table of the first 16 passes, 16 x 1024 x 4
 * values (loop start, loop end, wait end, HW_ID | XCC_ID << 32), into `out`
 * (65536 values) and returns 16. */
int pgdto_trace_read(pgdto_ctx* ctx, uint64_t* out, int max_records);

/* Layout introspection for language bindings: sizeof of the public structs.
 * which: 0 pgdto_problem, 1 pgdto_params, 2 pgdto_result, 3 pgdto_pgd_args,
 * 4 pgdto_pgd_out, 5 pgdto_batch_cfg, 6 pgdto_path_point.  Returns 0 for an
 * unknown index. */
size_t pgdto_struct_size(int which);

#ifdef __cplusplus
}
#endif
#endif /* PGDTO_H */
