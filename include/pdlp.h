/*
 * libpdlp -- PDLP (restarted, diagonally preconditioned primal-dual hybrid gradient) for the LP
 * relaxation of a MIP, on one AMD Instinct MI355X (gfx950).
 *
 * The problem is the LP of eq. (1) of the paper (Introduction):
 *     min c'x  s.t.  a_i'x <= b_i,  l <= x <= u,  l, u in R u {+-inf},
 * widened to per-row senses 'L' (<=), 'G' (>=) and 'E' (=) because the energy system models
 * (section "Energy system optimization models") carry balance equalities. The solver returns the
 * primal x, the duals y and the reduced costs r = c - A'y, which are what the LP-based variable and
 * value strategies of section 2 consume ("LP-based variable strategies", "LP-based fixing"). The
 * paper solves this relaxation with GPU PDLP to a low relative tolerance (1e-4, or 1e-6; section 4,
 * "Numerical results" and Table 8); 1e-4 is the default here.
 *
 * Sign convention of the duals: Lagrangian c'x - y'(Ax - b), so y_i >= 0 on 'G' rows, y_i <= 0 on
 * 'L' rows and y_i free on 'E' rows.
 *
 * Conventions for every entry point:
 *   - Return value 0 = success, negative = error (PDLP_ERR_*). No C++ exception crosses the ABI.
 *     pdlp_error_string() names a code; pdlp_last_error() gives detail for the calling thread.
 *   - Ownership: pdlp_create deep-copies every input; no caller pointer is retained. The handle owns
 *     all device memory it allocates and releases it in pdlp_destroy. Output buffers belong to the
 *     caller and are written by pdlp_get.
 *   - Pointers are host pointers unless pdlp_options.device_ptrs is set, in which case the CSR and
 *     vector arguments of pdlp_create and the warm start of pdlp_solve are device pointers on the
 *     handle's device (for example the data pointers of torch tensors).
 *   - All work is ordered on pdlp_options.stream (a hipStream_t; NULL = the library creates one).
 *     pdlp_solve and pdlp_get return after the stream has finished their work.
 *   - Determinism: the same input and options on the same GPU give bitwise identical results
 *     for a given chunk size, and an instance of a batch gets the bits it gets solved alone. With
 *     tile_nnz = 0 the chunk size is 512 unless, for 200,000 or more nonzeros, timing finds another
 *     candidate at least 15 % faster; set tile_nnz to pin it across processes.
 *   - Calls on one handle must not overlap; different handles are independent.
 */
#ifndef PDLP_H_
#define PDLP_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes (negative) -------------------------------------------------------------- */
#define PDLP_OK 0
#define PDLP_ERR_ARG (-1)   /* bad argument: NULL pointer, negative size, NaN data, l > u, bad sense */
#define PDLP_ERR_CSR (-2)   /* malformed CSR: row_ptr not monotone, column out of range, duplicate */
#define PDLP_ERR_OOM (-3)   /* device allocation failed or exceeded pdlp_options.device_mem_limit */
#define PDLP_ERR_HIP (-4)   /* a HIP runtime call failed */
#define PDLP_ERR_STATE (-5) /* call out of order, e.g. pdlp_get before pdlp_solve */

/* ---- solve status (pdlp_result.status) -------------------------------------------------- */
#define PDLP_STATUS_NONE 0
#define PDLP_STATUS_OPTIMAL 1    /* relative KKT error <= tol in the original space */
#define PDLP_STATUS_ITER_LIMIT 2 /* iteration limit reached; the current iterate is returned */
#define PDLP_STATUS_NUMERICAL 3  /* a step size or residual became NaN / Inf */

/* ---- precision modes --------------------------------------------------------------------- */
#define PDLP_FP32 0 /* matrix values and iterates FP32, int32 indices; norms, KKT, restart and
                       primal-weight arithmetic FP64 */
#define PDLP_FP64 1 /* everything FP64 */

typedef struct pdlp_options {
  int32_t precision;       /* PDLP_FP32 (default) or PDLP_FP64 */
  int32_t eval_every;      /* attempts between KKT evaluations / restart tests (default 64) */
  int32_t ruiz_iters;      /* Ruiz equilibration passes (default 10) */
  int32_t pock_chambolle;  /* 1 = one Pock-Chambolle pass with alpha = 1 after Ruiz (default 1) */
  int32_t use_graphs;      /* 1 = run each evaluation interval as one captured hipGraph (default 1) */
  int32_t device_ptrs;     /* 1 = data pointers are device pointers (default 0) */
  int32_t tile_nnz;        /* SpMV chunk size cap in nonzeros (512, 1024, 2048 or 4096);
                              0 = autotune (default 0) */
  int32_t verbose;         /* 0 silent, 1 one line per solve, 2 also one line per evaluation (the
                              first four instances; stderr) */
  int64_t device_mem_limit;/* > 0: cap on the bytes this handle may allocate (default 0 = none) */
  void *stream;            /* hipStream_t to order work on; NULL = library-owned stream */
  int32_t warm_fallback;   /* what happens to a warm start whose relative KKT error is not below
                              the cold start's: 2 = its point is replaced by the cold point and a
                              given omega0 is kept (default 2); 1 = the cold start in full (the
                              default primal weight too); 0 = the warm start is kept */
  int32_t kernel_timing;   /* 1 = time every launch of the iteration kernels with HIP events that
                              their own dispatches record (start and stop; graphs are not used then);
                              read the totals with pdlp_kernel_stats (default 0) */
  int32_t work_blocks;     /* most blocks per SpMV kernel for one instance (each block owns a
                              contiguous run of chunks; an instance gets one block per 1024 nonzeros
                              + rows up to this count); 0 = 16384 (default 0) */
  int32_t single_avg_updates; /* FP32 pairs the running-average updates of consecutive accepted
                              attempts (one pass over x-bar and y-bar for two updates); 1 = update on
                              every accepted attempt instead. Both give the same bits (default 0) */
  int32_t panel_rows;      /* FP32: rows of A with at least this many nonzeros are summed by column
                              panels (x held in LDS panel by panel, per-panel row sums added in panel
                              order) when such rows carry at least half of an instance's nonzeros;
                              0 = 64 (default 0), -1 = never. FP64 handles always use the chunk
                              engine */
  int32_t col_blocks;      /* FP32: A'y of an instance by column blocks (a work group owns 4096
                              columns and reads y in 16384-row panels held in LDS, the rows past the
                              dense panels gathered) instead of the chunk engine. 0 = for every
                              instance whose longest column has at most 64 nonzeros when the handle
                              holds at least 2^20 nonzeros in all (default 0); 1 = for every instance
                              the layout allows; -1 = never. An instance on column blocks that has
                              no column-panel rows and at most 131072 columns also forms A x' by row
                              blocks (a work group owns 4096 rows and reads x in 16384-column panels
                              held in LDS). A single-LP handle reproduces a batch member's trajectory
                              bit for bit when it takes the same choice for the instance (with 1 or
                              -1 as the batch's rule decided) */
  int32_t reserved[2];
} pdlp_options;

typedef struct pdlp_result {
  int32_t status;          /* PDLP_STATUS_* */
  int32_t restarts;        /* number of restarts */
  int64_t iterations;      /* PDHG attempts (accepted and rejected steps) */
  double rel_primal;       /* |r_p| / (1 + |b|), original space, FP64 */
  double rel_dual;         /* |r_d| / (1 + |c|) */
  double rel_gap;          /* |pobj - dobj| / (1 + |pobj| + |dobj|) */
  double primal_obj;       /* c'x */
  double dual_obj;         /* b'y + sum_{l finite} l_j lambda_j^+ - sum_{u finite} u_j lambda_j^- */
  double omega;            /* final primal weight (scaled space) */
  double eta;              /* final step size (scaled space) */
  double solve_seconds;    /* wall time of the last pdlp_solve */
  int32_t used_average;    /* 1 = the returned point is the weighted average iterate */
  int32_t warm_started;    /* 1 = a warm start was used, 0 = cold (including fallback) */
  int32_t fallback_used;   /* 1 = the warm start was rejected in favour of the cold start */
  int32_t final_checks;    /* how many times the FP64 re-check of the returned point ran */
} pdlp_result;

typedef struct pdlp_problem pdlp_problem;

/* Fill *opt with the defaults listed above. */
void pdlp_options_default(pdlp_options *opt);

/*
 * Create a solver handle for the LP (eq. (1) with row senses).
 *   m, n        rows and columns (m >= 0, n >= 0; nnz < 2^31)
 *   row_ptr     [m+1] int32 CSR row offsets, row_ptr[0] = 0, nondecreasing
 *   col_idx     [nnz] int32 column indices, strictly increasing within a row (no duplicates)
 *   val         [nnz] float64 values, finite
 *   c           [n] objective, finite;  b [m] right-hand sides, finite
 *   sense       [m] 'L', 'G' or 'E'
 *   l, u        [n] bounds, -inf <= l <= u <= +inf (NaN rejected)
 *   opt         NULL = defaults
 * On success *out receives the handle. The matrix is copied to the device, its transpose is built
 * there, both are equilibrated (10 Ruiz passes and one Pock-Chambolle pass) and the SpMV schedule
 * is chosen.
 */
int pdlp_create(pdlp_problem **out, int32_t m, int32_t n, int64_t nnz, const int32_t *row_ptr,
                const int32_t *col_idx, const double *val, const double *c, const double *b,
                const char *sense, const double *l, const double *u, const pdlp_options *opt);

/*
 * Solve to relative KKT tolerance tol (<= 0 means run to iter_limit) within iter_limit attempts.
 * x0 [n] / y0 [m] optional warm start in the original space (NULL = cold start at the projection
 * of 0); omega0 > 0 sets the initial primal weight (otherwise |c~|/|b~|). A warm start is projected
 * onto the bounds and sign sets; with warm_fallback set its point is replaced by the cold start's
 * when its relative KKT error is not smaller (see pdlp_options.warm_fallback for omega0). Each call
 * starts a fresh solve from its own start point.
 */
int pdlp_solve(pdlp_problem *p, double tol, int64_t iter_limit, const double *x0, const double *y0,
               double omega0);

/*
 * Copy the solution of the last pdlp_solve into caller buffers (each may be NULL):
 *   x [n] primal, y [m] duals, red_cost [n] = c - A'y, all float64 in the original space;
 *   res receives the status and FP64 residuals of the returned point.
 */
int pdlp_get(pdlp_problem *p, double *x, double *y, double *red_cost, pdlp_result *res);

/*
 * y = A x (trans = 0, x [n], y [m]) or y = A' x (trans = 1, x [m], y [n]) with the ORIGINAL
 * (unscaled) matrix, computed by the library's SpMV kernels in the handle's precision on the
 * handle's stream. trans = 2 computes A x the way the PDHG iteration forms it (FP32 handles sum
 * the long rows of A by column panels, see pdlp_options.panel_rows, and the rows of narrow
 * instances on column blocks by row blocks, see pdlp_options.col_blocks; otherwise the same as 0), and
 * trans = 3 computes A'x the way it does (FP32 handles may sum columns by column blocks, see
 * pdlp_options.col_blocks; otherwise the same as 1). x and y are host pointers unless device_ptrs
 * is set.
 */
int pdlp_spmv(pdlp_problem *p, int32_t trans, const double *x, double *y);

/*
 * Scaling diagnostics in the caller's numbering: Dr [m] and Dc [n] (A~ = diag(Dr) A diag(Dc)) and,
 * optionally, the scaled matrix values in the caller's CSR order (scaled_val [nnz], FP64). Any pointer
 * may be NULL. Host pointers.
 */
int pdlp_get_scaling(pdlp_problem *p, double *Dr, double *Dc, double *scaled_val);

/*
 * The matrix as stored on the device, for inspection: inside a handle the rows and the columns are
 * renumbered so that rows of A and of A' come sorted by length class (stable within a class).
 * row_ptr [m+1], col [nnz], val [nnz] is the scaled A (FP64) in internal numbering; t_row_ptr [n+1],
 * t_col [nnz], t_val [nnz] its transpose as built on the device; internal row i is the caller's
 * row row_perm[i] and internal column j the caller's column col_perm[j]. Any pointer may be NULL.
 */
int pdlp_get_internal(pdlp_problem *p, int32_t *row_ptr, int32_t *col, double *val, int32_t *t_row_ptr,
                      int32_t *t_col, double *t_val, int32_t *row_perm, int32_t *col_perm);

/* SpMV schedule chosen for A and A': chunk size cap in nonzeros and the number of chunks of each. */
int pdlp_get_schedule(pdlp_problem *p, int32_t *tile_nnz, int32_t *tiles_a, int32_t *tiles_at);

/*
 * Kernel timing of the last pdlp_solve with pdlp_options.kernel_timing = 1.
 *   kernel 0: A x' fused with the dual update and the step-size partial sums (from the start of the
 *             first to the end of the last of its launches: k_dual and / or the row-block form)
 *   kernel 1: A'y' fused with the primal update and the iterate averages
 *   kernel 2: the column-panel sums of the long rows of A x' (launched before kernel 0 when the
 *             handle uses column panels; no launches otherwise)
 *   kernel 3: the same launches and durations as kernel 1, counted only when kernel 1 includes the
 *             column-block form of A'y' (see pdlp_options.col_blocks; no launches otherwise)
 *   kernel 4: the same launches and durations as kernel 0, counted only when kernel 0 includes the
 *             row-block form of A x' (see pdlp_options.col_blocks; no launches otherwise)
 * (the step-size decision itself runs in a small per-instance kernel between them and is not timed)
 * *launches receives the number of launches, *total_ms their summed HIP-event durations.
 */
int pdlp_kernel_stats(pdlp_problem *p, int32_t kernel, int64_t *launches, double *total_ms);

/* Bytes of device memory held by the handle. */
int64_t pdlp_device_bytes(const pdlp_problem *p);

void pdlp_destroy(pdlp_problem *p);

const char *pdlp_error_string(int code);
const char *pdlp_last_error(void);

/* ==========================================================================================
 * Batched solve: many independent LPs of uneven sizes solved together, as the repeated LP
 * solves the paper mentions (periodic re-solves, section 2) and as training data for the warm-start
 * model need. Each instance follows exactly the single-instance method; instances share launches.
 * ========================================================================================== */
typedef struct pdlp_problem_desc {
  int32_t m, n;
  int64_t nnz;
  const int32_t *row_ptr;
  const int32_t *col_idx;
  const double *val;
  const double *c, *b;
  const char *sense;
  const double *l, *u;
} pdlp_problem_desc;

typedef struct pdlp_batch pdlp_batch;

/* Create a batch handle for k problems (host pointers). Validation as in pdlp_create. */
int pdlp_batch_create(pdlp_batch **out, int32_t k, const pdlp_problem_desc *descs,
                      const pdlp_options *opt);

/* Solve every instance to tol within iter_limit attempts each. x0s/y0s: NULL or arrays of k
 * pointers (entries may be NULL) to warm starts; omega0s: NULL or k values (<= 0 = default). */
int pdlp_batch_solve(pdlp_batch *bt, double tol, int64_t iter_limit, const double *const *x0s,
                     const double *const *y0s, const double *omega0s);

/* Solution of instance i (0 <= i < k), as pdlp_get. */
int pdlp_batch_get(pdlp_batch *bt, int32_t i, double *x, double *y, double *red_cost,
                   pdlp_result *res);

/* Re-solves after fixings (fix-and-propagate changes bounds and solves a final LP on them; the paper
 * does that with an IPM and names PDLP for it as future work; section 2 and the conclusion): replace the column bounds
 * l [n], u [n] (caller's numbering, validated as in pdlp_create; device pointers when the handle has
 * device_ptrs) of a handle, or of instance i of a batch. Matrix, costs, scaling and the SpMV
 * schedule are kept, so this costs one small upload instead of a new handle; a following solve is
 * bitwise the one a new handle created with these bounds would give (same options and chunk size),
 * and may be warm-started from the previous solution (x0/y0 of pdlp_solve / pdlp_batch_solve). */
int pdlp_update_bounds(pdlp_problem *p, const double *l, const double *u);
int pdlp_batch_update_bounds(pdlp_batch *bt, int32_t i, const double *l, const double *u);

/* SpMV schedule of the batch, as pdlp_get_schedule (chunk counts over all instances). An
 * instance's chunks and work blocks depend on the instance and the chunk size alone, so a single
 * problem created with pdlp_options.tile_nnz set to this chunk size (and the same other options)
 * follows the instance's trajectory bit for bit. */
int pdlp_batch_get_schedule(pdlp_batch *bt, int32_t *tile_nnz, int32_t *tiles_a, int32_t *tiles_at);

void pdlp_batch_destroy(pdlp_batch *bt);

/* ==========================================================================================
 * Reference snapshots: several LP reference solutions from one solve. The paper's conclusion
 * (section 5) proposes using the cycling convergence of PDLP to start several fix-and-propagate
 * searches from one LP solve. A snapshot is a restart point of the solve (the candidate of the
 * evaluation step, every eval_every attempts, that the method restarts to: the current iterate or the
 * average) whose relative KKT error in the original space, as that evaluation measured it, is at
 * most rel_tol. Each instance keeps the newest k of them; taking them does not change the solve
 * (its iterates and result are bitwise those of a solve without snapshots).
 * ========================================================================================== */

/* Keep up to k snapshots per instance (k = 0: none, the default) in later solves of the handle
 * (pdlp_set_snapshots) or of every instance of the batch (pdlp_batch_set_snapshots). Allocates
 * k (n + m) doubles of device memory (n, m: all instances) under device_mem_limit and replaces the
 * previous setting and snapshots. Each solve starts with no snapshots. Errors: PDLP_ERR_ARG for a
 * NULL handle, k < 0 or a NaN rel_tol; PDLP_ERR_OOM. */
int pdlp_set_snapshots(pdlp_problem *p, int32_t k, double rel_tol);
int pdlp_batch_set_snapshots(pdlp_batch *bt, int32_t k, double rel_tol);

/* Snapshots of the last solve (of instance i of a batch), oldest first: at most cap of them (the
 * newest cap when more are held); *count (host memory, required) = the number written. Per
 * snapshot s < *count: x[s n .. s n + n) and y[s m .. s m + m) the point in the original space and
 * the caller's numbering (n, m of this instance; host memory, or device memory when the handle has
 * device_ptrs; either may be NULL), attempt[s] the attempt count at which it was taken and
 * rel_kkt[s] its relative KKT error as measured then (host memory; either may be NULL). In FP32 the
 * evaluation works from the FP32 products A x and A'y, and an average enters the restart point
 * rounded to FP32 (the snapshot is that rounded point); unlike the returned solution, snapshots are
 * not re-checked in FP64, so an FP64 evaluation of a snapshot can differ from rel_kkt[s] by that
 * rounding. Errors: PDLP_ERR_STATE before a solve; PDLP_ERR_ARG for cap < 0, a NULL count or i out
 * of range. */
int pdlp_get_snapshots(pdlp_problem *p, int32_t cap, double *x, double *y, int64_t *attempt, double *rel_kkt,
                       int32_t *count);
int pdlp_batch_get_snapshots(pdlp_batch *bt, int32_t i, int32_t cap, double *x, double *y, int64_t *attempt,
                             double *rel_kkt, int32_t *count);

#ifdef __cplusplus
}
#endif
#endif /* PDLP_H_ */
