/*
 * hprlp.h -- C ABI of the MI355X (gfx950) HPR-LP library.
 *
 * The library solves, on one GPU,
 *
 *     min <c, x>  s.t.  A1 x = b1,  A2 x >= b2,  l <= x <= u          (paper, eq. primalLP)
 *
 * with the Halpern Peaceman-Rachford method with semi-proximal terms (Algorithm 2 of
 * "HPR-LP: An implementation of an HPR method for solving linear programming",
 * arXiv 2408.12179), including its restart rule (Section 3.1), its sigma update
 * (Section 3.2, Algorithm 3) and its GPU iteration (Section 3.3, eqs. update-z, update-x,
 * update-y-2).  Every step of the iteration runs in hand-written HIP kernels; the host only
 * takes the scalar decisions made every `check_every` iterations.
 *
 * Conventions shared by every entry point
 *   - Return value: an hprlp_err; 0 on success, negative on error.  The solve outcome is
 *     reported separately (hprlp_status).  After an error, hprlp_last_error(handle) (or
 *     hprlp_last_error(NULL) when no handle exists yet) gives a message.
 *   - Matrix: CSR of A = [A1; A2] with the m1 equality rows first, then the m2 inequality
 *     rows.  rowptr: int64[m+1], rowptr[0] = 0, non-decreasing, rowptr[m] = nnz < 2^31;
 *     colidx: int32[nnz] in [0, n) (order inside a row is free; repeats are rejected);
 *     val: double[nnz].  All of these are HOST pointers and are copied.
 *   - Vectors b[m], c[n], l[n], u[n] are host double arrays; l may hold -INFINITY and u
 *     +INFINITY.  They are copied.
 *   - Device memory: the library never allocates device memory.  The caller passes one
 *     device workspace of at least hprlp_workspace_bytes() bytes (256-byte aligned) and keeps
 *     it alive until hprlp_destroy.  All work of a single-LP handle is ordered on the
 *     caller's HIP stream (a batched handle has a stream of its own, see below).
 *   - Output vectors (x, y, z, iterates) may be host or device pointers; the library detects
 *     which.  They are always in the ORIGINAL (unscaled) space of the problem as given.
 *   - Threads: one call at a time per handle; different handles are independent.
 */
#ifndef HPRLP_H
#define HPRLP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hprlp_handle hprlp_handle;

typedef enum {
    HPRLP_OK = 0,
    HPRLP_EINVAL = -1,       /* null pointer, bad option value, workspace too small      */
    HPRLP_EDIM = -2,         /* bad sizes, rowptr not monotone, column index out of range */
    HPRLP_ENONFINITE = -3,   /* NaN anywhere, or an infinite value in A, b or c           */
    HPRLP_EBOUNDS = -4,      /* l_j > u_j, l_j = +inf or u_j = -inf                       */
    HPRLP_ENOTLOSSLESS = -5, /* FP32 storage of A asked but some A value is not FP32-exact */
    HPRLP_ENOMEM = -6,       /* host allocation failed                                    */
    HPRLP_EHIP = -7,         /* a HIP runtime call failed                                 */
    HPRLP_ESTATE = -8        /* call not valid in the handle's current state              */
} hprlp_err;

typedef enum {
    HPRLP_UNSOLVED = 0,
    HPRLP_OPTIMAL = 1,    /* max(rel_gap, rel_p, rel_d) <= tol (Section 4.1)            */
    HPRLP_ITER_LIMIT = 2,
    HPRLP_TIME_LIMIT = 3,
    HPRLP_NUMERICAL = 4   /* a NaN appeared in the check quantities                     */
} hprlp_status;

/* FP64: A~ stored in FP64, FP64 vectors (the plain solver).
 * MIXED: A stored in FP32 (must be exact), FP32 vectors until the relative KKT residual
 *   reaches tol_switch, then FP64 vectors; checks, restart merit and sigma always in FP64.
 *   In the FP32 phase the iterate is held as FP32 displacements from the FP64 anchor of the
 *   current outer loop (renewed at every restart), and the returned w_bar is FP64. 
 * FP64_A32: A stored in FP32 (must be exact), FP64 vectors throughout: FP64 results with
 *   8 instead of 12 bytes per nonzero (FP32 x FP64 products are exact in FP64). */
typedef enum { HPRLP_FP64 = 0, HPRLP_MIXED = 1, HPRLP_FP64_A32 = 2 } hprlp_precision;

typedef struct {
    double tol;              /* termination tolerance (default 1e-8; Section 4.1)          */
    long long check_every;   /* restart/termination check period (default 150; Sec. 4.1)  */
    long long max_iter;      /* default 10^7                                               */
    double time_limit;       /* seconds, <= 0: none (default 0)                            */
    double alpha1, alpha2, alpha3; /* restart parameters (default 0.2, 0.6, 0.2; Sec. 4.1) */
    double sigma0;           /* initial penalty (default 1; Section 4.1)                   */
    int ruiz_iters;          /* Ruiz passes (default 10; Section 4.1)                      */
    int pock_chambolle;      /* 1: one diagonal Pock-Chambolle pass, alpha = 1 (default 1) */
    int normalize_bc;        /* 1: divide b, c by (||b||+1), (||c||+1) (default 1)         */
    int power_max_iter;      /* power method cap (default 5000)                            */
    double power_tol;        /* relative change of the Rayleigh quotient (default 1e-10)   */
    double lambda_override;  /* > 0: use this lambda, skip the power method                */
    int use_halpern;         /* 1: Halpern averaging (Algorithm 2); 0: plain PR iteration  */
    int use_restart;         /* 1: restart criteria of Section 3.1                         */
    int sigma_update;        /* 1: SigmaUpdate (Algorithm 3); 0: sigma stays sigma0        */
    int precision;           /* hprlp_precision (default HPRLP_FP64)                       */
    double tol_switch;       /* MIXED: switch to FP64 once rel. KKT <= this (default 1e-5) */
    int stall_checks;        /* MIXED: also switch when the best rel. KKT of the FP32 phase */
                             /* has not fallen below stall_ratio x its earlier best over   */
                             /* this many checks (default 0: off; the FP32 phase keeps      */
                             /* displacements from the FP64 anchor, so it reaches tol_switch) */
    int tile_nnz;            /* schedule: nonzeros staged per tile (0 = default)           */
    int tile_rows;           /* schedule: rows per tile (0 = default)                      */
    int short_max;           /* schedule: longest row kept in tiles (0 = default)          */
    int split_len;           /* schedule: rows longer than this are split (0 = default)    */
    int chunk_nnz;           /* schedule: nonzeros per split chunk (0 = default)           */
    int reorder;             /* 1 (default): number the columns by decreasing nonzero count */
                             /* inside the library (denser gather cache lines); results    */
                             /* are returned in the caller's order either way              */
    int profile;             /* N > 0: time the passes of every N-th iteration with HIP    */
                             /* events (stats col/row_pass_ms and _launches); a batched     */
                             /* solve places the events as nodes of its chunk graphs; 0: off */
    int verbose;             /* 1: one log line per check on stderr                        */
    int autotune;            /* 1: at create, time candidate schedules of A and A^T on the  */
                             /* uploaded problem and keep the fastest per matrix (problems  */
                             /* with >= 1e5 nonzeros); the schedule fields above are then   */
                             /* the starting point.  0 (default): use them as given         */
    double stall_ratio;      /* MIXED stall rule: switch when the best rel. KKT of the last */
                             /* stall_checks checks is above stall_ratio x the best before */
                             /* them (default 0.5; in (0, 1])                               */
    int graph;               /* single LP: run the plain iterations between two checks as   */
                             /* one captured hipGraph (identical iterates; needs            */
                             /* check_every >= 3 and profile = 0).  1 (default): when nnz   */
                             /* < 1e5 (launch-bound passes); 2: always; 0: never             */
    double rho;              /* relaxation of Algorithm 2: w_hat = rho w_bar + (1-rho) w,   */
                             /* in (0, 2]; 2 (default) = Peaceman-Rachford (HPR), 1 =        */
                             /* Douglas-Rachford (the paper's ablation, Section 4.2)         */
    int t1_zero;             /* 1: the T1 = 0 variant of Section 3.2 for LPs without        */
                             /* inequality rows (m2 = 0): the y-step solves with A A^T      */
                             /* exactly (eq. AATy=R) through a dense inverse of A~A~^T      */
                             /* formed at create (m <= 65536, 8 m^2 bytes of workspace,     */
                             /* A of full row rank, FP64,                                    */
                             /* single LPs; EINVAL / EDIM otherwise), sigma by eq.          */
                             /* sigma_T1=0; no power method.  0 (default): T1 = lambda I -  */
                             /* A A^T                                                        */
    int setup_on_host;       /* 0 (default): create renumbers, transposes and scales the    */
                             /* problem on the GPU, in scratch inside the workspace (which  */
                             /* hprlp_workspace_bytes then includes); 1: on the host, with  */
                             /* a smaller workspace.  Both give bit-identical arrays        */
    int tile_order;          /* order of the nonzeros inside each tile of A and A^T (the    */
                             /* schedules' runs of short rows): 0 (default) = row order;    */
                             /* 1 = column order (the gathers of a wavefront then walk the  */
                             /* gathered vector in increasing address order and share cache */
                             /* lines; each product is put back in its row-order slot before */
                             /* the sums, so results are bit-identical; 2 more bytes read   */
                             /* per nonzero); -1 = chosen per matrix by the autotuner (row  */
                             /* order when autotune = 0).  Not with t1_zero (EINVAL for 1;  */
                             /* -1 means row order there)                                    */
    int bundle_rows;         /* row bundles: runs of >= 2 consecutive rows of equal length  */
                             /* (<= 16384) stored k-major in groups of up to 64, one lane   */
                             /* per row, so where each row's columns are its predecessor's  */
                             /* plus one (demand rows of transportation and transport LPs,  */
                             /* QAP rows) the gathers coalesce.  -1 (default): such runs of */
                             /* A of length >= 16 (the row pass); 0: none; 1: every         */
                             /* equal-length run of A and A^T of length >= 256.  Sums keep  */
                             /* a fixed order.  With t1_zero: -1 (A only);  */
                             /* 1 is EINVAL.  Adds a bounded share to hprlp_workspace_bytes */
                             /* when not 0                                                   */
} hprlp_options;

typedef struct {
    long long iters;         /* iterations done (the k of Algorithm 2)                     */
    long long restarts;      /* outer loops started after the first (the r)               */
    long long iters_fp32;    /* MIXED: iterations done in the FP32 phase                   */
    int status;              /* hprlp_status of the last solve                             */
    int power_iters;
    double sigma, lambda;
    double rel_p, rel_d, rel_gap;  /* of the returned w_bar, original data (Section 4.1)  */
    double pobj, dobj;
    double beta_b, beta_c;   /* b/c normalisation factors                                  */
    double t_power_ms;       /* power method (counted in the solve time, Section 4.1)      */
    double t_solve_ms;       /* whole solve incl. power method; excludes create            */
    double bytes_per_iter;   /* algorithmic HBM bytes of one iteration in the final phase  */
    double col_pass_ms, row_pass_ms;   /* profile=1: summed time of the main SpMV kernel of  */
                                       /* the column (x-step) and row (y-step) passes       */
    long long col_pass_launches, row_pass_launches;
    double split_ms;         /* profile=1: summed time of the split-row finishing kernels  */
    long long n_checks;
    long long n_compactions; /* batched: times the schedules were rebuilt without the      */
                             /* instances that had stopped                                  */
    double t_setup_ms;       /* hprlp_create: validation, preconditioning, transpose,       */
                             /* schedules (and autotuning), upload                          */
    double t_prep_ms;        /* the part of t_setup_ms from the renumbering to the data     */
                             /* vectors (host or device preprocessing, uploads included)    */
    double t_tune_ms;        /* the part of t_setup_ms spent autotuning the schedules       */
} hprlp_stats_t;

/* Iterates that hprlp_get_iterate can return (original space unless noted). */
typedef enum {
    HPRLP_XBAR = 0,  /* x_bar of the last checked iteration (the returned primal)         */
    HPRLP_YBAR = 1,  /* y_bar of the last checked iteration (the returned dual, length m) */
    HPRLP_ZBAR = 2,  /* z_bar of the last checked iteration (eq. update-z)                */
    HPRLP_XCUR = 3,  /* current iterate x^{r,t} after the last Halpern step (single LP)   */
    HPRLP_YCUR = 4,  /* current iterate y^{r,t}                                           */
    HPRLP_DROW = 5,  /* row scaling D_r (length m; A~ = D_r A D_c)                        */
    HPRLP_DCOL = 6   /* column scaling D_c (length n)                                     */
} hprlp_iterate;

/* Fill *opt with the defaults listed above (the paper's settings, Section 4.1). */
void hprlp_default_options(hprlp_options *opt);

/* Upper bound of the device workspace needed for a problem with m1 + m2 rows, n columns and
 * nnz nonzeros under *opt (NULL: defaults).  Writes *bytes.  Host only; EDIM on bad sizes. */
int hprlp_workspace_bytes(int64_t m1, int64_t m2, int64_t n, int64_t nnz,
                          const hprlp_options *opt, size_t *bytes);

/* Validate and preprocess one LP (eq. primalLP) and upload it into d_workspace:
 *   - validation (see hprlp_err), done before any HIP call;
 *   - the column renumbering, CSR(A) and a stored CSR(A^T) (so neither sparse product
 *     needs atomics), and the preconditioning: 10 Ruiz passes, one Pock-Chambolle
 *     alpha=1 pass, b/c normalisation (Section 4.1, "Presolve and preconditioning"); on
 *     the GPU inside the workspace, or on the host with setup_on_host = 1;
 *   - the row-length tile schedules of both matrices (host), the autotuner's choice
 *     among them (autotune = 1), and with t1_zero the dense inverse of A~A~^T.
 * Errors after validation: EHIP (a HIP call failed), EINVAL (workspace too small, or
 * t1_zero with A of deficient row rank).
 * m1 >= 0 equality rows, m2 >= 0 inequality rows, m1 + m2 >= 1, n >= 1, nnz >= 1 (A != 0,
 * Section 1).  stream: a hipStream_t (NULL = default stream).  On success *out owns host
 * metadata only; the workspace stays owned by the caller. */
int hprlp_create(hprlp_handle **out, int64_t m1, int64_t m2, int64_t n,
                 const int64_t *rowptr, const int32_t *colidx, const double *val,
                 const double *b, const double *c, const double *l, const double *u,
                 const hprlp_options *opt, void *d_workspace, size_t ws_bytes, void *stream);

/* hprlp_create for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same create, with the
 * same arguments except the workspace, whose role is taken by a static scratch array of 64
 * MiB that the library holds on every GPU it runs on (reserved when the library is loaded
 * there, kept until the process ends).  The scratch of the CURRENT device is used.  This
 * call and the handle it returns make no device or pinned-host allocation: no hipMalloc,
 * hipHostMalloc, captured graph or timing event (so profile and autotune must be 0, else
 * EINVAL; graph is forced to 0).  Limits and sharing:
 *   - problems whose hprlp_workspace_bytes exceeds 64 MiB are refused with EINVAL before
 *     any GPU work (about 7e5 nonzeros for a general LP);
 *   - single LPs only (no batched variant);
 *   - one live handle per device: while a handle from this call exists on a device, a second
 *     call on that device returns ESTATE; hprlp_destroy frees the scratch for the next one.
 *     The scratch keeps the previous handle's data; create overwrites everything a solve
 *     reads, so no clearing is needed;
 *   - every call on one GPU shares that GPU's scratch: calls that overlap on it (a solve
 *     still running on one stream while another thread creates on the same device after a
 *     destroy, or one handle used from two threads) race; the guard above only orders
 *     create and destroy.
 * Everything else (validation, errors, stream ordering, outputs) is as for hprlp_create. */
int hprlp_create_noalloc(hprlp_handle **out, int64_t m1, int64_t m2, int64_t n,
                         const int64_t *rowptr, const int32_t *colidx, const double *val,
                         const double *b, const double *c, const double *l, const double *u,
                         const hprlp_options *opt, void *stream);
/* Workspace bound for a batch of n_inst LPs packed block-diagonally into m rows, n columns
 * and nnz nonzeros (see hprlp_create_batched).  Host only; EDIM on bad sizes
 * (n_inst must be in [1, min(m, n)]). */
int hprlp_workspace_bytes_batched(int32_t n_inst, int64_t m, int64_t n, int64_t nnz,
                                  const hprlp_options *opt, size_t *bytes);

/* Create a handle that solves n_inst independent LPs (each of the form eq. primalLP) in one
 * run.  The LPs are packed block-diagonally into one CSR: instance i owns rows
 * [inst_row_off[i], inst_row_off[i+1]) and columns [inst_col_off[i], inst_col_off[i+1]);
 * inside its rows, its first inst_m1[i] rows are equalities and the rest inequalities;
 * no row may have a nonzero outside its instance's columns (EDIM otherwise).  rowptr,
 * colidx, val, b, c, l, u are as for hprlp_create over the packed problem; inst_row_off and
 * inst_col_off are int64[n_inst + 1] host arrays starting at 0 and ending at m and n, strictly
 * increasing (every instance has a row, a column and a nonzero).  lambda_inst (host,
 * double[n_inst], nullable): lambda of every instance; NULL: lambda_override if > 0, else the
 * power method run on all instances at once.
 * Every instance is solved exactly as hprlp_create + hprlp_solve would solve it alone
 * (its own preconditioning is the restriction of the packed one, since Ruiz and
 * Pock-Chambolle scale rows and columns independently; its own beta_b, beta_c, sigma,
 * lambda, restart counters and termination test, Sections 3.1, 3.2 and 4.1), except that:
 * check_every must be >= 2; the columns are never renumbered (reorder is ignored); a MIXED
 * batch switches every instance to FP64 together, when all instances still iterating have
 * reached tol_switch or the largest rel. KKT among them stalls (stall_checks); and
 * max_iter / time_limit are tested every check_every iterations.  An instance that
 * terminates stops iterating; its returned w_bar is that of its last check.
 * Work runs on a stream owned by the handle (the caller's `stream` is synchronised at
 * create and at every solve); each check_every-iteration chunk is one captured hipGraph. */
int hprlp_create_batched(hprlp_handle **out, int32_t n_inst, const int64_t *inst_row_off,
                         const int64_t *inst_col_off, const int64_t *inst_m1,
                         const int64_t *rowptr, const int32_t *colidx, const double *val,
                         const double *b, const double *c, const double *l, const double *u,
                         const double *lambda_inst, const hprlp_options *opt,
                         void *d_workspace, size_t ws_bytes, void *stream);

/* Run Algorithm 2 from the origin (Section 4.1) until the relative KKT residual of w_bar
 * is <= tol at a check, or a limit is hit.  lambda = lambda_1(A~ A~^T) by the power
 * method unless overridden (T1 = lambda I - A~ A~^T, Section 3.2).  Writes the returned
 * w_bar = (x, y, z) in the original space (x: n, y: m, z: n; any may be NULL) and *status.
 * The call blocks until the result is ready.  Batched handle: every instance is solved;
 * *status is OPTIMAL only if every instance is, else the first other status met. */
int hprlp_solve(hprlp_handle *h, double *x, double *y, double *z, int *status);

/* Start a solve without iterating: lambda by the power method unless given (Section 4.1,
 * "Initialization and parameter setting"), sigma = sigma0 and the origin w = 0 with
 * t = k = r = 0 (every instance of a batched handle).  The iterations then advance with
 * hprlp_step; hprlp_stats reports power_iters, lambda and t_power_ms.  If the power method
 * gives lambda <= 0, the stats report HPRLP_NUMERICAL and hprlp_step returns ESTATE.  Blocks
 * until done. */
int hprlp_begin(hprlp_handle *h);

/* Advance the solve of Algorithm 2 from the current state (left by hprlp_begin or a solve).
 * Single-LP handle: `iters` more iterations (the column and row passes, Section 3.3),
 *   continuing the current outer loop (t and k advance) with no check, restart or sigma
 *   update: a debugging / parity aid that exposes the plain fixed-point map.  The returned
 *   w_bar (XBAR, YBAR, ZBAR) stays that of the last check; XCUR / YCUR give the new current
 *   iterate.
 * Batched handle: `iters` must be a multiple of check_every; runs iters / check_every whole
 *   chunks exactly as hprlp_solve runs them (each with its checks, the restart, sigma and
 *   termination decisions of every instance, Sections 3.1, 3.2 and 4.1), stopping early once
 *   every instance has stopped or max_iter / time_limit (counted from hprlp_begin) is hit,
 *   after which further steps run nothing; hprlp_stats / hprlp_stats_instance and the XBAR,
 *   YBAR, ZBAR iterates then describe the batch as it stands.
 * ESTATE before hprlp_begin or a solve; EINVAL on iters < 0 (or not a multiple of
 * check_every for a batch).  Blocks until done. */
int hprlp_step(hprlp_handle *h, int iters);

/* Statistics of the last solve.  Batched handle: iters = iterations run, restarts summed,
 * residuals the largest over the instances, objectives summed; per-instance figures come
 * from hprlp_stats_instance. */
int hprlp_stats(const hprlp_handle *h, hprlp_stats_t *out);

/* Statistics of instance i (0 <= i < n_inst; a single-LP handle has instance 0 only) of
 * the last solve: its own iters (iterations until it stopped), restarts, sigma, lambda,
 * residuals, objectives, beta_b, beta_c, n_checks and status.  Batched: t_solve_ms is the
 * time from the start of the solve to the end of the chunk whose check stopped the instance
 * (the time so far while it still iterates).  ESTATE before a solve. */
int hprlp_stats_instance(const hprlp_handle *h, int32_t i, hprlp_stats_t *out);

/* Copy one iterate (hprlp_iterate) of the last solve into out (host or device pointer,
 * length n or m). */
int hprlp_get_iterate(const hprlp_handle *h, int which, double *out);

/* Check trace of the last solve: one row of 18 doubles per check, columns
 * (k, t, r, sigma, merit, merit0, merit_prev, rel_p, rel_d, rel_gap, pobj, dobj,
 *  Delta_x, Delta_y, err_p, err_d, restarted, sigma_next).  Copies at most cap rows into
 * out (host) and writes the total row count to *n_rows. */
int hprlp_get_trace(const hprlp_handle *h, double *out, long long cap, long long *n_rows);

/* Check trace of instance i of a batched solve, kept on the device for its first 64
 * checks: rows of 10 doubles (k, t, r, sigma, merit, rel_p, rel_d, rel_gap, restarted,
 * sigma_next).  Copies at most cap rows into out (host) and writes min(checks, 64) to
 * *n_rows.  EINVAL on a single-LP handle. */
int hprlp_get_trace_instance(const hprlp_handle *h, int32_t i, double *out, long long cap,
                             long long *n_rows);

/* Schedule in use for A (matrix = 0, the row pass) or A^T (matrix = 1, the column pass):
 * params[5] = {tile_nnz, tile_rows, short_max, split_len, chunk_nnz} (nullable),
 * counts[6] = {work items incl. padding, tiles, whole-workgroup rows, split chunks,
 * 1 if the tiles hold their nonzeros in column order (tile_order) else 0, row-bundle work
 * items (bundle_rows)} (nullable), *tuned_ms = the autotuner's measured time of one pass launch with it (0 when
 * the autotuner did not run; nullable).  Host only. */
int hprlp_get_schedule(const hprlp_handle *h, int matrix, int32_t *params, int64_t *counts,
                       double *tuned_ms);

/* The schedule hprlp_create would build for A (matrix = 0) or A^T (matrix = 1) of a single
 * LP with m rows, n columns and the CSR (rowptr, colidx) of A (host arrays), under *opt
 * (NULL: defaults): counts[6] as in hprlp_get_schedule (counts[4] = 0: column order is
 * applied after create).  The options' schedule parameters are used as they are (no
 * autotuner, which needs the GPU).  A^T's rows are A's columns after the renumbering of
 * option reorder.  Host only: no GPU is needed.  EDIM on bad sizes, EINVAL on a bad index,
 * row pointer or option. */
int hprlp_plan_schedule(int64_t m, int64_t n, const int64_t *rowptr, const int32_t *colidx,
                        const hprlp_options *opt, int matrix, int64_t *counts);

/* Time the two iteration passes on the current state: `reps` launches of the column pass
 * (x-step over A~^T) and of the row pass (y-step over A~), each bracketed by HIP events on
 * the handle's stream.  Writes the mean duration of one launch in milliseconds.  The state
 * is advanced by these launches (call after a solve, not before one). */
int hprlp_time_passes(hprlp_handle *h, int reps, double *col_ms, double *row_ms);

/* Human-readable message of the last error on this handle (or of the last failed create
 * on this thread when h is NULL).  Never NULL. */
const char *hprlp_last_error(const hprlp_handle *h);

/* Release the handle's host resources (the workspace remains the caller's). */
void hprlp_destroy(hprlp_handle *h);

#ifdef __cplusplus
}
#endif
#endif /* HPRLP_H */
