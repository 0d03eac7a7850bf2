/*
 * HPR-LP oracle: a plain, slow, FP64 CPU implementation of the HPR-LP iteration.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or load this
 * file; only the test-suite, the smoke check and the benchmark's CPU-baseline leg use it.
 * It shares no code, header or helper with the GPU library.
 *
 * What it follows (paper: "HPR-LP: An implementation of an HPR method for solving linear
 * programming", arXiv 2408.12179):
 *   - problem: primal LP (Section 1, eq. primalLP), dual (eq. dualLP), cone D = R^m1 x R^m2_+
 *   - preconditioning: 10 Ruiz passes, one diagonal Pock-Chambolle pass with alpha = 1,
 *     then b and c divided by (||b||+1) and (||c||+1)  (Section 4.1, "Presolve and
 *     preconditioning")
 *   - lambda = lambda_1(A A^T) of the scaled matrix by the power method, T1 = lambda I - A A^T
 *     (Section 4.1, "Initialization and parameter setting")
 *   - one iteration: eq. update-z, eq. update-x, eq. update-y-2 (Section 3.3), then the
 *     reflection and Halpern steps of Algorithm 2
 *   - merit R~ = ||w - w_hat||_M with M of eq. def:M (Section 3.1)
 *   - restart criteria eqs. restart_1..3 with alpha = (0.2, 0.6, 0.2)  (Sections 3.1, 4.1)
 *   - SigmaUpdate (Algorithm 3) with eq. sigma_T1!=0 and the safeguards eqs. Dx_Dy and
 *     primal_dual_infeasibility (Section 3.2)
 *   - termination: the three relative inequalities of Section 4.1, evaluated at w_bar on
 *     the original (unscaled) data, every check_every (=150) iterations
 *   - option t1_zero, the choice T1 = 0 of Section 3.2 (item 1) for LPs without inequality
 *     rows: the y-step is the exact minimiser, A A^T y_bar = (b - A(x_bar + sigma(z_bar -
 *     c))) / sigma (eq. AATy=R), solved with a dense Cholesky factor of A~ A~^T.  Written
 *     with the x-step it is y_bar = y + (A~A~^T)^{-1} (b~ - A~(2 x_bar - x)) / sigma.  M of
 *     eq. def:M then has the block sigma A A^T, so ||d||_M^2 = sigma ||A~^T dy||^2 +
 *     2 <dy, A~ dx> + ||dx||^2 / sigma, and SigmaUpdate uses eq. sigma_T1=0
 *     (Delta_y = ||A~^T (y_bar - y0)||).  No lambda is needed.
 *
 * Readings where the paper is silent (kept identical in the GPU library):
 *   - R~_{r,0} is evaluated on the first iteration of every outer loop; the merit used by
 *     the restart test is the one of the iteration that just finished, and criterion 2
 *     compares it with the merit of the previous check of the same outer loop (or R~_{r,0}).
 *   - the check runs after iteration k whenever k % check_every == 0 (k counts completed
 *     iterations), and also after the last allowed iteration; criterion 3 uses the
 *     post-increment t and k.
 *   - power method: v0 = (1/sqrt(m)) * ones, stop when the Rayleigh quotient changes by at
 *     most power_tol relative (or power_max_iter), lambda = the last Rayleigh quotient.
 *   - Ruiz/Pock-Chambolle factors of an empty row or column are 1.
 *   - sigma-update residuals error_p / error_d use the scaled data (sigma lives there);
 *     the termination test uses the original data.
 *   - delta*_C(-z) = sum_j ( max(-z_j,0) u_j - max(z_j,0) l_j ) with 0 * inf := 0.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared (no fast-math).  This plain
 * single-thread build is the pinned oracle.  The same source built with -fopenmp runs the
 * products and the per-element loops of an iteration on several threads, with every sum in
 * the same order (reductions stay serial), so its results are bit-identical; it exists only
 * to time the oracle on all host cores.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double tol;            /* termination tolerance epsilon                         */
    long long check_every; /* restart/termination check period (paper: 150)         */
    long long max_iter;
    double time_limit;     /* seconds (<= 0: none)                                  */
    double alpha1, alpha2, alpha3;
    double sigma0;
    int ruiz_iters;        /* 10 */
    int pock_chambolle;    /* 1: one diagonal Pock-Chambolle pass, alpha = 1         */
    int normalize_bc;      /* 1: divide b, c by (||b||+1), (||c||+1)                 */
    int power_max_iter;
    double power_tol;
    double lambda_override; /* > 0: use this lambda instead of the power method     */
    int use_halpern;       /* 1: Halpern averaging (Algorithm 2); 0: w <- w_hat     */
    double rho;            /* w_hat = rho*w_bar + (1-rho)*w; 2 = Peaceman-Rachford  */
    int use_restart;       /* 1: restart criteria of Section 3.1                    */
    int sigma_update;      /* 1: SigmaUpdate (Algorithm 3); 0: sigma fixed          */
    int trace_every_iter;  /* 1: record merit and KKT residual after every iteration */
    int t1_zero;           /* 1: T1 = 0 (Section 3.2, item 1); needs m2 = 0 and A of   */
                           /*    full row rank                                          */
} oracle_opts;

typedef struct {
    long long iters, restarts;
    int status; /* 1 optimal, 2 iteration limit, 3 time limit, 4 numerical */
    int power_iters;
    double sigma, lambda, rel_p, rel_d, rel_gap, pobj, dobj, beta_b, beta_c;
    double t_power, t_solve;
    long long n_checks, n_iter_trace;
} oracle_result;

enum { ST_OPTIMAL = 1, ST_ITER = 2, ST_TIME = 3, ST_NUMERICAL = 4 };

/* one row of the check trace */
enum {
    TR_K, TR_T, TR_R, TR_SIGMA, TR_MERIT, TR_MERIT0, TR_MERIT_PREV, TR_REL_P, TR_REL_D,
    TR_REL_GAP, TR_POBJ, TR_DOBJ, TR_DX, TR_DY, TR_ERR_P, TR_ERR_D, TR_RESTART,
    TR_SIGMA_NEW, TR_NCOL
};

static double now_s(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return ts.tv_sec + 1e-9 * ts.tv_nsec;
}

/* A CSR matrix M (m rows, n columns).  The OpenMP build (compiled with -fopenmp, used only
 * to time the oracle on all host cores) also stores M^T, with the entries of each column in
 * increasing row order, so that M^T y is a per-column gather whose sums run in the same
 * order as the row-by-row scatter of the plain build: both builds give identical bits. */
typedef struct {
    long long m, n;
    const int64_t *rp; const int32_t *ci; const double *v;
    int64_t *tp; int32_t *tr; double *tv;   /* transpose (OpenMP build), else NULL */
} csr_t;

static int csr_init(csr_t *M, long long m, long long n, const int64_t *rp, const int32_t *ci,
                    const double *v) {
    M->m = m; M->n = n; M->rp = rp; M->ci = ci; M->v = v;
    M->tp = NULL; M->tr = NULL; M->tv = NULL;
#ifdef _OPENMP
    long long nnz = rp[m];
    M->tp = calloc(n + 1, sizeof(int64_t));
    M->tr = malloc(sizeof(int32_t) * (nnz ? nnz : 1));
    M->tv = malloc(sizeof(double) * (nnz ? nnz : 1));
    int64_t *fill = malloc(sizeof(int64_t) * (n ? n : 1));
    if (!M->tp || !M->tr || !M->tv || !fill) { free(fill); return -6; }
    for (int64_t p = 0; p < nnz; ++p) M->tp[ci[p] + 1]++;
    for (long long j = 0; j < n; ++j) M->tp[j + 1] += M->tp[j];
    for (long long j = 0; j < n; ++j) fill[j] = M->tp[j];
    for (long long i = 0; i < m; ++i)
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
            int64_t q = fill[ci[p]]++;
            M->tr[q] = (int32_t)i;
            M->tv[q] = v[p];
        }
    free(fill);
#endif
    return 0;
}

static void csr_free(csr_t *M) { free(M->tp); free(M->tr); free(M->tv); }

/* out = M x */
static void csr_mv(const csr_t *M, const double *x, double *out) {
#pragma omp parallel for schedule(static)
    for (long long i = 0; i < M->m; ++i) {
        double s = 0.0;
        for (int64_t p = M->rp[i]; p < M->rp[i + 1]; ++p) s += M->v[p] * x[M->ci[p]];
        out[i] = s;
    }
}

/* out = M^T y: row by row, scattering (the plain build); per column over the stored
 * transpose, in the same order (the OpenMP build). */
static void csr_mtv(const csr_t *M, const double *y, double *out) {
    if (M->tp) {
#pragma omp parallel for schedule(static)
        for (long long j = 0; j < M->n; ++j) {
            double s = 0.0;
            for (int64_t q = M->tp[j]; q < M->tp[j + 1]; ++q) s += M->tv[q] * y[M->tr[q]];
            out[j] = s;
        }
        return;
    }
    for (long long j = 0; j < M->n; ++j) out[j] = 0.0;
    for (long long i = 0; i < M->m; ++i)
        for (int64_t p = M->rp[i]; p < M->rp[i + 1]; ++p) out[M->ci[p]] += M->v[p] * y[i];
}

/* Number of threads of the OpenMP build (1 in the plain build). */
int oracle_set_threads(int k) {
#ifdef _OPENMP
    if (k > 0) omp_set_num_threads(k);
    return omp_get_max_threads();
#else
    (void)k;
    return 1;
#endif
}

static double dot(long long k, const double *a, const double *b) {
    double s = 0.0;
    for (long long i = 0; i < k; ++i) s += a[i] * b[i];
    return s;
}

static double nrm2(long long k, const double *a) { return sqrt(dot(k, a, a)); }

static double clampd(double v, double lo, double hi) {
    if (v < lo) v = lo;
    if (v > hi) v = hi;
    return v;
}

/* product a*b with the convention 0 * (+-inf) := 0 */
static double mul0(double a, double b) { return (a == 0.0) ? 0.0 : a * b; }

/*
 * Preconditioning (Section 4.1): Ruiz equilibration, then one diagonal Pock-Chambolle
 * pass with alpha = 1, then normalisation of b and c.
 * Scaled problem: A~ = D_r A D_c, b~ = D_r b / beta_b, c~ = D_c c / beta_c,
 * l~ = l / (D_c beta_b), u~ = u / (D_c beta_b).
 */
int oracle_scale(long long m, long long n, const int64_t *rp, const int32_t *ci,
                 const double *val, const double *b, const double *c, const double *l,
                 const double *u, const oracle_opts *o, double *val_s, double *dr, double *dc,
                 double *b_s, double *c_s, double *l_s, double *u_s, double *beta_b,
                 double *beta_c) {
    long long nnz = rp[m];
    double *rs = malloc(sizeof(double) * (m > 0 ? m : 1));
    double *cs = malloc(sizeof(double) * (n > 0 ? n : 1));
    if (!rs || !cs) { free(rs); free(cs); return -6; }
    for (long long p = 0; p < nnz; ++p) val_s[p] = val[p];
    for (long long i = 0; i < m; ++i) dr[i] = 1.0;
    for (long long j = 0; j < n; ++j) dc[j] = 1.0;

    for (int it = 0; it < o->ruiz_iters + (o->pock_chambolle ? 1 : 0); ++it) {
        int ruiz = it < o->ruiz_iters;
        /* row and column norms: infinity-norm for Ruiz, 1-norm for Pock-Chambolle */
        for (long long i = 0; i < m; ++i) rs[i] = 0.0;
        for (long long j = 0; j < n; ++j) cs[j] = 0.0;
        for (long long i = 0; i < m; ++i)
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
                double a = fabs(val_s[p]);
                if (ruiz) {
                    if (a > rs[i]) rs[i] = a;
                    if (a > cs[ci[p]]) cs[ci[p]] = a;
                } else {
                    rs[i] += a;
                    cs[ci[p]] += a;
                }
            }
        for (long long i = 0; i < m; ++i) rs[i] = (rs[i] > 0.0) ? sqrt(rs[i]) : 1.0;
        for (long long j = 0; j < n; ++j) cs[j] = (cs[j] > 0.0) ? sqrt(cs[j]) : 1.0;
        for (long long i = 0; i < m; ++i)
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p) val_s[p] = val_s[p] / (rs[i] * cs[ci[p]]);
        for (long long i = 0; i < m; ++i) dr[i] = dr[i] / rs[i];
        for (long long j = 0; j < n; ++j) dc[j] = dc[j] / cs[j];
    }
    for (long long i = 0; i < m; ++i) b_s[i] = dr[i] * b[i];
    for (long long j = 0; j < n; ++j) {
        c_s[j] = dc[j] * c[j];
        l_s[j] = l[j] / dc[j];
        u_s[j] = u[j] / dc[j];
    }
    *beta_b = 1.0;
    *beta_c = 1.0;
    if (o->normalize_bc) {
        *beta_b = nrm2(m, b_s) + 1.0;
        *beta_c = nrm2(n, c_s) + 1.0;
        for (long long i = 0; i < m; ++i) b_s[i] /= *beta_b;
        for (long long j = 0; j < n; ++j) {
            c_s[j] /= *beta_c;
            l_s[j] /= *beta_b; /* +-inf stays +-inf */
            u_s[j] /= *beta_b;
        }
    }
    free(rs);
    free(cs);
    return 0;
}

/* Power method for lambda_1(A A^T) (Section 4.1).  Returns the number of iterations. */
int oracle_power(long long m, long long n, const int64_t *rp, const int32_t *ci,
                 const double *val, int max_iter, double tol, double *lambda) {
    double *v = malloc(sizeof(double) * m), *w = malloc(sizeof(double) * n);
    double *s = malloc(sizeof(double) * m);
    csr_t M;
    if (!v || !w || !s || csr_init(&M, m, n, rp, ci, val)) {
        free(v); free(w); free(s); return -6;
    }
    for (long long i = 0; i < m; ++i) v[i] = 1.0 / sqrt((double)m);
    double rq = 0.0, rq_prev = 0.0;
    int it = 0;
    for (it = 1; it <= max_iter; ++it) {
        csr_mtv(&M, v, w);                /* w = A^T v           */
        rq = dot(n, w, w);                /* v^T A A^T v, ||v||=1 */
        csr_mv(&M, w, s);                 /* s = A A^T v          */
        double ns = nrm2(m, s);
        if (ns == 0.0) break;
        for (long long i = 0; i < m; ++i) v[i] = s[i] / ns;
        if (it > 1 && fabs(rq - rq_prev) <= tol * rq) break;
        rq_prev = rq;
    }
    if (it > max_iter) it = max_iter;
    *lambda = rq;
    free(v); free(w); free(s);
    csr_free(&M);
    return it;
}

/* ||Pi_D(r)||^2 for a residual r = b - A x: the equality part counts fully, the
 * inequality part (rows >= m1) only where it is positive (A2 x >= b2 violated). */
static double proj_D_sq(long long m1, long long m, const double *r) {
    double s = 0.0;
    for (long long i = 0; i < m; ++i) {
        double ri = (i < m1) ? r[i] : (r[i] > 0.0 ? r[i] : 0.0);
        s += ri * ri;
    }
    return s;
}

typedef struct {
    long long m1, m, n;
    const int64_t *rp; const int32_t *ci;
    const double *val;     /* original A */
    csr_t Ao;              /* original A as a product operand */
    const double *b, *c, *l, *u;
    const double *val_s;   /* scaled A~ */
    const double *dr, *dc, *b_s, *c_s, *l_s, *u_s;
    double beta_b, beta_c;
} problem;

/* Relative KKT quantities of w_bar on the ORIGINAL data (Section 4.1, termination). */
static void original_residuals(const problem *P, const double *xb, const double *yb,
                               const double *zb, double *work_m, double *work_n,
                               double *xo, double *yo, double *zo, double *rel_p,
                               double *rel_d, double *rel_gap, double *pobj, double *dobj) {
    long long m = P->m, n = P->n;
    for (long long j = 0; j < n; ++j) {
        xo[j] = P->beta_b * P->dc[j] * xb[j];
        zo[j] = P->beta_c * zb[j] / P->dc[j];
    }
    for (long long i = 0; i < m; ++i) yo[i] = P->beta_c * P->dr[i] * yb[i];
    csr_mv(&P->Ao, xo, work_m); /* A x */
    for (long long i = 0; i < m; ++i) work_m[i] = P->b[i] - work_m[i];
    double np = sqrt(proj_D_sq(P->m1, m, work_m));
    csr_mtv(&P->Ao, yo, work_n); /* A^T y */
    for (long long j = 0; j < n; ++j) work_n[j] = P->c[j] - work_n[j] - zo[j];
    double nd = nrm2(n, work_n);
    double bnorm = nrm2(m, P->b), cnorm = nrm2(n, P->c);
    double po = dot(n, P->c, xo);
    double supp = 0.0; /* delta*_C(-z) */
    for (long long j = 0; j < n; ++j) {
        double zp = zo[j] > 0.0 ? zo[j] : 0.0, zm = zo[j] < 0.0 ? -zo[j] : 0.0;
        supp += mul0(zm, P->u[j]) - mul0(zp, P->l[j]);
    }
    double dobj_ = dot(m, P->b, yo) - supp;
    *rel_p = np / (1.0 + bnorm);
    *rel_d = nd / (1.0 + cnorm);
    *rel_gap = fabs(dobj_ - po) / (1.0 + fabs(dobj_) + fabs(po));
    *pobj = po;
    *dobj = dobj_;
}

/*
 * Full HPR-LP solve (Algorithm 2).  Inputs are the original problem data in CSR; outputs
 * x, y, z (original space) of the returned w_bar, and the current iterate w^{r,t}
 * (x_cur, y_cur, original space) after the last iteration.  Any output pointer may be NULL.
 * trace: check_cap rows of TR_NCOL doubles; iter_trace: iter_cap rows of 4 doubles
 * (merit ||w^k - w_hat^{k+1}||_M, ||R(w_bar^{k+1})|| on the scaled data, max bound
 * violation of x_bar, max cone violation of y_bar).
 */
/* Dense lower Cholesky factor L (row-major m x m) of A~ A~^T.  Returns 0, or -7 when the
 * matrix is not positive definite (A without full row rank). */
static int gram_cholesky(long long m, long long n, const int64_t *rp, const int32_t *ci,
                         const double *val, double *L) {
    double *row = calloc(n, sizeof(double));
    if (!row) return -6;
    for (long long i = 0; i < m; ++i) {
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) row[ci[p]] = val[p];
        for (long long k = 0; k <= i; ++k) {  /* (A A^T)_{ik} = <row i, row k> */
            double acc = 0.0;
            for (int64_t p = rp[k]; p < rp[k + 1]; ++p) acc += val[p] * row[ci[p]];
            L[i * m + k] = acc;
        }
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) row[ci[p]] = 0.0;
    }
    free(row);
    for (long long j = 0; j < m; ++j) {  /* column by column, in place on the lower part */
        double d = L[j * m + j];
        for (long long k = 0; k < j; ++k) d -= L[j * m + k] * L[j * m + k];
        if (!(d > 0.0)) return -7;
        const double ljj = sqrt(d);
        L[j * m + j] = ljj;
        for (long long i = j + 1; i < m; ++i) {
            double a = L[i * m + j];
            for (long long k = 0; k < j; ++k) a -= L[i * m + k] * L[j * m + k];
            L[i * m + j] = a / ljj;
        }
    }
    return 0;
}

/* x := (L L^T)^{-1} x (forward, then backward substitution). */
static void chol_solve(long long m, const double *L, double *x) {
    for (long long i = 0; i < m; ++i) {
        double a = x[i];
        for (long long k = 0; k < i; ++k) a -= L[i * m + k] * x[k];
        x[i] = a / L[i * m + i];
    }
    for (long long i = m - 1; i >= 0; --i) {
        double a = x[i];
        for (long long k = i + 1; k < m; ++k) a -= L[k * m + i] * x[k];
        x[i] = a / L[i * m + i];
    }
}

int oracle_solve(long long m1, long long m2, long long n, const int64_t *rp,
                 const int32_t *ci, const double *val, const double *b, const double *c,
                 const double *l, const double *u, const oracle_opts *o, double *x_out,
                 double *y_out, double *z_out, double *x_cur, double *y_cur,
                 oracle_result *res, double *trace, long long check_cap, double *iter_trace,
                 long long iter_cap, double *scaling_out /* dr[m], dc[n] or NULL */) {
    long long m = m1 + m2, nnz = rp[m];
    memset(res, 0, sizeof(*res));
    problem P = {0};
    P.m1 = m1; P.m = m; P.n = n; P.rp = rp; P.ci = ci; P.val = val;
    P.b = b; P.c = c; P.l = l; P.u = u;

    double *val_s = malloc(sizeof(double) * (nnz ? nnz : 1));
    double *dr = malloc(sizeof(double) * m), *dc = malloc(sizeof(double) * n);
    double *b_s = malloc(sizeof(double) * m), *c_s = malloc(sizeof(double) * n);
    double *l_s = malloc(sizeof(double) * n), *u_s = malloc(sizeof(double) * n);
    /* iterate state (scaled space) */
    double *x = calloc(n, sizeof(double)), *y = calloc(m, sizeof(double));
    double *x0 = calloc(n, sizeof(double)), *y0 = calloc(m, sizeof(double));
    double *xb = calloc(n, sizeof(double)), *yb = calloc(m, sizeof(double));
    double *zb = calloc(n, sizeof(double)), *v = calloc(n, sizeof(double));
    double *g = calloc(n, sizeof(double)), *s = calloc(m, sizeof(double));
    double *xr = calloc(n, sizeof(double)); /* 2 x_bar - x */
    double *dx = calloc(n, sizeof(double)), *dy = calloc(m, sizeof(double));
    double *wm = calloc(m, sizeof(double)), *wn = calloc(n, sizeof(double));
    double *xo = calloc(n, sizeof(double)), *yo = calloc(m, sizeof(double));
    double *zo = calloc(n, sizeof(double));
    if (!val_s || !dr || !dc || !b_s || !c_s || !l_s || !u_s || !x || !y || !x0 || !y0 ||
        !xb || !yb || !zb || !v || !g || !s || !xr || !dx || !dy || !wm || !wn || !xo ||
        !yo || !zo)
        return -6;

    oracle_scale(m, n, rp, ci, val, b, c, l, u, o, val_s, dr, dc, b_s, c_s, l_s, u_s,
                 &P.beta_b, &P.beta_c);
    csr_t As; /* the scaled matrix A~ */
    if (csr_init(&As, m, n, rp, ci, val_s) || csr_init(&P.Ao, m, n, rp, ci, val)) return -6;
    P.val_s = val_s; P.dr = dr; P.dc = dc; P.b_s = b_s; P.c_s = c_s; P.l_s = l_s;
    P.u_s = u_s;
    if (scaling_out) {
        for (long long i = 0; i < m; ++i) scaling_out[i] = dr[i];
        for (long long j = 0; j < n; ++j) scaling_out[m + j] = dc[j];
    }
    res->beta_b = P.beta_b;
    res->beta_c = P.beta_c;

    double t0 = now_s();
    double lambda;
    double *Lc = NULL, *gt = NULL; /* T1 = 0: Cholesky factor of A~A~^T, and A~^T dy */
    if (o->t1_zero) {
        if (m2 != 0) return -1;
        Lc = malloc(sizeof(double) * (size_t)(m * m));
        gt = malloc(sizeof(double) * (size_t)n);
        if (!Lc || !gt) return -6;
        int rcc = gram_cholesky(m, n, rp, ci, val_s, Lc);
        if (rcc) return rcc;
        lambda = 0.0;  /* not used */
        res->power_iters = 0;
    } else if (o->lambda_override > 0.0) {
        lambda = o->lambda_override;
        res->power_iters = 0;
    } else {
        res->power_iters = oracle_power(m, n, rp, ci, val_s, o->power_max_iter, o->power_tol,
                                        &lambda);
    }
    res->lambda = lambda;
    double t1 = now_s();
    res->t_power = t1 - t0;

    double bs_norm = nrm2(m, b_s), cs_norm = nrm2(n, c_s);
    double sigma = o->sigma0;
    long long r = 0, t = 0, k = 0;
    double merit0 = 0.0, merit_prev = 0.0;
    int status = 0;
    long long ntr = 0, nit = 0;

    /* initial point: the origin (Section 4.1); w^{0,0} = (0, 0, 0) */
    for (;;) {
        /* ---- one iteration of Algorithm 2 ---- */
        /* z-step and x-step (eqs. update-z, update-x): v = x + sigma (A^T y - c) */
        csr_mtv(&As, y, g);
#pragma omp parallel for schedule(static)
        for (long long j = 0; j < n; ++j) {
            v[j] = x[j] + sigma * (g[j] - c_s[j]);
            xb[j] = clampd(v[j], l_s[j], u_s[j]);
            zb[j] = (xb[j] - v[j]) / sigma;
            xr[j] = 2.0 * xb[j] - x[j];
        }
        /* y-step (eq. update-y-2) with T1 = lambda I - A A^T */
        csr_mv(&As, xr, s);
        if (o->t1_zero) {  /* T1 = 0: exact minimiser (eq. AATy=R), no inequality rows */
            for (long long i = 0; i < m; ++i) wm[i] = b_s[i] - s[i];
            chol_solve(m, Lc, wm);
            for (long long i = 0; i < m; ++i) yb[i] = y[i] + wm[i] / sigma;
        } else {
#pragma omp parallel for schedule(static)
            for (long long i = 0; i < m; ++i) {
                double yi = y[i] + (b_s[i] - s[i]) / (lambda * sigma);
                if (i >= m1 && yi < 0.0) yi = 0.0;
                yb[i] = yi;
            }
        }
        /* reflection w_hat = rho w_bar + (1 - rho) w, and d = w - w_hat for the merit */
#pragma omp parallel for schedule(static)
        for (long long j = 0; j < n; ++j) {
            double xh = o->rho * xb[j] + (1.0 - o->rho) * x[j];
            dx[j] = x[j] - xh;
            wn[j] = xh;
        }
#pragma omp parallel for schedule(static)
        for (long long i = 0; i < m; ++i) {
            double yh = o->rho * yb[i] + (1.0 - o->rho) * y[i];
            dy[i] = y[i] - yh;
            wm[i] = yh;
        }
        int first = (t == 0);
        int want_check = 0;
        k += 1;
        t += 1;
        if (k % o->check_every == 0 || k >= o->max_iter) want_check = 1;
        double el = now_s() - t0;
        if (o->time_limit > 0.0 && el >= o->time_limit) want_check = 1;

        double merit = -1.0;
        if (first || want_check || o->trace_every_iter) {
            /* R~ = ||w - w_hat||_M, M of eq. def:M with T1 = lambda I - A A^T:
             * ||d||_M^2 = sigma lambda ||dy||^2 + 2 <dy, A dx> + ||dx||^2 / sigma */
            csr_mv(&As, dx, s);
            double ty;  /* <dy, (T1 + A A^T) dy> */
            if (o->t1_zero) {
                csr_mtv(&As, dy, gt);
                ty = dot(n, gt, gt);
            } else {
                ty = lambda * dot(m, dy, dy);
            }
            double q = sigma * ty + 2.0 * dot(m, dy, s) + dot(n, dx, dx) / sigma;
            merit = sqrt(q > 0.0 ? q : 0.0);
        }
        if (o->trace_every_iter && iter_trace && nit < iter_cap) {
            /* KKT residual map R(w_bar) on the scaled problem (Section 2, eq. def:KKT_residual) */
            double acc = 0.0, viol_x = 0.0, viol_y = 0.0;
            csr_mv(&As, xb, s);
            for (long long i = 0; i < m; ++i) {
                double arg = yb[i] - s[i] + b_s[i];
                double pr = (i >= m1 && arg < 0.0) ? 0.0 : arg;
                double e = yb[i] - pr;
                acc += e * e;
                if (i >= m1 && -yb[i] > viol_y) viol_y = -yb[i];
            }
            for (long long j = 0; j < n; ++j) {
                double e = xb[j] - clampd(xb[j] - zb[j], l_s[j], u_s[j]);
                acc += e * e;
                double vl = l_s[j] - xb[j], vu = xb[j] - u_s[j];
                if (vl > viol_x) viol_x = vl;
                if (vu > viol_x) viol_x = vu;
            }
            csr_mtv(&As, yb, g);
            for (long long j = 0; j < n; ++j) {
                double e = c_s[j] - g[j] - zb[j];
                acc += e * e;
            }
            double *row = iter_trace + 4 * nit;
            row[0] = merit;
            row[1] = sqrt(acc);
            row[2] = viol_x;
            row[3] = viol_y;
            nit++;
        }

        /* Halpern step (Algorithm 2): w = w0/(t+2) + (t+1)/(t+2) w_hat, with t the inner
         * counter before the increment above */
        double tb = (double)(t - 1);
#pragma omp parallel for schedule(static)
        for (long long j = 0; j < n; ++j)
            x[j] = o->use_halpern ? x0[j] / (tb + 2.0) + ((tb + 1.0) / (tb + 2.0)) * wn[j] : wn[j];
#pragma omp parallel for schedule(static)
        for (long long i = 0; i < m; ++i)
            y[i] = o->use_halpern ? y0[i] / (tb + 2.0) + ((tb + 1.0) / (tb + 2.0)) * wm[i] : wm[i];

        if (first) {
            merit0 = merit;
            merit_prev = merit;
        }
        if (!want_check) continue;

        /* ---- check: termination on the original data ---- */
        double rel_p, rel_d, rel_gap, pobj, dobj;
        original_residuals(&P, xb, yb, zb, wm, wn, xo, yo, zo, &rel_p, &rel_d, &rel_gap,
                           &pobj, &dobj);
        res->rel_p = rel_p; res->rel_d = rel_d; res->rel_gap = rel_gap;
        res->pobj = pobj; res->dobj = dobj;
        double kkt = rel_p > rel_d ? rel_p : rel_d;
        if (rel_gap > kkt) kkt = rel_gap;
        double *tr = (trace && ntr < check_cap) ? trace + TR_NCOL * ntr : NULL;
        if (tr) {
            for (int q = 0; q < TR_NCOL; ++q) tr[q] = 0.0;
            tr[TR_K] = (double)k; tr[TR_T] = (double)t; tr[TR_R] = (double)r;
            tr[TR_SIGMA] = sigma; tr[TR_MERIT] = merit; tr[TR_MERIT0] = merit0;
            tr[TR_MERIT_PREV] = merit_prev; tr[TR_REL_P] = rel_p; tr[TR_REL_D] = rel_d;
            tr[TR_REL_GAP] = rel_gap; tr[TR_POBJ] = pobj; tr[TR_DOBJ] = dobj;
            tr[TR_SIGMA_NEW] = sigma;
            ntr++;
        }
        if (!(kkt == kkt)) { status = ST_NUMERICAL; break; }
        if (kkt <= o->tol) { status = ST_OPTIMAL; break; }
        if (k >= o->max_iter) { status = ST_ITER; break; }
        if (o->time_limit > 0.0 && now_s() - t0 >= o->time_limit) { status = ST_TIME; break; }

        /* ---- restart criteria (Section 3.1) ---- */
        int restart = 0;
        if (o->use_restart) {
            if (merit <= o->alpha1 * merit0) restart = 1;
            if (merit <= o->alpha2 * merit0 && merit > merit_prev) restart = 1;
            if ((double)t >= o->alpha3 * (double)k) restart = 1;
        }
        if (!restart) {
            merit_prev = merit;
            continue;
        }
        /* ---- SigmaUpdate (Algorithm 3), T1 = lambda I - A A^T (eq. sigma_T1!=0) ---- */
        double Dx = 0.0, Dy = 0.0, err_p = 0.0, err_d = 0.0, sigma_new = sigma;
        if (o->sigma_update) {
            for (long long j = 0; j < n; ++j) wn[j] = xb[j] - x0[j];
            for (long long i = 0; i < m; ++i) wm[i] = yb[i] - y0[i];
            Dx = nrm2(n, wn);
            if (o->t1_zero) {  /* eq. sigma_T1=0 */
                csr_mtv(&As, wm, gt);
                Dy = nrm2(n, gt);
            } else {
                Dy = sqrt(lambda) * nrm2(m, wm);
            }
            csr_mv(&As, xb, s);
            for (long long i = 0; i < m; ++i) wm[i] = b_s[i] - s[i];
            err_p = sqrt(proj_D_sq(m1, m, wm)) / (1.0 + bs_norm);
            csr_mtv(&As, yb, g);
            for (long long j = 0; j < n; ++j) wn[j] = c_s[j] - g[j] - zb[j];
            err_d = nrm2(n, wn) / (1.0 + cs_norm);
            int ok = Dx > 1e-16 && Dx < 1e12 && Dy > 1e-16 && Dy < 1e12 && err_p > 0.0 &&
                     err_d / err_p > 1e-8 && err_d / err_p < 1e8;
            sigma_new = ok ? Dx / Dy : 1.0;
        }
        if (tr) {
            tr[TR_DX] = Dx; tr[TR_DY] = Dy; tr[TR_ERR_P] = err_p; tr[TR_ERR_D] = err_d;
            tr[TR_RESTART] = 1.0; tr[TR_SIGMA_NEW] = sigma_new;
        }
        sigma = sigma_new;
        /* w^{r+1,0} = w_bar^{r,tau_r} */
        for (long long j = 0; j < n; ++j) { x0[j] = xb[j]; x[j] = xb[j]; }
        for (long long i = 0; i < m; ++i) { y0[i] = yb[i]; y[i] = yb[i]; }
        t = 0;
        r += 1;
    }
    res->t_solve = now_s() - t0;
    res->iters = k;
    res->restarts = r;
    res->status = status;
    res->sigma = sigma;
    res->n_checks = ntr;
    res->n_iter_trace = nit;
    /* outputs: w_bar of the last iteration (original space) and the current iterate */
    for (long long j = 0; j < n; ++j) {
        if (x_out) x_out[j] = P.beta_b * dc[j] * xb[j];
        if (z_out) z_out[j] = P.beta_c * zb[j] / dc[j];
        if (x_cur) x_cur[j] = P.beta_b * dc[j] * x[j];
    }
    for (long long i = 0; i < m; ++i) {
        if (y_out) y_out[i] = P.beta_c * dr[i] * yb[i];
        if (y_cur) y_cur[i] = P.beta_c * dr[i] * y[i];
    }
    free(val_s); free(dr); free(dc); free(b_s); free(c_s); free(l_s); free(u_s);
    free(x); free(y); free(x0); free(y0); free(xb); free(yb); free(zb); free(v); free(g);
    free(s); free(xr); free(dx); free(dy); free(wm); free(wn); free(xo); free(yo); free(zo);
    free(Lc); free(gt);
    csr_free(&As); csr_free(&P.Ao);
    return 0;
}
