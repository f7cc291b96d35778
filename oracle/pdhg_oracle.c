/*
 * FP64 CPU oracle for the PDLP solve of an LP relaxation (restarted, diagonally preconditioned
 * primal-dual hybrid gradient).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the independent reference that the GPU library is checked
 * against. Only the test suite, the smoke check and the benchmark's CPU-baseline leg load it. It
 * shares no code, header, table or constant generator with the GPU library, and the GPU library
 * never calls it.
 *
 * What it computes. The paper (Introduction, eq. (1)) states the LP as min c'x s.t. Ax <= b,
 * l <= x <= u with l, u in R u {+-inf}, and uses GPU PDLP (the PDHG variant specialised to LP of
 * its reference ApplegatePDLP) to solve the LP relaxation of a MIP to a low relative tolerance
 * (sections 1 and 2, "Fix-and-Propagate Using Low-Precision LP Solutions"; tolerances 1e-4 and
 * 1e-6 in section 4). The paper does not spell PDLP out, so the steps below follow the published
 * PDLP method and every constant is a reading:
 *   O0  rows a_i'x {<=, >=, =} b_i (eq. (1) widened to the senses the energy models carry),
 *       Lagrangian c'x - y'(Ax - b): y_i >= 0 on >= rows, y_i <= 0 on <= rows, free on = rows.
 *   O1  diagonal preconditioning: 10 Ruiz passes (row/column inf-norm equilibration) then one
 *       Pock-Chambolle pass with alpha = 1 (row/column 1-norm), A~ = Dr A Dc.
 *   O2  start point projected onto the bounds; primal weight w = |c~|/|b~|; eta = 1/max|a~|.
 *   O3  one PDHG attempt with the adaptive step size rule, weighted averages on acceptance.
 *   O4  every `eval_every` attempts: the weighted KKT error of current and average iterates, the
 *       restart test (beta = 0.2 / 0.8 / 0.36) and the primal weight update (theta = 0.5).
 *   O5  termination on the relative KKT error in the original space.
 *   O6  unscaling of the output.
 * The evaluation runs on the last committed iterate; attempt counter k counts accepted and rejected
 * steps alike.
 *
 * Build: gcc -O3 -fPIC -shared [-fopenmp] pdhg_oracle.c -o liboracle.so -lm
 * With OpenMP only the row loops of the matrix products run in parallel; every sum is taken
 * serially, so the results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------------------------- */
/* Interface types (mirrored by the ctypes wrapper in oracle/__init__.py)                       */
/* ------------------------------------------------------------------------------------------- */
typedef struct {
  int32_t m, n;
  const int32_t *row_ptr; /* [m+1] */
  const int32_t *col;     /* [nnz] */
  const double *val;      /* [nnz] */
  const double *c;        /* [n] */
  const double *b;        /* [m] */
  const uint8_t *sense;   /* [m] 'L' | 'G' | 'E' */
  const double *l, *u;    /* [n], +-inf allowed */
} orc_lp;

typedef struct {
  double tol;           /* relative KKT tolerance, <= 0 never terminates on it */
  int64_t iter_limit;   /* maximum number of attempts */
  int32_t ruiz_iters;   /* 10 */
  int32_t pock_chambolle; /* 1 = apply the alpha = 1 pass */
  int32_t eval_every;   /* 64 */
  int32_t trace_len;    /* number of attempts to record (<= 0: none) */
  const double *x0, *y0; /* optional start point in the original space */
  double omega0;        /* > 0: initial primal weight */
  double *trace_x;      /* [trace_len * n] committed x after attempt k, original space */
  double *trace_y;      /* [trace_len * m] */
  double *trace_eta;    /* [trace_len] step size after attempt k */
  double *trace_omega;  /* [trace_len] primal weight after attempt k */
  int32_t *trace_flags; /* [trace_len] bit0 accepted, bit1 evaluated, bit2 restarted, bit3 average */
  double *trace_margin; /* [trace_len] smallest relative margin of a discrete decision at attempt k */
  double *trace_cond;   /* [trace_len] 1 + |x|/|dx| + |y|/|dy| of attempt k (scaled space): the factor
                           by which relative errors of the iterates enter the step-size ratio */
  int32_t sum_order;    /* 0: every sum in index order; 1: every sum (matrix rows, reductions, norms,
                           scaling sums) in reverse index order; 2: even indices first, then odd.
                           Any order is a valid evaluation of the same formulas; comparing them
                           measures how far rounding alone moves the iterates. */
  int32_t pad_;
} orc_opts;

typedef struct {
  int32_t status;   /* 1 optimal to tolerance, 2 iteration limit, 3 numerical trouble */
  int32_t restarts;
  int64_t iterations;
  double rel_p, rel_d, rel_gap, pobj, dobj, omega, eta;
  int32_t which;    /* 0 current iterate returned, 1 average */
  int32_t pad;
  double omega_init, eta_init; /* primal weight and step size the first attempt started from (O2) */
} orc_result;

enum { ORC_OPTIMAL = 1, ORC_ITER_LIMIT = 2, ORC_NUMERICAL = 3 };

/* ------------------------------------------------------------------------------------------- */
/* Sparse helpers                                                                               */
/* ------------------------------------------------------------------------------------------- */

/* The index visited at step t of a sum over [0, len): in index order (mode 0), in reverse order
 * (mode 1), or the even indices in order and then the odd ones (mode 2). Every mode is a valid
 * evaluation of the same sum with its own rounding. */
static int32_t ord(int32_t t, int32_t len, int mode) {
  if (mode == 1) return len - 1 - t;
  if (mode == 2) {
    const int32_t half = (len + 1) / 2;
    return t < half ? 2 * t : 2 * (t - half) + 1;
  }
  return t;
}

/* y = A x for A in CSR; each row sum in the order `rev` selects */
static void spmv_ord(int32_t m, const int32_t *rp, const int32_t *ci, const double *v, const double *x,
                     double *y, int rev) {
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < m; ++i) {
    double s = 0.0;
    const int32_t len = rp[i + 1] - rp[i];
    for (int32_t t = 0; t < len; ++t) {
      const int32_t k = rp[i] + ord(t, len, rev);
      s += v[k] * x[ci[k]];
    }
    y[i] = s;
  }
}

/* y = A x for A in CSR */
void orc_spmv(int32_t m, const int32_t *rp, const int32_t *ci, const double *v, const double *x,
              double *y) {
  spmv_ord(m, rp, ci, v, x, y, 0);
}

/* CSR of A^T by counting sort: entries of each transposed row come in increasing row order of A. */
void orc_transpose(int32_t m, int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
                   int32_t *trp, int32_t *tci, double *tv) {
  int32_t nnz = rp[m];
  memset(trp, 0, sizeof(int32_t) * ((size_t)n + 1));
  for (int32_t k = 0; k < nnz; ++k) trp[ci[k] + 1]++;
  for (int32_t j = 0; j < n; ++j) trp[j + 1] += trp[j];
  int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  memcpy(fill, trp, sizeof(int32_t) * (size_t)n);
  for (int32_t i = 0; i < m; ++i)
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
      int32_t p = fill[ci[k]]++;
      tci[p] = i;
      tv[p] = v[k];
    }
  free(fill);
}

/* ------------------------------------------------------------------------------------------- */
/* O1: diagonal preconditioning                                                                 */
/* ------------------------------------------------------------------------------------------- */

/* One equilibration pass on sv (values of A in CSR with row index ri): divide a_ij by
 * sqrt(nr_i) * sqrt(nc_j) where nr/nc are the row/column norms (inf-norm if use_sum == 0,
 * 1-norm if use_sum == 1) of the current matrix, both taken before any entry changes.
 * Empty rows/columns use 1. Dr and Dc accumulate the divisions. */
static void equilibrate_pass(int32_t m, int32_t n, const int32_t *rp, const int32_t *ci, double *sv,
                             double *Dr, double *Dc, int use_sum, double *rho, double *kap, int rev) {
  int32_t nnz = rp[m];
  for (int32_t i = 0; i < m; ++i) rho[i] = 0.0;
  for (int32_t j = 0; j < n; ++j) kap[j] = 0.0;
  for (int32_t ti = 0; ti < m; ++ti)
    for (int32_t tk = 0; tk < rp[ord(ti, m, rev) + 1] - rp[ord(ti, m, rev)]; ++tk) {
      const int32_t i = ord(ti, m, rev);
      const int32_t k = rp[i] + ord(tk, rp[i + 1] - rp[i], rev);
      double a = fabs(sv[k]);
      int32_t j = ci[k];
      if (use_sum) {
        rho[i] += a;
        kap[j] += a;
      } else {
        if (a > rho[i]) rho[i] = a;
        if (a > kap[j]) kap[j] = a;
      }
    }
  for (int32_t i = 0; i < m; ++i) rho[i] = rho[i] > 0.0 ? sqrt(rho[i]) : 1.0;
  for (int32_t j = 0; j < n; ++j) kap[j] = kap[j] > 0.0 ? sqrt(kap[j]) : 1.0;
  for (int32_t i = 0; i < m; ++i)
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) sv[k] = sv[k] / (rho[i] * kap[ci[k]]);
  for (int32_t i = 0; i < m; ++i) Dr[i] = Dr[i] / rho[i];
  for (int32_t j = 0; j < n; ++j) Dc[j] = Dc[j] / kap[j];
  (void)nnz;
}

/* Ruiz passes then (optionally) one Pock-Chambolle pass with alpha = 1.
 * Outputs Dr[m], Dc[n] and the scaled values sv[nnz] (A~ = Dr A Dc in the CSR pattern of A). */
static int scale_ord(int32_t m, int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
                     int32_t ruiz_iters, int32_t pock_chambolle, double *Dr, double *Dc, double *sv, int rev) {
  int32_t nnz = rp[m];
  double *rho = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
  double *kap = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  if (!rho || !kap) {
    free(rho);
    free(kap);
    return -1;
  }
  memcpy(sv, v, sizeof(double) * (size_t)nnz);
  for (int32_t i = 0; i < m; ++i) Dr[i] = 1.0;
  for (int32_t j = 0; j < n; ++j) Dc[j] = 1.0;
  for (int32_t it = 0; it < ruiz_iters; ++it) equilibrate_pass(m, n, rp, ci, sv, Dr, Dc, 0, rho, kap, rev);
  if (pock_chambolle) equilibrate_pass(m, n, rp, ci, sv, Dr, Dc, 1, rho, kap, rev);
  free(rho);
  free(kap);
  return 0;
}

int orc_scale(int32_t m, int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
              int32_t ruiz_iters, int32_t pock_chambolle, double *Dr, double *Dc, double *sv) {
  return scale_ord(m, n, rp, ci, v, ruiz_iters, pock_chambolle, Dr, Dc, sv, 0);
}

/* ------------------------------------------------------------------------------------------- */
/* O0 projections                                                                               */
/* ------------------------------------------------------------------------------------------- */
static double clip(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }

/* projection onto the dual sign set Y_i of a row */
static double proj_y(double y, uint8_t s) {
  if (s == 'G') return y > 0.0 ? y : 0.0;
  if (s == 'L') return y < 0.0 ? y : 0.0;
  return y;
}

/* projection of g_j onto the reduced-cost set Lambda_j fixed by which bounds are finite */
static double proj_lambda(double g, double lo, double hi) {
  int lf = isfinite(lo), uf = isfinite(hi);
  if (lf && uf) return g;
  if (lf) return g > 0.0 ? g : 0.0;
  if (uf) return g < 0.0 ? g : 0.0;
  return 0.0;
}

/* ------------------------------------------------------------------------------------------- */
/* O3 building block: one PDHG step (exported for the fixed-point and sign tests)               */
/*   x' = proj_[l,u](x - tau (c - A'y))                                                          */
/*   y' = proj_Y(y + sigma (b - A(2x' - x)))                                                     */
/* aty = A'y and ax = Ax are passed in; axn receives A x'.                                      */
/* ------------------------------------------------------------------------------------------- */
static void pdhg_step(int32_t m, int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
                      const double *c, const double *b, const uint8_t *sense, const double *l,
                      const double *u, const double *x, const double *y, const double *ax,
                      const double *aty, double tau, double sigma, double *xn, double *yn,
                      double *axn, int rev) {
  for (int32_t j = 0; j < n; ++j) xn[j] = clip(x[j] - tau * (c[j] - aty[j]), l[j], u[j]);
  spmv_ord(m, rp, ci, v, xn, axn, rev);
  for (int32_t i = 0; i < m; ++i) yn[i] = proj_y(y[i] + sigma * (b[i] - 2.0 * axn[i] + ax[i]), sense[i]);
}

/* One step on an unscaled problem from (x, y) with the given tau and sigma. */
int orc_pdhg_step(const orc_lp *lp, const double *x, const double *y, double tau, double sigma,
                  double *xn, double *yn) {
  int32_t m = lp->m, n = lp->n, nnz = lp->row_ptr[m];
  int32_t *trp = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
  int32_t *tci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  double *tv = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
  double *ax = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
  double *aty = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  double *axn = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
  orc_transpose(m, n, lp->row_ptr, lp->col, lp->val, trp, tci, tv);
  orc_spmv(m, lp->row_ptr, lp->col, lp->val, x, ax);
  orc_spmv(n, trp, tci, tv, y, aty);
  pdhg_step(m, n, lp->row_ptr, lp->col, lp->val, lp->c, lp->b, lp->sense, lp->l, lp->u, x, y, ax,
            aty, tau, sigma, xn, yn, axn, 0);
  free(trp);
  free(tci);
  free(tv);
  free(ax);
  free(aty);
  free(axn);
  return 0;
}

/* ------------------------------------------------------------------------------------------- */
/* O4/O5 residuals                                                                              */
/* ------------------------------------------------------------------------------------------- */
typedef struct {
  double rp2, rd2;         /* squared 2-norms of primal / dual residual (space of the inputs) */
  double rp2_orig, rd2_orig; /* same after division by Dr / Dc (original space) */
  double pobj, dobj;
} residuals;

/* Residuals of (x, y) with ax = A x and aty = A'y given, for the problem (c, b, sense, l, u).
 * Dr/Dc may be NULL (then the original-space fields equal the plain ones). */
static residuals eval_residuals(int32_t m, int32_t n, const double *c, const double *b,
                                const uint8_t *sense, const double *l, const double *u,
                                const double *x, const double *y, const double *ax,
                                const double *aty, const double *Dr, const double *Dc, int rev) {
  residuals r = {0, 0, 0, 0, 0, 0};
  double by = 0.0, bound_terms = 0.0, cx = 0.0;
  for (int32_t ti = 0; ti < m; ++ti) {
    const int32_t i = ord(ti, m, rev);
    double t = b[i] - ax[i];
    if (sense[i] == 'G') t = t > 0.0 ? t : 0.0;
    else if (sense[i] == 'L') t = t < 0.0 ? t : 0.0;
    r.rp2 += t * t;
    double to = Dr ? t / Dr[i] : t;
    r.rp2_orig += to * to;
    by += b[i] * y[i];
  }
  for (int32_t tj = 0; tj < n; ++tj) {
    const int32_t j = ord(tj, n, rev);
    double g = c[j] - aty[j];
    double lam = proj_lambda(g, l[j], u[j]);
    double rd = g - lam;
    r.rd2 += rd * rd;
    double rdo = Dc ? rd / Dc[j] : rd;
    r.rd2_orig += rdo * rdo;
    if (isfinite(l[j]) && lam > 0.0) bound_terms += l[j] * lam;
    if (isfinite(u[j]) && lam < 0.0) bound_terms += u[j] * lam; /* -u * lambda^- with lambda^- = -lambda */
    cx += c[j] * x[j];
  }
  r.pobj = cx;
  r.dobj = by + bound_terms;
  return r;
}

/* O4: KKT error weighted by the primal weight, sqrt(w^2 |r_p|^2 + |r_d|^2 / w^2 + gap^2), from the
 * squared residual norms and the gap pobj - dobj (scaled space). */
double orc_kkt_weighted(double omega, double rp2, double rd2, double gap) {
  return sqrt(omega * omega * rp2 + rd2 / (omega * omega) + gap * gap);
}

static double kkt_weighted(const residuals *r, double omega) {
  return orc_kkt_weighted(omega, r->rp2, r->rd2, r->pobj - r->dobj);
}

static void relative_errors(const residuals *r, double nb, double nc, double *rel_p, double *rel_d,
                            double *rel_gap) {
  *rel_p = sqrt(r->rp2_orig) / (1.0 + nb);
  *rel_d = sqrt(r->rd2_orig) / (1.0 + nc);
  *rel_gap = fabs(r->pobj - r->dobj) / (1.0 + fabs(r->pobj) + fabs(r->dobj));
}

static double norm2_ord(const double *v, int32_t len, int rev) {
  double s = 0.0;
  for (int32_t t = 0; t < len; ++t) s += v[ord(t, len, rev)] * v[ord(t, len, rev)];
  return sqrt(s);
}
static double norm2(const double *v, int32_t len) { return norm2_ord(v, len, 0); }

/* Relative errors of (x, y) on the unscaled problem:
 * out = {rel_p, rel_d, rel_gap, pobj, dobj, |r_p|, |r_d|}. */
int orc_kkt(const orc_lp *lp, const double *x, const double *y, double *out) {
  int32_t m = lp->m, n = lp->n, nnz = lp->row_ptr[m];
  int32_t *trp = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
  int32_t *tci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  double *tv = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
  double *ax = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
  double *aty = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  orc_transpose(m, n, lp->row_ptr, lp->col, lp->val, trp, tci, tv);
  orc_spmv(m, lp->row_ptr, lp->col, lp->val, x, ax);
  orc_spmv(n, trp, tci, tv, y, aty);
  residuals r = eval_residuals(m, n, lp->c, lp->b, lp->sense, lp->l, lp->u, x, y, ax, aty, NULL, NULL, 0);
  relative_errors(&r, norm2(lp->b, m), norm2(lp->c, n), &out[0], &out[1], &out[2]);
  out[3] = r.pobj;
  out[4] = r.dobj;
  out[5] = sqrt(r.rp2);
  out[6] = sqrt(r.rd2);
  free(trp);
  free(tci);
  free(tv);
  free(ax);
  free(aty);
  return 0;
}

/* ------------------------------------------------------------------------------------------- */
/* The scalar rules of PDLP, one function each (the solve below calls exactly these)            */
/* ------------------------------------------------------------------------------------------- */

/* O2: the initial primal weight. omega0 > 0 is taken as given; otherwise |c~|_2 / |b~|_2 of the
 * scaled cost and right-hand side when both norms exceed 1e-10, else 1. */
double orc_initial_weight(double omega0, double norm_c_scaled, double norm_b_scaled) {
  if (omega0 > 0.0) return omega0;
  if (norm_c_scaled > 1e-10 && norm_b_scaled > 1e-10) return norm_c_scaled / norm_b_scaled;
  return 1.0;
}

/* O2: the initial step size 1 / max |a~_ij| over the scaled matrix (1 when it has no nonzero). */
double orc_initial_step(const double *sv, int64_t nnz) {
  double amax = 0.0;
  for (int64_t k = 0; k < nnz; ++k)
    if (fabs(sv[k]) > amax) amax = fabs(sv[k]);
  return amax > 0.0 ? 1.0 / amax : 1.0;
}

/* O3: the adaptive step-size rule after attempt k (k counts this attempt) that used step eta and
 * primal weight omega, from |dx|^2, |dy|^2 and the interaction dy'(A~ dx):
 *   eta_bar = (omega |dx|^2 + |dy|^2 / omega) / (2 |dy'(A~ dx)|), +inf when the interaction is 0;
 *   eta_new = min((1 - (k+1)^-0.3) eta_bar, (1 + (k+1)^-0.6) eta).
 * Returns 1 when the attempt is accepted (eta <= eta_bar, inclusive), else 0. */
int orc_step_rule(double omega, double dx2, double dy2, double inter, double eta, int64_t k,
                  double *eta_bar_out, double *eta_new_out) {
  double denom = 2.0 * fabs(inter);
  double eta_bar = denom > 0.0 ? (omega * dx2 + dy2 / omega) / denom : INFINITY;
  double kk = (double)(k + 1);
  *eta_new_out = fmin((1.0 - pow(kk, -0.3)) * eta_bar, (1.0 + pow(kk, -0.6)) * eta);
  *eta_bar_out = eta_bar;
  return eta <= eta_bar;
}

/* O4: the restart decision at an evaluation. The candidate is the average when its weighted KKT
 * error is strictly smaller than the current iterate's (ties go to the current iterate). With
 * KKT_c the candidate's error, KKT_a the anchor's (last restart point) and KKT_p the candidate's
 * error at the previous evaluation without restart (+inf right after a restart), restart iff
 *   KKT_c <= 0.2 KKT_a  (sufficient decay), or
 *   KKT_c <= 0.8 KKT_a and KKT_c > KKT_p  (necessary decay, no longer improving), or
 *   t >= 0.36 k  (artificial: t attempts since the last restart, k attempts in total).
 * Writes the candidate (0 current, 1 average) and its error; returns 1 to restart. */
int orc_restart_rule(double kkt_cur, double kkt_avg, double kkt_anchor, double kkt_prev,
                     int64_t t_since, int64_t k, int32_t *use_avg, double *kkt_cand) {
  int avg = kkt_avg < kkt_cur;
  double kkt_c = avg ? kkt_avg : kkt_cur;
  *use_avg = avg;
  *kkt_cand = kkt_c;
  return (kkt_c <= 0.2 * kkt_anchor) || (kkt_c <= 0.8 * kkt_anchor && kkt_c > kkt_prev) ||
         ((double)t_since >= 0.36 * (double)k);
}

/* O4: the primal weight after a restart, from the distances of the restart point to the anchor,
 * dx = |x_c - x_a|_2 and dy = |y_c - y_a|_2: exp(0.5 ln(dy / dx) + 0.5 ln omega), the geometric
 * mean of dy / dx and the old weight; unchanged unless both distances exceed 1e-10. */
double orc_primal_weight(double omega, double dx, double dy) {
  if (dx > 1e-10 && dy > 1e-10) return exp(0.5 * log(dy / dx) + 0.5 * log(omega));
  return omega;
}

/* ------------------------------------------------------------------------------------------- */
/* The solve: O1 .. O6                                                                          */
/* ------------------------------------------------------------------------------------------- */
typedef struct {
  double *x, *y, *ax, *aty;
} iterate;

static int alloc_iterate(iterate *z, int32_t m, int32_t n) {
  size_t mm = (size_t)(m > 0 ? m : 1), nn = (size_t)(n > 0 ? n : 1);
  z->x = (double *)malloc(sizeof(double) * nn);
  z->aty = (double *)malloc(sizeof(double) * nn);
  z->y = (double *)malloc(sizeof(double) * mm);
  z->ax = (double *)malloc(sizeof(double) * mm);
  return (z->x && z->y && z->ax && z->aty) ? 0 : -1;
}
static void free_iterate(iterate *z) {
  free(z->x);
  free(z->y);
  free(z->ax);
  free(z->aty);
}
static void copy_iterate(iterate *dst, const iterate *src, int32_t m, int32_t n) {
  memcpy(dst->x, src->x, sizeof(double) * (size_t)n);
  memcpy(dst->aty, src->aty, sizeof(double) * (size_t)n);
  memcpy(dst->y, src->y, sizeof(double) * (size_t)m);
  memcpy(dst->ax, src->ax, sizeof(double) * (size_t)m);
}

static double rel_margin(double a, double b) {
  double s = fabs(a) > fabs(b) ? fabs(a) : fabs(b);
  if (!(s > 0.0) || !isfinite(s)) return INFINITY;
  return fabs(a - b) / s;
}

int orc_solve(const orc_lp *lp, const orc_opts *o, double *x_out, double *y_out, double *rc_out,
              orc_result *res) {
  const int32_t m = lp->m, n = lp->n, nnz = lp->row_ptr[m];
  const int32_t every = o->eval_every > 0 ? o->eval_every : 64;
  const size_t mm = (size_t)(m > 0 ? m : 1), nn = (size_t)(n > 0 ? n : 1);
  const size_t zz = (size_t)(nnz > 0 ? nnz : 1);
  memset(res, 0, sizeof(*res));

  /* ---- O1: scaling --------------------------------------------------------------------- */
  double *Dr = (double *)malloc(sizeof(double) * mm), *Dc = (double *)malloc(sizeof(double) * nn);
  double *sv = (double *)malloc(sizeof(double) * zz);
  int32_t *trp = (int32_t *)malloc(sizeof(int32_t) * (nn + 1));
  int32_t *tci = (int32_t *)malloc(sizeof(int32_t) * zz);
  double *tv = (double *)malloc(sizeof(double) * zz);
  double *cs = (double *)malloc(sizeof(double) * nn), *ls = (double *)malloc(sizeof(double) * nn);
  double *us = (double *)malloc(sizeof(double) * nn), *bs = (double *)malloc(sizeof(double) * mm);
  double *xn = (double *)malloc(sizeof(double) * nn), *yn = (double *)malloc(sizeof(double) * mm);
  double *axn = (double *)malloc(sizeof(double) * mm), *atyn = (double *)malloc(sizeof(double) * nn);
  double *xa = (double *)malloc(sizeof(double) * nn), *ya = (double *)malloc(sizeof(double) * mm);
  iterate cur, avg;
  if (alloc_iterate(&cur, m, n) || alloc_iterate(&avg, m, n) || !Dr || !Dc || !sv || !trp || !tci ||
      !tv || !cs || !ls || !us || !bs || !xn || !yn || !axn || !atyn || !xa || !ya)
    return -1;

  const int rev = (o->sum_order == 1 || o->sum_order == 2) ? o->sum_order : 0;
  scale_ord(m, n, lp->row_ptr, lp->col, lp->val, o->ruiz_iters, o->pock_chambolle, Dr, Dc, sv, rev);
  orc_transpose(m, n, lp->row_ptr, lp->col, sv, trp, tci, tv);
  for (int32_t j = 0; j < n; ++j) {
    cs[j] = Dc[j] * lp->c[j];
    ls[j] = isfinite(lp->l[j]) ? lp->l[j] / Dc[j] : lp->l[j];
    us[j] = isfinite(lp->u[j]) ? lp->u[j] / Dc[j] : lp->u[j];
  }
  for (int32_t i = 0; i < m; ++i) bs[i] = Dr[i] * lp->b[i];
  const double nb = norm2_ord(lp->b, m, rev), nc = norm2_ord(lp->c, n, rev);

  /* ---- O2: initialisation ---------------------------------------------------------------- */
  for (int32_t j = 0; j < n; ++j) cur.x[j] = clip(o->x0 ? o->x0[j] / Dc[j] : 0.0, ls[j], us[j]);
  for (int32_t i = 0; i < m; ++i) cur.y[i] = proj_y(o->y0 ? o->y0[i] / Dr[i] : 0.0, lp->sense[i]);
  double omega = orc_initial_weight(o->omega0, norm2_ord(cs, n, rev), norm2_ord(bs, m, rev));
  double eta = orc_initial_step(sv, nnz);
  res->omega_init = omega;
  res->eta_init = eta;
  spmv_ord(m, lp->row_ptr, lp->col, sv, cur.x, cur.ax, rev);
  spmv_ord(n, trp, tci, tv, cur.y, cur.aty, rev);
  copy_iterate(&avg, &cur, m, n);
  memcpy(xa, cur.x, sizeof(double) * (size_t)n);
  memcpy(ya, cur.y, sizeof(double) * (size_t)m);
  double wsum = 0.0;
  residuals r0 = eval_residuals(m, n, cs, bs, lp->sense, ls, us, cur.x, cur.y, cur.ax, cur.aty, Dr, Dc, rev);
  double kkt_anchor = kkt_weighted(&r0, omega);
  double kkt_prev = INFINITY;
  int64_t k = 0, last_restart = 0;
  int32_t restarts = 0;
  int status = 0, which = 0;
  double out_rel[3] = {0, 0, 0}, out_obj[2] = {0, 0};

  /* ---- main loop ------------------------------------------------------------------------- */
  while (1) {
    /* O3: one attempt */
    double tau = eta / omega, sigma = eta * omega;
    pdhg_step(m, n, lp->row_ptr, lp->col, sv, cs, bs, lp->sense, ls, us, cur.x, cur.y, cur.ax,
              cur.aty, tau, sigma, xn, yn, axn, rev);
    spmv_ord(n, trp, tci, tv, yn, atyn, rev);
    k += 1;
    double dx2 = 0.0, dy2 = 0.0, inter = 0.0;
    for (int32_t tj = 0; tj < n; ++tj) {
      const int32_t j = ord(tj, n, rev);
      dx2 += (xn[j] - cur.x[j]) * (xn[j] - cur.x[j]);
    }
    for (int32_t ti = 0; ti < m; ++ti) {
      const int32_t i = ord(ti, m, rev);
      double dy = yn[i] - cur.y[i];
      dy2 += dy * dy;
      inter += dy * (axn[i] - cur.ax[i]);
    }
    double eta_bar, eta_new;
    int accepted = orc_step_rule(omega, dx2, dy2, inter, eta, k, &eta_bar, &eta_new);
    double margin = rel_margin(eta, eta_bar);
    double cond = 1.0;
    {
      double xx = 0.0, yy = 0.0;
      for (int32_t tj = 0; tj < n; ++tj) xx += cur.x[ord(tj, n, rev)] * cur.x[ord(tj, n, rev)];
      for (int32_t ti = 0; ti < m; ++ti) yy += cur.y[ord(ti, m, rev)] * cur.y[ord(ti, m, rev)];
      if (dx2 > 0.0) cond += sqrt(xx / dx2);
      if (dy2 > 0.0) cond += sqrt(yy / dy2);
    }
    if (accepted) {
      memcpy(cur.x, xn, sizeof(double) * (size_t)n);
      memcpy(cur.y, yn, sizeof(double) * (size_t)m);
      memcpy(cur.ax, axn, sizeof(double) * (size_t)m);
      memcpy(cur.aty, atyn, sizeof(double) * (size_t)n);
      wsum += eta;
      double w = eta / wsum;
      for (int32_t j = 0; j < n; ++j) {
        avg.x[j] += w * (cur.x[j] - avg.x[j]);
        avg.aty[j] += w * (cur.aty[j] - avg.aty[j]);
      }
      for (int32_t i = 0; i < m; ++i) {
        avg.y[i] += w * (cur.y[i] - avg.y[i]);
        avg.ax[i] += w * (cur.ax[i] - avg.ax[i]);
      }
    }
    eta = eta_new;
    if (!isfinite(eta) || !(eta > 0.0)) {
      status = ORC_NUMERICAL;
      break;
    }
    int flags = accepted ? 1 : 0;

    /* O4 + O5: evaluation */
    if (k % every == 0) {
      flags |= 2;
      residuals rc_ = eval_residuals(m, n, cs, bs, lp->sense, ls, us, cur.x, cur.y, cur.ax, cur.aty, Dr, Dc, rev);
      residuals ra_ = eval_residuals(m, n, cs, bs, lp->sense, ls, us, avg.x, avg.y, avg.ax, avg.aty, Dr, Dc, rev);
      double relc[3], rela[3];
      relative_errors(&rc_, nb, nc, &relc[0], &relc[1], &relc[2]);
      relative_errors(&ra_, nb, nc, &rela[0], &rela[1], &rela[2]);
      double kc = fmax(relc[0], fmax(relc[1], relc[2]));
      double ka = fmax(rela[0], fmax(rela[1], rela[2]));
      if (!isfinite(kc) && !isfinite(ka)) {
        status = ORC_NUMERICAL;
        break;
      }
      int pass_c = kc <= o->tol, pass_a = ka <= o->tol;
      if (pass_c || pass_a) {
        which = (pass_a && (!pass_c || ka < kc)) ? 1 : 0;
        const double *rel = which ? rela : relc;
        const residuals *rr = which ? &ra_ : &rc_;
        out_rel[0] = rel[0], out_rel[1] = rel[1], out_rel[2] = rel[2];
        out_obj[0] = rr->pobj, out_obj[1] = rr->dobj;
        status = ORC_OPTIMAL;
        if (which) copy_iterate(&cur, &avg, m, n);
        break;
      }
      double kkt_c_cur = kkt_weighted(&rc_, omega), kkt_c_avg = kkt_weighted(&ra_, omega);
      int32_t use_avg;
      double kkt_c;
      int64_t t_since = k - last_restart;
      int restart = orc_restart_rule(kkt_c_cur, kkt_c_avg, kkt_anchor, kkt_prev, t_since, k, &use_avg, &kkt_c);
      double mg = rel_margin(kkt_c_avg, kkt_c_cur);
      if (mg < margin) margin = mg;
      mg = rel_margin(kkt_c, 0.2 * kkt_anchor);
      if (mg < margin) margin = mg;
      mg = rel_margin(kkt_c, 0.8 * kkt_anchor);
      if (mg < margin) margin = mg;
      if (isfinite(kkt_prev)) {
        mg = rel_margin(kkt_c, kkt_prev);
        if (mg < margin) margin = mg;
      }
      if (!restart) {
        kkt_prev = kkt_c;
      } else {
        flags |= 4 | (use_avg ? 8 : 0);
        if (use_avg) copy_iterate(&cur, &avg, m, n);
        double ddx = 0.0, ddy = 0.0;
        for (int32_t tj = 0; tj < n; ++tj) {
          const int32_t j = ord(tj, n, rev);
          ddx += (cur.x[j] - xa[j]) * (cur.x[j] - xa[j]);
        }
        for (int32_t ti = 0; ti < m; ++ti) {
          const int32_t i = ord(ti, m, rev);
          ddy += (cur.y[i] - ya[i]) * (cur.y[i] - ya[i]);
        }
        ddx = sqrt(ddx);
        ddy = sqrt(ddy);
        omega = orc_primal_weight(omega, ddx, ddy);
        memcpy(xa, cur.x, sizeof(double) * (size_t)n);
        memcpy(ya, cur.y, sizeof(double) * (size_t)m);
        kkt_anchor = kkt_weighted(use_avg ? &ra_ : &rc_, omega);
        kkt_prev = INFINITY;
        copy_iterate(&avg, &cur, m, n);
        wsum = 0.0;
        last_restart = k;
        restarts += 1;
      }
    }

    if (o->trace_len > 0 && k <= o->trace_len) {
      int64_t t = k - 1;
      if (o->trace_x)
        for (int32_t j = 0; j < n; ++j) o->trace_x[t * n + j] = Dc[j] * cur.x[j];
      if (o->trace_y)
        for (int32_t i = 0; i < m; ++i) o->trace_y[t * m + i] = Dr[i] * cur.y[i];
      if (o->trace_eta) o->trace_eta[t] = eta;
      if (o->trace_omega) o->trace_omega[t] = omega;
      if (o->trace_flags) o->trace_flags[t] = flags;
      if (o->trace_margin) o->trace_margin[t] = margin;
      if (o->trace_cond) o->trace_cond[t] = cond;
    }

    if (k >= o->iter_limit) {
      status = ORC_ITER_LIMIT;
      break;
    }
  }

  if (status != ORC_OPTIMAL) {
    /* report the current iterate and its errors */
    residuals rc_ = eval_residuals(m, n, cs, bs, lp->sense, ls, us, cur.x, cur.y, cur.ax, cur.aty, Dr, Dc, rev);
    relative_errors(&rc_, nb, nc, &out_rel[0], &out_rel[1], &out_rel[2]);
    out_obj[0] = rc_.pobj, out_obj[1] = rc_.dobj;
    which = 0;
  }

  /* ---- O6: output in the original space --------------------------------------------------- */
  if (x_out)
    for (int32_t j = 0; j < n; ++j) x_out[j] = Dc[j] * cur.x[j];
  if (y_out || rc_out) {
    double *yo = (double *)malloc(sizeof(double) * mm);
    for (int32_t i = 0; i < m; ++i) yo[i] = Dr[i] * cur.y[i];
    if (y_out) memcpy(y_out, yo, sizeof(double) * (size_t)m);
    if (rc_out) {
      /* r = c - A'y with the unscaled matrix */
      int32_t *orp = (int32_t *)malloc(sizeof(int32_t) * (nn + 1));
      int32_t *oci = (int32_t *)malloc(sizeof(int32_t) * zz);
      double *ov = (double *)malloc(sizeof(double) * zz);
      orc_transpose(m, n, lp->row_ptr, lp->col, lp->val, orp, oci, ov);
      orc_spmv(n, orp, oci, ov, yo, rc_out);
      for (int32_t j = 0; j < n; ++j) rc_out[j] = lp->c[j] - rc_out[j];
      free(orp);
      free(oci);
      free(ov);
    }
    free(yo);
  }
  res->status = status;
  res->restarts = restarts;
  res->iterations = k;
  res->rel_p = out_rel[0];
  res->rel_d = out_rel[1];
  res->rel_gap = out_rel[2];
  res->pobj = out_obj[0];
  res->dobj = out_obj[1];
  res->omega = omega;
  res->eta = eta;
  res->which = which;

  free(Dr); free(Dc); free(sv); free(trp); free(tci); free(tv); free(cs); free(ls); free(us);
  free(bs); free(xn); free(yn); free(axn); free(atyn); free(xa); free(ya);
  free_iterate(&cur);
  free_iterate(&avg);
  return 0;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
