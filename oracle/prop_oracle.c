/*
 * Linear-constraint (activity) bound propagation, plain C in FP64 (TEST INFRASTRUCTURE ONLY: the
 * tests and the benchmark's CPU leg call it; the GPU library never does).
 *
 * The paper runs fix-and-propagate with the original framework's propagators, linear-constraint
 * propagation among them (section 2, first paragraph), and does not spell the propagator out; this
 * follows the standard activity-based bound strengthening, in Jacobi rounds as GPU domain
 * propagation runs it (every row reads the bounds of the round's start; a bound takes the tightest
 * proposal of any row). Readings:
 *   - row i: a_i'x <= b_i ('L'), >= b_i ('G'), both ('E'); bounds may be infinite.
 *   - minimum activity: sum over j of a_ij l_j (a_ij > 0) or a_ij u_j (a_ij < 0), kept as a finite
 *     part summed in row order (product, then sum) and a count of infinite terms; likewise the
 *     maximum activity with the bounds swapped.
 *   - for a 'L' / 'E' row, with the residual minimum activity r_j (the finite part minus j's term
 *     when no term is infinite; the finite part when j's term is the only infinite one; otherwise
 *     nothing is derived): a_ij > 0 proposes u_j = (b_i - r_j) / a_ij, a_ij < 0 proposes
 *     l_j = (b_i - r_j) / a_ij. 'G' / 'E' rows do the same with the residual maximum activity
 *     (a_ij > 0 proposes l_j, a_ij < 0 proposes u_j).
 *   - integer and binary variables round proposals inward: u = floor(p + 1e-6), l = ceil(p - 1e-6),
 *     and take any strict improvement; continuous variables take a proposal only when it improves
 *     the bound by more than 1e-3 max(1, |bound|) (an infinite bound: any finite proposal).
 *   - after a round: infeasible if some l_j > u_j + 1e-6, or a row's finite minimum activity exceeds
 *     b_i + 1e-6 max(1, |b_i|) ('L' / 'E') or its finite maximum activity falls short of
 *     b_i - 1e-6 max(1, |b_i|) ('G' / 'E'); a fixpoint when no bound changed; else the next round,
 *     up to max_rounds.
 * Status: 0 fixpoint, 1 infeasible, 2 round limit.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static const double kFeasTol = 1e-6;
static const double kContTol = 1e-3;

static double rmax(double a, double b) { return a > b ? a : b; }

/* Tighter of the current bound and a proposal, for one variable. */
static double tighten_upper(double cur, double p, int integral) {
  if (integral) {
    const double q = floor(p + kFeasTol);
    return q < cur ? q : cur;
  }
  if (isinf(cur)) return isinf(p) ? cur : p;
  return p < cur - kContTol * rmax(1.0, fabs(cur)) ? p : cur;
}
static double tighten_lower(double cur, double p, int integral) {
  if (integral) {
    const double q = ceil(p - kFeasTol);
    return q > cur ? q : cur;
  }
  if (isinf(cur)) return isinf(p) ? cur : p;
  return p > cur + kContTol * rmax(1.0, fabs(cur)) ? p : cur;
}

int orc_propagate(int32_t m, int32_t n, const int32_t *rp, const int32_t *ci, const double *val, const double *b,
                  const uint8_t *sense, const uint8_t *vtype, double *l, double *u, int32_t max_rounds,
                  int32_t *rounds_out) {
  double *ln = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  double *un = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  if (!ln || !un) {
    free(ln);
    free(un);
    return -1;
  }
  int status = 2, r = 0;
  for (r = 0; r < max_rounds; ++r) {
    memcpy(ln, l, sizeof(double) * (size_t)n);
    memcpy(un, u, sizeof(double) * (size_t)n);
    int row_infeasible = 0;
    for (int32_t i = 0; i < m; ++i) {
      /* activities from the round's start bounds, in row order */
      double minf = 0.0, maxf = 0.0;
      int mininf = 0, maxinf = 0;
      for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
        const double a = val[k], lo = l[ci[k]], hi = u[ci[k]];
        if (a == 0.0) continue; /* an explicit zero bounds nothing */
        const double tmin = a > 0.0 ? lo : hi, tmax = a > 0.0 ? hi : lo;
        if (isinf(tmin)) mininf++;
        else minf = minf + a * tmin;
        if (isinf(tmax)) maxinf++;
        else maxf = maxf + a * tmax;
      }
      const double tolb = kFeasTol * rmax(1.0, fabs(b[i]));
      const int le = sense[i] == 'L' || sense[i] == 'E', ge = sense[i] == 'G' || sense[i] == 'E';
      if ((le && mininf == 0 && minf > b[i] + tolb) || (ge && maxinf == 0 && maxf < b[i] - tolb)) row_infeasible = 1;
      for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
        const int32_t j = ci[k];
        const double a = val[k], lo = l[j], hi = u[j];
        if (a == 0.0) continue;
        const int integral = vtype[j] != 0;
        if (le) {
          const double t = a > 0.0 ? lo : hi;
          double res;
          int ok = 1;
          if (mininf == 0) res = minf - a * t;
          else if (mininf == 1 && isinf(t)) res = minf;
          else ok = 0;
          if (ok) {
            const double p = (b[i] - res) / a;
            if (a > 0.0) un[j] = fmin(un[j], tighten_upper(hi, p, integral));
            else ln[j] = fmax(ln[j], tighten_lower(lo, p, integral));
          }
        }
        if (ge) {
          const double t = a > 0.0 ? hi : lo;
          double res;
          int ok = 1;
          if (maxinf == 0) res = maxf - a * t;
          else if (maxinf == 1 && isinf(t)) res = maxf;
          else ok = 0;
          if (ok) {
            const double p = (b[i] - res) / a;
            if (a > 0.0) ln[j] = fmax(ln[j], tighten_lower(lo, p, integral));
            else un[j] = fmin(un[j], tighten_upper(hi, p, integral));
          }
        }
      }
    }
    int changed = 0, col_infeasible = 0;
    for (int32_t j = 0; j < n; ++j) {
      if (ln[j] != l[j] || un[j] != u[j]) changed = 1;
      l[j] = ln[j];
      u[j] = un[j];
      if (l[j] > u[j] + kFeasTol) col_infeasible = 1;
    }
    if (row_infeasible || col_infeasible) {
      status = 1;
      ++r;
      break;
    }
    if (!changed) {
      status = 0;
      ++r;
      break;
    }
  }
  free(ln);
  free(un);
  *rounds_out = r;
  return status;
}
