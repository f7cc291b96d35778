/*
 * libpdlp linear-constraint propagation and integer-aware branching -- the propagate step and the
 * branching rule of fix-and-propagate (section 2 of the paper: the framework's linear-constraint
 * propagator, and "Integer-aware branching strategy", Alg. 1).
 *
 * Propagation (the paper names the propagator but does not define it; this is the standard
 * activity-based bound strengthening, in Jacobi rounds):
 *   rows a_i'x <= b_i ('L'), >= b_i ('G') or = b_i ('E'); every round, each row forms its minimum and
 *   maximum activity over the bounds of the round's start (finite part summed in row order, plus a
 *   count of infinite terms) and proposes for each of its variables the bound the other terms leave
 *   room for: a 'L' / 'E' row gives x_j <= (b_i - r_j) / a_ij when a_ij > 0 (>= when a_ij < 0), r_j
 *   being the residual minimum activity (its finite part without j's term; the finite part when j's
 *   term is the only infinite one; nothing when another term is infinite); 'G' / 'E' rows likewise
 *   with the maximum activity. Integer and binary variables round proposals inward within 1e-6
 *   (floor(p + 1e-6), ceil(p - 1e-6)) and take any strict gain; continuous variables take a gain
 *   larger than 1e-3 max(1, |bound|). A bound takes the tightest accepted proposal of any row.
 *   Stops at a fixpoint (no bound moved), at infeasibility (some l_j > u_j + 1e-6, or a row's finite
 *   activity beyond b_i by more than 1e-6 max(1, |b_i|)), or after max_rounds rounds.
 *
 * Conventions as in pdlp.h: 0 or a negative PDLP_ERR_* code, pdlp_last_error() has detail. The
 * handle deep-copies the constraint matrix (host arrays) and owns its device memory; bounds passed to
 * pdlp_propagate may be host or device memory (told apart with hipPointerGetAttributes; device
 * bounds are not checked). Work runs on pdlp_options.stream (NULL: a stream of the handle's own) and
 * each call returns after it finished. Results are bitwise reproducible: row sums keep row order,
 * and the tightest proposal of a set does not depend on the order rows deliver them.
 */
#ifndef PDLP_PROP_H
#define PDLP_PROP_H

#include <stdint.h>

#include "pdlp.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { PDLP_PROP_FIXPOINT = 0, PDLP_PROP_INFEASIBLE = 1, PDLP_PROP_ROUND_LIMIT = 2 };

typedef struct pdlp_prop pdlp_prop;

/* Propagation handle for the rows of a MIP: CSR as in pdlp_create (host arrays, validated the same
 * way), b [m], sense [m] ('L', 'G', 'E'), var_type [n] (PDLP_VAR_* of pdlp_fix.h: 0 continuous,
 * 1 binary, 2 integer). opt: NULL for defaults; stream and device_mem_limit are used. */
int pdlp_prop_create(pdlp_prop **out, int32_t m, int32_t n, int64_t nnz, const int32_t *row_ptr,
                     const int32_t *col_idx, const double *val, const double *b, const char *sense,
                     const uint8_t *var_type, const pdlp_options *opt);

/* Propagate bounds l [n], u [n] in place (+-HUGE_VAL allowed, no NaN) for at most max_rounds (>= 1)
 * rounds. *rounds receives the rounds run, *status a PDLP_PROP_* code (host memory; either may be
 * NULL). On
 * PDLP_PROP_INFEASIBLE the bounds are those after the round that showed it. */
int pdlp_propagate(pdlp_prop *p, double *l, double *u, int32_t max_rounds, int32_t *rounds, int32_t *status);

void pdlp_prop_destroy(pdlp_prop *p);

/* Integer-aware branching (Alg. 1): the bound changes for an integer variable with bounds [l, u],
 * fixing value a (integral, l <= a <= u) and objective coefficient c, in increasing priority (the
 * last is tried first). a strictly inside: (a+1, u) and (l, a-1) -- the one in the objective
 * direction (c > 0: downwards) later -- then (a, a); a on a bound: the other bound, then a.
 * lower [3], upper [3] receive the bounds, *count 2 or 3. PDLP_ERR_ARG for a outside [l, u], a
 * fractional a or NaN. Host-only. */
int pdlp_branching(double l, double u, double a, double c, double *lower, double *upper, int32_t *count);

#ifdef __cplusplus
}
#endif

#endif /* PDLP_PROP_H */
