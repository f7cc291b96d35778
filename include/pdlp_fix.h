/*
 * libpdlp LP-based variable strategies and LP-based fixing -- the first consumers of the PDLP
 * solution in fix-and-propagate (section 2 of the paper: "LP-based variable strategies", "LP-based
 * fixing", "Tiebreaking and hybrid strategies").
 *
 * Given a point of the LP held by a single-problem handle (normally the x, y and reduced costs that
 * pdlp_get returned) and the type of each variable, these calls compute on the GPU
 *   - the order in which fix-and-propagate fixes the binary and integer variables, and
 *   - the value each of them is fixed to.
 * The paper names the keys; the directions and tie rules below are this library's readings:
 *   PDLP_ORDER_FRAC     ascending fractionality min(x - floor x, ceil x - x): nearly integral first
 *   PDLP_ORDER_REDCOST  descending |red_cost|
 *   PDLP_ORDER_DUAL     constraints in descending |y| (equal |y|: lower row first); each contributes
 *                       the binary / integer variables it holds that no earlier constraint held, in
 *                       RedCost order; variables in no constraint come last, in RedCost order
 *   PDLP_ORDER_TYPE     binaries first, then integers
 * A tiebreak strategy (PDLP_ORDER_NONE for none) orders what the strategy ranks equally (the paper's
 * hybrid strategies, e.g. Frac with ties broken by Dual); variables still equal keep index order.
 * LP-based fixing: with d_j = x_j - floor x_j and one sample s_j in (0, 1) per variable, the value is
 * floor x_j if s_j > d_j, else ceil x_j, clamped to [ceil l_j, floor u_j]; continuous variables keep
 * x_j. The samples are the caller's (any uniform source), so a run is reproducible.
 *
 * Conventions as in pdlp.h: return 0 or a negative PDLP_ERR_* code; vectors are in the caller's
 * numbering. Each pointer may be host memory or device memory on the handle's GPU (told apart with
 * hipPointerGetAttributes): device inputs are read in place and are not checked (they must be
 * finite), device outputs are written in place, so a caller with resident data moves nothing over
 * PCIe. Device workspace is kept in the handle between calls (grown on demand, counted against
 * device_mem_limit, freed by pdlp_destroy). Work runs on the handle's stream and each call returns
 * after it finished; results are bitwise reproducible (integer work and comparisons, no rounding).
 */
#ifndef PDLP_FIX_H
#define PDLP_FIX_H

#include <stdint.h>

#include "pdlp.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { PDLP_VAR_CONTINUOUS = 0, PDLP_VAR_BINARY = 1, PDLP_VAR_INTEGER = 2 };
enum { PDLP_ORDER_NONE = 0, PDLP_ORDER_FRAC = 1, PDLP_ORDER_REDCOST = 2, PDLP_ORDER_DUAL = 3, PDLP_ORDER_TYPE = 4 };

/* Order of the binary and integer variables under `strategy`, ties broken by `tiebreak`.
 *   var_type [n]  PDLP_VAR_* per variable
 *   x [n]         needed by FRAC; y [m] by DUAL; red_cost [n] by REDCOST and DUAL (others may be NULL)
 *   order [n]     receives the *count variable indices, first to fix first (count: host memory)
 * PDLP_ERR_ARG for a NULL handle or needed pointer, an unknown strategy, a batch handle, or (host
 * inputs) non-finite values. */
int pdlp_variable_strategy(pdlp_problem *p, int32_t strategy, int32_t tiebreak, const uint8_t *var_type,
                           const double *x, const double *y, const double *red_cost, int32_t *order,
                           int32_t *count);

/* Allocation-free variant of pdlp_variable_strategy, for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid hipMalloc). Same arguments,
 * same result bit for bit, with these differences:
 *   - var_type, x, y, red_cost and order must be device memory on the handle's GPU, which must be
 *     the current device (count stays host memory); otherwise PDLP_ERR_ARG;
 *   - the workspace is a static device buffer of 64 MiB that the library holds on each GPU it runs
 *     on until the process ends; a call needs about 20.25 max(n, m) bytes, plus 4 n + 12 m when DUAL
 *     is the strategy or the tiebreak (so max(n, m) up to 3.3 million, or n = m up to 1.85 million
 *     with DUAL); a larger problem is rejected with PDLP_ERR_ARG before any work is launched;
 *   - it never calls hipMalloc or hipFree. All calls on one GPU share the buffer, so calls that
 *     overlap in time on one GPU (several threads or streams) race and must be serialised by the
 *     caller. Each call writes every part of the buffer it reads, so nothing carries over. */
int pdlp_variable_strategy_noalloc(pdlp_problem *p, int32_t strategy, int32_t tiebreak, const uint8_t *var_type,
                                   const double *x, const double *y, const double *red_cost, int32_t *order,
                                   int32_t *count);

/* Fixing values of LP-based fixing for every variable.
 *   var_type [n], x [n], l [n], u [n] (original bounds, +-HUGE_VAL allowed), uniform [n] in (0, 1)
 *   value [n]     receives the fixing value (x_j for continuous variables)
 * PDLP_ERR_ARG for NULL pointers, a batch handle, or (host inputs) non-finite x, NaN bounds or
 * samples outside (0, 1). */
int pdlp_lp_fixing(pdlp_problem *p, const uint8_t *var_type, const double *x, const double *l, const double *u,
                   const double *uniform, double *value);

#ifdef __cplusplus
}
#endif

#endif /* PDLP_FIX_H */
