/*
 * libpdlp learned warm start -- a bipartite variable/constraint message-passing network that
 * predicts a starting point (x0, y0) and primal weight omega0 for pdlp_solve / pdlp_batch_solve.
 *
 * The paper solves the initial LP relaxation with PDLP from a cold start (section 2, "LP-based
 * variable strategies"; section 4 reports PDLP to 1e-4 and 1e-6 relative tolerance). This header is
 * an extension on top of that solve, not part of the paper's method: the prediction only chooses
 * where PDLP starts, and pdlp_solve's own check (pdlp_options.warm_fallback) discards a predicted
 * start whose relative KKT error is not below the cold start's.
 *
 * Model (hidden width 64, three rounds; inputs are the handle's scaled problem, see pdlp_get_scaling):
 *   node features  variable j:   slog c_j, [l_j finite], [u_j finite], slog l_j, slog u_j,
 *                                log(1 + column degree)/4, 1, 0
 *                  constraint i: slog b_i, [<=], [>=], [=], log(1 + row degree)/4, 1, 0, 0
 *                  (slog v = sign(v) log(1 + |v|); scaled c, b, l, u; infinite bounds give 0)
 *   embedding      hv = relu(fv Wv_in + bv_in),  hc = relu(fc Wc_in + bc_in)
 *   round t        hc = relu(hc W1 + (A hv) W2 + b1);  hv = relu(hv W3 + (A' hc) W4 + b3)
 *   heads          x~ = hv wx + bx,  y~ = hc wy + by,
 *                  log omega = mean(hv) wov + mean(hc) woc + bo        (means over one instance)
 *   outputs        x0 = Dc x~, y0 = Dr y~ (original space), omega0 = exp(clamp(log omega, -20, 20))
 *   loss           mean over instances of mean_j (x~_j - x*_j/Dc_j)^2 + mean_i (y~_i - y*_i/Dr_i)^2
 *                  + w_omega (log omega - log omega*)^2     (w_omega = 1 unless set)
 * Dense products run on the BF16 matrix cores with FP32 accumulation (both operands rounded to
 * BF16, nearest even); everything else is FP32. Training uses Adam (beta 0.9 / 0.999, eps 1e-8,
 * bias-corrected) on FP32 master weights.
 *
 * Parameters: one FP32 vector of pdlp_gnn_num_params() = 50947 values in this order (matrices
 * row-major [input channel][output channel]): Wv_in[8x64], bv_in[64], Wc_in[8x64], bc_in[64], then
 * for each of the 3 rounds W1, W2 [64x64], b1[64], W3, W4 [64x64], b3[64], then wx[64], bx,
 * wy[64], by, wov[64], woc[64], bo.
 *
 * Conventions: return 0 or a negative PDLP_ERR_* code (pdlp_last_error() has detail); all buffers
 * are host buffers owned by the caller; vectors of a batch are the instances' vectors concatenated
 * in instance order (the numbering pdlp_batch_create received). Work runs on the problem's stream
 * and every call returns after it finished. A model may be used with any number of problems, one
 * call at a time. Results are bitwise reproducible on one GPU.
 */
#ifndef PDLP_GNN_H
#define PDLP_GNN_H

#include <stdint.h>

#include "pdlp.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pdlp_gnn pdlp_gnn;

/* Number of FP32 parameters (50947). */
int64_t pdlp_gnn_num_params(void);

/* New model: Glorot-uniform weights drawn from a 64-bit Mersenne twister seeded with `seed`,
 * zero biases, zero Adam state. */
int pdlp_gnn_create(pdlp_gnn **out, uint64_t seed);

/* Copy the FP32 master parameters out (params: num_params floats). */
int pdlp_gnn_get_params(pdlp_gnn *g, float *params);

/* Replace the parameters (all finite, else PDLP_ERR_ARG) and reset the Adam state. */
int pdlp_gnn_set_params(pdlp_gnn *g, const float *params);

/* Weight w_omega >= 0 of the log-omega term of the loss (default 1); PDLP_ERR_ARG otherwise. */
int pdlp_gnn_set_omega_weight(pdlp_gnn *g, float w);

/* Predict a warm start for a single problem: x0 [n], y0 [m] in the original space and the
 * caller's numbering, omega0 [1]. Any output pointer may be NULL. Pass the results to pdlp_solve. */
int pdlp_gnn_predict(pdlp_gnn *g, pdlp_problem *p, double *x0, double *y0, double *omega0);

/* Same for every instance of a batch: x0 [sum n], y0 [sum m], omega0 [k]. */
int pdlp_gnn_predict_batch(pdlp_gnn *g, pdlp_batch *b, double *x0, double *y0, double *omega0);

/* Raw head outputs in the handle's internal numbering and scaled space (see
 * pdlp_batch_get_internal): xhat [sum n], yhat [sum m], logw [k]. For testing. */
int pdlp_gnn_predict_raw(pdlp_gnn *g, pdlp_batch *b, float *xhat, float *yhat, float *logw);

/* Loss and gradient without an update, for targets x* [sum n], y* [sum m] (original space,
 * caller's numbering) and omega* [k] (> 0). grad: num_params floats or NULL. */
int pdlp_gnn_gradients(pdlp_gnn *g, pdlp_batch *b, const double *x_star, const double *y_star,
                       const double *omega_star, double *loss, float *grad);

/* One Adam step (learning rate lr > 0) on the loss of the batch against the targets; *loss is the
 * loss before the step. */
int pdlp_gnn_train_step(pdlp_gnn *g, pdlp_batch *b, const double *x_star, const double *y_star,
                        const double *omega_star, float lr, double *loss);

void pdlp_gnn_destroy(pdlp_gnn *g);

/* Scaling and internal (renumbered, scaled) matrix of a batch; same meaning as pdlp_get_scaling and
 * pdlp_get_internal, over the concatenation of the instances. */
int pdlp_batch_get_scaling(pdlp_batch *b, double *Dr, double *Dc, double *scaled_val);
int pdlp_batch_get_internal(pdlp_batch *b, int32_t *row_ptr, int32_t *col, double *val, int32_t *t_row_ptr,
                            int32_t *t_col, double *t_val, int32_t *row_perm, int32_t *col_perm);

#ifdef __cplusplus
}
#endif

#endif /* PDLP_GNN_H */
