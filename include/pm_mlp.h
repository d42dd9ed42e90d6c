/*
 * pm_mlp.h -- learned surrogate of the particle forward map (part of libpm.so).
 *
 * A multilayer perceptron maps the unknown u (the stream-function coefficients
 * of eq. v_expand) to the N_o observations G(u) of eq. Gmap:
 *     h_0 = u * in_scale,  h_l = GELU(h_{l-1} W_l + b_l)  (l = 1..L),
 *     y = h_L W_{L+1} + b_{L+1},  G(u) ~ y * out_std + out_mean,
 * with GELU(z) = z Phi(z) (exact, erf form).  It is trained on (u, G(u))
 * pairs produced by the particle map itself and serves as the first stage of
 * delayed-acceptance pCN; the particle map still decides acceptance.
 *
 * Arithmetic: matrix products run on the MFMA units in BF16 with FP32
 * accumulation (v_mfma_f32_16x16x32_bf16); master weights, Adam moments,
 * biases, pre-activations, the loss and all gradients are FP32.
 *
 * Parameters in "logical" order (used by get/set/grads), FP32:
 *     W_1 [d_in][h], b_1 [h], W_2 [h][h], b_2 [h], ..., W_{L+1} [h][d_out], b_{L+1} [d_out]
 * (row-major, W_l maps its input index to its output index).
 * All data arrays are device pointers unless marked host; calls enqueue on the
 * context's stream.  Errors as in pm.h.
 */
#ifndef PM_MLP_H
#define PM_MLP_H

#include <stdint.h>

#include "pm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pm_mlp pm_mlp;

/* d_in, d_hidden, d_out >= 1, n_hidden >= 1 hidden layers, max_batch >= 1
 * rows per call.  Weights are drawn on the host from N(0, 1/fan_in) with the
 * given seed, biases zero; in_scale = 1, out_mean = 0, out_std = 1. */
int pm_mlp_create(pm_ctx *ctx, int d_in, int d_hidden, int n_hidden, int d_out, int max_batch,
                  uint64_t seed, pm_mlp **out);
void pm_mlp_destroy(pm_mlp *m);

/* Number of logical parameters. */
int64_t pm_mlp_n_params(const pm_mlp *m);

/* Copy parameters (logical order, FP32) from / to host memory.  set also
 * resets the Adam moments and step count.  Synchronous. */
int pm_mlp_set_params(pm_mlp *m, const float *host_params);
int pm_mlp_get_params(pm_mlp *m, float *host_params);

/* Input scaling and output de-standardisation (host arrays of d_in, d_out,
 * d_out floats; any may be NULL to keep the current value). Synchronous. */
int pm_mlp_set_io(pm_mlp *m, const float *in_scale, const float *out_mean, const float *out_std);

/* y = G~(x) in physical units.  x device [n][d_in] FP32, y device [n][d_out]
 * FP32, 1 <= n <= max_batch. */
int pm_mlp_forward(pm_mlp *m, const float *x, int n, float *y);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on the
 * mean squared error between the standardised output and the standardised
 * target t (device [n][d_out], physical units):
 *     L = 1/(n d_out) sum ((y - t) / out_std)^2.
 * loss (device FP32 [1], nullable) receives L for this batch. */
int pm_mlp_train_step(pm_mlp *m, const float *x, const float *t, int n, float lr, float *loss);

/* Gradient of L (as in pm_mlp_train_step) with respect to every parameter,
 * logical order, into host memory (n_params floats); no update.  Synchronous. */
int pm_mlp_grads(pm_mlp *m, const float *x, const float *t, int n, float *host_grads);

#ifdef __cplusplus
}
#endif

#endif /* PM_MLP_H */
