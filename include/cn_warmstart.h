/* Learned initial guess for the all-at-once CN solve.
 *
 * GMRES applied to the preconditioned system reduces the residual it starts
 * from (the minimal-residual property and its bound, Sec. 4, eq. (4.1)): the
 * bound is proportional to the initial residual, so a better initial guess
 * u_0 saves iterations.  This library part predicts u_0 from the coefficients
 * of a problem: a small network maps features of the problem (volatility
 * samples and scalar parameters) to a coarse 128 x 64 space-time solution,
 * which is interpolated to the fine grid.  The solver itself takes the guess
 * through cn_gmres_opts.use_x0 (cn_aao.h); use_x0 = 2 falls back to a zero
 * start for any instance where the guess does not reduce the residual below
 * ||b||, so a poor prediction cannot make a solve worse than the plain method.
 *
 * Network: n_in -> w -> w -> w -> n_out, ReLU after the three hidden layers,
 * linear output.  Parameters are one flat float32 array (the masters), in the
 * order W1 [w x n_in], b1 [w], W2 [w x w], b2 [w], W3 [w x w], b3 [w],
 * W4 [n_out x w], b4 [n_out], matrices row-major with one row per output unit.
 * Products run on the matrix cores in bf16 (weights rounded from the masters,
 * activations and gradients rounded as they are staged) with float32
 * accumulation; bias, ReLU, loss, bias gradients and Adam run in float32.
 *
 * All array arguments are device pointers unless stated otherwise; every
 * call is asynchronous on the network's stream (or the given stream) and
 * returns CN_EINVAL for NULL or out-of-range arguments, CN_ENOMEM / CN_EHIP
 * for device failures (message in cn_ws_last_error()).
 */
#ifndef CN_WARMSTART_H
#define CN_WARMSTART_H

#include <stdint.h>

#include "cn_aao.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cn_mlp cn_mlp;

/* Create a network with zero parameters and zero Adam moments; activation
 * buffers are sized for batches of up to max_batch rows.  stream: hipStream_t
 * or NULL for the default stream.  On failure *out is NULL. */
cn_status cn_mlp_create(int32_t n_in, int32_t width, int32_t n_out, int32_t max_batch,
                        void *stream, cn_mlp **out);
/* Synchronises the network's stream and releases everything. */
cn_status cn_mlp_destroy(cn_mlp *net);

/* Number of float32 parameters (host output). */
cn_status cn_mlp_num_params(const cn_mlp *net, int64_t *n);
/* Copy the flat parameter array in (resets the Adam moments and step count)
 * or out. */
cn_status cn_mlp_set_params(cn_mlp *net, const float *params);
cn_status cn_mlp_get_params(const cn_mlp *net, float *params);

/* Standardisation constants (float32, device): the network sees
 * (x - in_mean) / in_scale (n_in values each) and its last layer produces
 * z, reported as y = out_mean + out_scale * z (n_out values each); the
 * training loss compares z with (target - out_mean) / out_scale.  Defaults:
 * means 0, scales 1.  Scales must be non-zero (not checked). */
cn_status cn_mlp_set_normalization(cn_mlp *net, const float *in_mean, const float *in_scale,
                                   const float *out_mean, const float *out_scale);

/* Y [B x n_out] = network(X [B x n_in]), rows = samples, 1 <= B <= max_batch. */
cn_status cn_mlp_forward(cn_mlp *net, const float *X, int32_t B, float *Y);

/* Forward pass, mean-squared error against Yt [B x n_out] in standardised
 * units (loss = mean over all B*n_out entries of (z - (Yt - out_mean) /
 * out_scale)^2, z the last layer's output) and the gradient of
 * that loss with respect to every parameter, kept in the network for
 * cn_mlp_adam_step.  grads (flat, parameter order; may be NULL) receives a
 * copy of the gradient, loss (one float, device; may be NULL) the loss. */
cn_status cn_mlp_loss_grad(cn_mlp *net, const float *X, const float *Yt, int32_t B,
                           float *grads, float *loss);

/* One Adam update of the masters with the gradient of the last
 * cn_mlp_loss_grad (bias-corrected moments, no weight decay), then the bf16
 * copies are refreshed.  Requires lr > 0, 0 <= beta1, beta2 < 1, eps > 0. */
cn_status cn_mlp_adam_step(cn_mlp *net, float lr, float beta1, float beta2, float eps);

/* Coarse grid of the prediction: 128 points in space (cell centres of 128
 * equal cells between the two Dirichlet ends) by 64 levels in time
 * (t = (q+1) T / 64), stored [q][c] (8192 floats per instance).  A fine grid
 * of nx interior points and nt levels (the all-at-once layout, row k = level
 * k+1) is compatible when nx + 1 is a multiple of 128 with ratio >= 2 and nt
 * is a multiple of 64; CN_EINVAL otherwise.
 *
 * cn_ws_restrict: coarse[i] = inv_scale[i] * x_i at the fine points that
 * coincide with the coarse nodes, for `count` instances of one shape packed
 * back to back (x: count*nx*nt doubles, inv_scale: count doubles, coarse:
 * count*8192 floats).
 *
 * cn_ws_interpolate: x0_i = bilinear interpolation of scale[i] * coarse_i on
 * the coarse grid extended by the initial condition u0_i at t = 0 (nx values
 * each) and the Dirichlet data gl_i, gr_i at the two space ends (nt values
 * each, at the fine levels); x0 as x above. */
cn_status cn_ws_restrict(const double *x, int32_t count, int32_t nx, int32_t nt,
                         const double *inv_scale, float *coarse, void *stream);
cn_status cn_ws_interpolate(const float *coarse, int32_t count, int32_t nx, int32_t nt,
                            const double *u0, const double *gl, const double *gr,
                            const double *scale, double *x0, void *stream);

/* The initial guess in one call: the network's forward pass on `count`
 * feature rows (device, count x n_in, run in chunks of max_batch), the
 * de-standardised coarse prediction into `coarse` (device workspace,
 * count x 8192 floats, left holding the prediction), then cn_ws_interpolate
 * into x0 -- all on the network's stream.  The network must have
 * n_out = 8192. */
cn_status cn_ws_predict(cn_mlp *net, const float *features, int32_t count, int32_t nx,
                        int32_t nt, const double *u0, const double *gl, const double *gr,
                        const double *scale, float *coarse, double *x0);

/* The initial guess of every instance of a batch in one call, instances of
 * uneven N_x and N_t included: the network's forward pass on the batch's
 * feature rows (features: count x n_in, count = the batch's instances, in
 * chunks of max_batch) into `coarse` (count x 8192 floats, left holding the
 * predictions), then each instance's interpolation to its own grid, written
 * into x0 at the batch's packed offsets (cn_batch_offsets).  u0: the packed
 * initial conditions (space offsets of cn_batch_offsets), gl, gr: the packed
 * Dirichlet data at the levels t_{k+1} (instance i's N_t values after those of
 * the instances before it), scale: count factors.  Every instance needs
 * N_x + 1 a multiple of 128 (>= 256) and N_t a multiple of 64 (CN_EINVAL
 * otherwise).  All on the network's stream.  Device pointers throughout. */
cn_status cn_ws_predict_batch(cn_mlp *net, const float *features, const cn_batch *b,
                              const double *u0, const double *gl, const double *gr,
                              const double *scale, float *coarse, double *x0);

const char *cn_ws_last_error(void);

#ifdef __cplusplus
}
#endif

#endif
