/*
 * lbm_no: the warm-start network of the axisymmetric lattice Boltzmann
 * solver (lbm_axi.h) on MI355X (gfx950).
 *
 * A convolutional encoder-decoder maps six feature planes of an annulus
 * problem (normalised log10 Ra, log10 Da, porosity, log10 Pr, ln R* and the
 * radius r / r_o of each node) to three planes, u_z / U, u_r / U and T
 * (U = Ma c_s), on the same height x width grid; the prediction is the start
 * state handed to lbm_axi_create (init_uzurT), from which the lattice
 * Boltzmann iteration runs to its own steady-state criterion.
 *
 * Layers (all 3x3 with zero padding 1 unless stated; relu after each but the
 * last; widths c1..c4):
 *   e1 = relu(conv(x, 6 -> c1))                   H
 *   e2 = relu(conv(e1, c1 -> c2, stride 2))        H / 2
 *   e3 = relu(conv(e2, c2 -> c3, stride 2))        H / 4
 *   e4 = relu(conv(e3, c3 -> c4, stride 2))        H / 8
 *   d1 = relu(conv(up2(e4), c4 -> c3)) + e3        H / 4
 *   d2 = relu(conv(up2(d1), c3 -> c2)) + e2        H / 2
 *   d3 = relu(conv(up2(d2), c2 -> c1)) + e1        H
 *   y  = conv1x1(d3, c1 -> 3)
 * up2 repeats each value over a 2 x 2 block.  Loss: mean of (y - target)^2.
 * Optimiser: Adam with bias correction.
 *
 * Arithmetic: the convolutions run as GEMMs on MFMA with bfloat16 operands
 * (rounded to nearest even) and FP32 accumulation: weights, activations and
 * activation gradients, or, where a layer runs in an equivalent form, the
 * sums those forms take first (the taps of an upsampling layer that meet one
 * source pixel, the 2 x 2 sums of its output gradient).  Master weights, Adam
 * moments, biases, activations and gradients are FP32.
 *
 * Parameters are packed layer by layer: W[cout][cin][k][k] then b[cout]
 * (FP32).  Tensors passed in or out are device arrays in
 * [batch][channel][height][width] order.  H and W must be multiples of 8.
 *
 * Conventions as in lbm_axi.h: 0 or a negative LBM_NO_E* code, nothing
 * aborts; lbm_no_last_error() describes the last failure of this thread;
 * handles are not thread-safe; all work is ordered on the handle's stream.
 */
#ifndef LBM_NO_H
#define LBM_NO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { LBM_NO_OK = 0, LBM_NO_EINVAL = -1, LBM_NO_ENOMEM = -2, LBM_NO_EDEVICE = -3 };

typedef struct lbm_no lbm_no;

/* Number of packed parameters for widths[4] = {c1, c2, c3, c4}, each in
 * [1, 1024]. */
int lbm_no_param_count(const int32_t* widths, int64_t* count);

/*
 * Network for height x width inputs and batches of at most max_batch.
 * params: host array of lbm_no_param_count floats (copied).  hip_stream:
 * the hipStream_t all work is ordered on; NULL is the null (default) stream.
 * Widths even, in [2, 1024]; height and width multiples of 8 in [8, 2048];
 * max_batch >= 1 with max_batch * height * width <= 2^25.  Other values:
 * LBM_NO_EINVAL.
 */
int lbm_no_create(const int32_t* widths, int32_t height, int32_t width, int32_t max_batch,
                  const float* params, void* hip_stream, lbm_no** out);

/* y[batch][3][H][W] = network(x[batch][6][H][W]); device pointers. */
int lbm_no_forward(lbm_no* h, const float* x, int32_t batch, float* y);

/*
 * Forward pass, loss against target[batch][3][H][W] (device) and the
 * gradient of the loss with respect to every parameter (kept in the handle).
 * *loss (host, may be NULL) receives the loss; the call then waits for the
 * stream.
 */
int lbm_no_gradients(lbm_no* h, const float* x, const float* target, int32_t batch, double* loss);

/* One Adam step with the kept gradients (step counter kept in the handle). */
int lbm_no_adam(lbm_no* h, float lr, float beta1, float beta2, float eps);

/* Copy the parameters (which = 0) or the last gradients (which = 1) to host. */
int lbm_no_get(lbm_no* h, int32_t which, float* host_out);

/* Replace the parameters (host array) and reset the Adam state. */
int lbm_no_set_params(lbm_no* h, const float* params);

/* Wait for the handle's stream. */
int lbm_no_sync(lbm_no* h);

void lbm_no_destroy(lbm_no* h);

const char* lbm_no_last_error(void);

#ifdef __cplusplus
}
#endif

#endif
