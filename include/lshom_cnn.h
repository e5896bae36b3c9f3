/*
 * lshom_cnn: the learned initial guess for the CG solve of lshom.h.
 *
 * The paper starts CG from e = E (Sec. 2.3, the solution of the collocation
 * system Eq. (15)); any initial guess whose admissible part E + P(x0) is used
 * leaves the converged answer unchanged and moves only the iteration count.
 * This network predicts that guess for 2-D two-phase images: a four-level
 * U-Net (widths c0, 2c0, 4c0, 8c0; two circular 3x3 convolutions + ReLU per
 * level, 3x3 stride-3 convolutions between levels, nearest x3 upsampling +
 * 3x3 convolution on the way up, skip concatenation, 1x1 head to 2 channels)
 * with input (phase != 0, log10(contrast) / 4) and output the fluctuation
 * e - E of the load case E = e1.  The load case e2 uses the prediction for the
 * transposed image (the two cases are exchanged by transposition).
 *
 * Arithmetic: bfloat16 weights and activations (round to nearest even), FP32
 * accumulation on the matrix cores, FP32 master weights and Adam moments.
 * Images are square, N divisible by 27 (three x3 levels).
 *
 * Memory: the caller owns all device memory.  The parameter buffer
 * (lshom_cnn_param_size) holds master weights, gradients, Adam moments and
 * bfloat16 copies; the workspace (lshom_cnn_workspace_size) holds the
 * activations of one (batch, N) shape.  Status codes are those of lshom.h;
 * lshom_cnn_last_error gives a message.  Calls are blocking and ordered after
 * work already queued on the stream given at creation.
 */
#ifndef LSHOM_CNN_H
#define LSHOM_CNN_H

#include <stddef.h>
#include <stdint.h>

#include "lshom.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lshom_cnn lshom_cnn;

/* base_channels = c0 (32 for the product network). */
lshom_status lshom_cnn_create(lshom_cnn** out, int device, void* hip_stream, int base_channels);
void lshom_cnn_destroy(lshom_cnn* net);
const char* lshom_cnn_last_error(const lshom_cnn* net);

/*
 * n_params: number of parameters in the compact order used by
 * lshom_cnn_set_params / get_params / get_grads: for every layer in
 * execution order (enc0a enc0b down0 enc1a enc1b down1 enc2a enc2b down2
 * bot_a bot_b up2 dec2a dec2b up1 dec1a dec1b up0 dec0a dec0b head) the
 * weights w[p][q][c][o] (3x3 layers) or w[c][o] (head), then the bias[o].
 * buffer_bytes: size of the device parameter buffer.
 */
lshom_status lshom_cnn_param_size(lshom_cnn* net, int64_t* n_params, size_t* buffer_bytes);
lshom_status lshom_cnn_set_param_buffer(lshom_cnn* net, void* dev, size_t bytes);
/* Host FP32 parameters in the compact order; resets the Adam state. */
lshom_status lshom_cnn_set_params(lshom_cnn* net, const float* host, int64_t n);
lshom_status lshom_cnn_get_params(lshom_cnn* net, float* host, int64_t n);
/* Gradients of the last lshom_cnn_train_step, compact order. */
lshom_status lshom_cnn_get_grads(lshom_cnn* net, float* host, int64_t n);

/* Activation workspace for batch images of N x N; training adds the
 * backward buffers. */
lshom_status lshom_cnn_workspace_size(lshom_cnn* net, int batch, int n, int training, size_t* bytes);
lshom_status lshom_cnn_set_workspace(lshom_cnn* net, void* dev, size_t bytes, int batch, int n, int training);

/*
 * Prediction for batch images (phase_dev: uint8 [batch][n][n], nonzero =
 * the inclusion phase; log10_rho_dev: float [batch] contrasts).  load_axis 0
 * predicts the field of E = e1, 1 that of E = e2.  scale 1 runs the network
 * on the n x n image; scale 3 runs it on the n/3 x n/3 image whose pixels
 * are the majority phase of 3 x 3 blocks and spreads each prediction over
 * its block (the workspace is then set for n/3).  e_dev (may be NULL): FP64
 * [batch][2][n][n], E + prediction (usable as x0_dev of lshom_solve).
 * raw_dev (may be NULL): FP32 [batch][n/scale][n/scale][2], the network
 * output.
 */
lshom_status lshom_cnn_forward(lshom_cnn* net, const uint8_t* phase_dev, const float* log10_rho_dev, int batch,
                               int n, int load_axis, int scale, double* e_dev, float* raw_dev);

/*
 * One training step on a batch: target fields e_dev FP64 [batch][2][n][n]
 * (solutions for E = e1); loss = mean over the batch of
 * ||pred - (e - E)||^2 / ||e - E||^2, written to loss_host.  update != 0
 * applies an Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr)
 * to the master weights; update == 0 only computes the gradients.
 */
lshom_status lshom_cnn_train_step(lshom_cnn* net, const uint8_t* phase_dev, const float* log10_rho_dev,
                                  const double* e_dev, int batch, int n, float lr, int update, double* loss_host);

/*
 * Layer calls: one convolution of the network (the building blocks of
 * lshom_cnn_forward and lshom_cnn_train_step) on caller tensors, with the
 * bfloat16 copies of the parameters last set or updated.  layer: index in
 * the execution order above (0 = enc0a ... 20 = head).  The shape is that of
 * the workspace set last (batch images of n x n); layer l works on its
 * level's grid: output side ho = n / 3^level, input side hi = ho except
 * 3 ho for the down layers (3x3 stride-3 convolution) and ho / 3 for the up
 * layers (whose convolution reads the nearest-neighbour upsampling of its
 * input).  Tensors are NHWC; bfloat16 tensors are raw 16-bit words.  cin is
 * the channel count the layer reads (8 for enc0a, whose channels 2..7 meet
 * zero weights), cout its output channels, cout8 = cout rounded up to 8.
 *
 * lshom_cnn_layer_forward: x_dev bf16 [batch][hi][hi][cin]; the FP32 value
 *   y = bias + conv(x, w), then ReLU except for the head, goes rounded to
 *   nearest even into y_dev (bf16 [batch][ho][ho][cout]) and as is into
 *   yf_dev (FP32, same shape); either may be NULL, not both.
 * lshom_cnn_layer_dgrad: gy_dev bf16 [batch][ho][ho][cout8], the gradient at
 *   the layer's pre-activation output (channels >= cout finite; they meet
 *   zero weights); gx_dev FP32 [batch][hi][hi][cin] receives the gradient
 *   with respect to the layer's input (the adjoint of the convolution, and
 *   for up layers that of the upsampling: the sum over each 3 x 3 block).
 *   Needs a training workspace.
 * lshom_cnn_layer_wgrad: x_dev, gy_dev as above; the layer's weight and bias
 *   gradients (sums over all pixels of the batch) overwrite its entries of
 *   the gradient buffer (read with lshom_cnn_get_grads; the other layers'
 *   entries are unchanged).  Needs a training workspace.
 * Products of bfloat16 values are exact in FP32; the sums are FP32 (matrix
 * cores, then a fixed-order sum of the weight gradient's pixel splits).
 * Blocking; INVALID_ARG for NULL pointers or a layer out of range,
 * STATE / WORKSPACE when parameters or a suitable workspace are missing.
 */
lshom_status lshom_cnn_layer_forward(lshom_cnn* net, int layer, const uint16_t* x_dev, uint16_t* y_dev,
                                     float* yf_dev);
lshom_status lshom_cnn_layer_dgrad(lshom_cnn* net, int layer, const uint16_t* gy_dev, float* gx_dev);
lshom_status lshom_cnn_layer_wgrad(lshom_cnn* net, int layer, const uint16_t* x_dev, const uint16_t* gy_dev);

#ifdef __cplusplus
}
#endif

#endif /* LSHOM_CNN_H */
