/*
 * rlbm_surrogate.h -- C ABI of the convolutional warm-start surrogate of the
 * rlbm library (gfx950): a U-Net that maps a lattice description (solid
 * mask, source and drain contact masks, tau and drive planes) to the steady
 * density and velocity fields, trained on steady states the lattice
 * Boltzmann solver itself produces and used to initialise it (the solver
 * has the last word: a warm start that fails its health check falls back to
 * a cold start).
 *
 * Network: NHWC input with cin channels (a multiple of 16; unused channels
 * zero), H and W multiples of 16.  Encoder blocks of two 3x3 convolutions
 * (zero padding) + bias + ReLU at widths c, 2c, 4c, 8c with 2x2 average
 * pooling between them, a bottleneck block at 8c, decoder blocks that
 * upsample (nearest, x2), concatenate [upsampled, skip] along channels and
 * apply two 3x3 convolutions + ReLU, and a 1x1 head to cout channels.
 * Parameters form one flat FP32 vector: for each layer in order (e1a, e1b,
 * e2a, e2b, e3a, e3b, e4a, e4b, ba, bb, d4a, d4b, d3a, d3b, d2a, d2b, d1a,
 * d1b, head), W[cout][kh][kw][cin] then b[cout].
 *
 * Precision: BF16 activations and weights on the matrix cores
 * (v_mfma_f32_16x16x32_bf16 / 16x16x16), FP32 accumulation, FP32 master
 * weights, gradients and Adam moments, FP32 output.  The loss is the mean
 * squared error.  Every call returns an rlbm_status (rlbm.h) and is ordered
 * on the network's stream; device pointers are caller-owned.
 */
#ifndef RLBM_SURROGATE_H
#define RLBM_SURROGATE_H

#include <stddef.h>
#include <stdint.h>

#include "rlbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rlbm_unet rlbm_unet;

/* Create a network for inputs of max_batch x height x width x cin.
 * base: channels of the first level (multiple of 16).  Weights: seeded
 * He-normal (library's own generator), zero biases.  hip_stream may be NULL. */
rlbm_status rlbm_unet_create(int base, int cin, int cout, int height, int width, int max_batch, uint64_t seed,
                             void *hip_stream, rlbm_unet **out);
void rlbm_unet_destroy(rlbm_unet *net);

/* Number of parameters (length of the flat vector). */
rlbm_status rlbm_unet_param_count(rlbm_unet *net, int64_t *n);

/* Host copies of the FP32 parameters / accumulated gradients (n floats). */
rlbm_status rlbm_unet_set_params(rlbm_unet *net, const float *theta);
rlbm_status rlbm_unet_get_params(rlbm_unet *net, float *theta);
rlbm_status rlbm_unet_get_grads(rlbm_unet *net, float *grad);

/* y = net(x): x device FP32 batch x H x W x cin, y device FP32 batch x H x W
 * x cout.  Keeps the activations for rlbm_unet_backward. */
rlbm_status rlbm_unet_forward(rlbm_unet *net, const float *x, float *y, int batch);

/* Mean squared error of y against t (device FP32, same shape); writes the
 * loss to *loss (host) and dL/dy to dy (device, may be NULL).  Synchronises. */
rlbm_status rlbm_unet_mse(rlbm_unet *net, const float *y, const float *t, int batch, float *loss, float *dy);

/* Accumulate the parameter gradient of the loss whose gradient with respect
 * to the last forward's output is dy (device FP32).  dx (device FP32,
 * batch x H x W x cin, may be NULL) receives the input gradient. */
rlbm_status rlbm_unet_backward(rlbm_unet *net, const float *dy, int batch, float *dx);

rlbm_status rlbm_unet_zero_grad(rlbm_unet *net);

/* One Adam step (bias-corrected) on the accumulated gradient. */
rlbm_status rlbm_unet_adam_step(rlbm_unet *net, float lr, float beta1, float beta2, float eps);

/* Single 3x3 convolution layer kernels on device BF16 tensors (the
 * building blocks of the network, exposed for testing and reuse):
 * y = act(conv(x, w) + b); dx = conv(dy, adjoint(w)); gw += sum dy (x) x.
 * x: B x H x W x ci, w: co x 3 x 3 x ci, y/dy: B x H x W x co (all BF16);
 * b, gw, gb: FP32.  ci, co multiples of 16; the BF16 tensors must start on
 * 16-byte boundaries (the kernels move 8 channels per access), else
 * RLBM_EINVAL.  stream may be NULL. */
rlbm_status rlbm_conv3x3_forward(const void *x, const void *w, const float *b, void *y, int B, int H, int W, int ci,
                                 int co, int relu, void *hip_stream);
rlbm_status rlbm_conv3x3_backward_data(const void *dy, const void *w, void *dx, int B, int H, int W, int ci, int co,
                                       void *hip_stream);
rlbm_status rlbm_conv3x3_backward_weight(const void *dy, const void *x, float *gw, float *gb, int B, int H, int W,
                                         int ci, int co, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* RLBM_SURROGATE_H */
