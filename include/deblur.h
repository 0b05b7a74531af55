/*
 * deblur.h - C ABI of the deblurring network in libfwi.so: a UNet-like
 * convolutional encoder-decoder that learns the action of the inverse
 * Gauss-Newton Hessian (paper section 2.3 and section 2.4, architecture in
 * Appendix A, Table 1). It is trained to map the doubly migrated image
 * dm1 = J^T J g (eq. 15) to the gradient g, then applied to g to give the
 * preconditioned update direction; its weights carry over from one FWI
 * iteration to the next (transfer learning, section 2.3) and are reset at a
 * new frequency band.
 *
 * Network (depth D, base width B, C_l = B * 2^l):
 *   input block   conv3x3(1 -> C_0), act, conv3x3(C_0 -> C_0), act
 *   down l=1..D   avgpool 3x3 stride 2 pad 1 (zero padding counted),
 *                 conv3x3(C_{l-1} -> C_l), act, conv3x3(C_l -> C_l), act
 *   up l=D-1..0   transposed conv 2x2 stride 2 (C_{l+1} -> C_l, bias),
 *                 concatenation [encoder features of level l, up-sampled],
 *                 conv3x3(2 C_l -> C_l), act, conv3x3(C_l -> C_l), act
 *   output        conv1x1(C_0 -> 1), no activation
 * with 3x3 convolutions of stride 1 and zero padding 1, biases on every
 * convolution and act(x) = x for x > 0, slope * x otherwise (slope 0 is
 * ReLU, 0.2 the paper's LeakyReLU).
 *
 * Arithmetic: bf16 activations and weights on the matrix cores with FP32
 * accumulation; FP32 master weights, gradients and Adam state.
 *
 * Parameter vector (deblur_get_params / deblur_set_params): FP32, host
 * memory, the tensors concatenated in this order, each in PyTorch's layout:
 *   input block  W[C0][1][3][3], b[C0], W[C0][C0][3][3], b[C0]
 *   down l       W[C_l][C_{l-1}][3][3], b[C_l], W[C_l][C_l][3][3], b[C_l]
 *   up l         Wt[C_{l+1}][C_l][2][2], bt[C_l], W[C_l][2C_l][3][3], b[C_l],
 *                W[C_l][C_l][3][3], b[C_l]          (l = D-1 down to 0)
 *   output       W[1][C0][1][1], b[1]
 *
 * Images (x, y of deblur_train / deblur_apply) are device FP32 [nz][nx]
 * with nz <= in_h, nx <= in_w: they are scaled by 1 / max|.| and
 * reflect-padded to in_h x in_w, floor((in_h - nz) / 2) rows above and the
 * rest below (columns alike: floor((in_w - nx) / 2) on the left), each
 * padding narrower than the image; the network
 * output is cropped back and multiplied by max|x| (apply). Training uses
 * the MSE loss on the padded grid, Adam (beta 0.9, 0.999, eps 1e-8) with a
 * cosine-annealed learning rate from lr_max to 0 over the call's steps; Adam
 * state and the schedule restart at every deblur_train call, the weights do
 * not.
 *
 * Errors: FWI_* codes of fwi.h; deblur_last_error(net) gives a message.
 */
#ifndef DEBLUR_H
#define DEBLUR_H

#include <stdint.h>

#include "fwi.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct deblur_net deblur_net;

typedef struct {
    int32_t depth;      /* number of down-sampling blocks, >= 1 */
    int32_t base_ch;    /* C_0, multiple of 8 */
    float leaky_slope;  /* 0 = ReLU */
    int32_t in_h, in_w; /* network grid, divisible by 2^depth */
} deblur_cfg;

/* Create a network on the context's device with weights drawn from the
 * default initialisation (uniform +-1/sqrt(fan_in), seeded). */
int deblur_create(fwi_ctx *ctx, const deblur_cfg *cfg, uint64_t seed, deblur_net **out);
void deblur_destroy(deblur_net *net);
const char *deblur_last_error(const deblur_net *net);
int deblur_num_params(const deblur_net *net, int64_t *n);
/* Host FP32 parameter vector in the order documented above. */
int deblur_set_params(fwi_ctx *ctx, deblur_net *net, const float *params);
int deblur_get_params(fwi_ctx *ctx, const deblur_net *net, float *params);
/* Re-draw the weights (a new frequency band, section 4 of the paper). */
int deblur_reset(fwi_ctx *ctx, deblur_net *net, uint64_t seed);

/* Train for `steps` Adam steps on the pair (x_blurred -> y_target), both
 * device FP32 [nz][nx]; loss_hist (host, nullable) receives the MSE of
 * every step (before that step's update). Waits for completion. */
int deblur_train(fwi_ctx *ctx, deblur_net *net, const float *x_blurred, const float *y_target, int32_t nz,
                 int32_t nx, int32_t steps, float lr_max, float *loss_hist);
/* Steps first .. first+count-1 of a training run of `total` steps on the
 * pair (x_blurred -> y_target), as deblur_train runs them: the cosine
 * schedule spans the run's `total` steps and the Adam moments carry from
 * one call to the next, so a run split over several calls (to watch the
 * loss, stop early or inspect the weights between steps) gives the same
 * weights as one deblur_train(total) call. first = 0 starts a run (moments
 * zeroed); first > 0 must continue the run the previous call on this
 * network left at step `first`, with the same total and lr_max, else
 * FWI_ESTATE (deblur_set_params, deblur_reset and deblur_load end a run;
 * deblur_grad_raw, deblur_forward_raw, deblur_apply and deblur_get_params
 * leave it). loss_hist (host, nullable) receives `count` losses. Waits for
 * completion. deblur_train(steps) is deblur_train_range(0, steps, steps). */
int deblur_train_range(fwi_ctx *ctx, deblur_net *net, const float *x_blurred, const float *y_target,
                       int32_t nz, int32_t nx, int32_t first, int32_t count, int32_t total, float lr_max,
                       float *loss_hist);
/* y = max|x| * N(pad(x / max|x|)) cropped to [nz][nx]; device FP32. */
int deblur_apply(fwi_ctx *ctx, deblur_net *net, const float *x, int32_t nz, int32_t nx, float *y);

/* The network on its own grid, without scaling or padding: y = N(x),
 * x and y device FP32 [in_h][in_w]. */
int deblur_forward_raw(fwi_ctx *ctx, deblur_net *net, const float *x, float *y);
/* Loss 1/P sum (N(x) - t)^2 on the network grid and its gradient with
 * respect to every parameter (host FP32, parameter-vector order), without
 * updating the weights. x, t: device FP32 [in_h][in_w]. */
int deblur_grad_raw(fwi_ctx *ctx, deblur_net *net, const float *x, const float *t, double *loss,
                    float *grads);

/* Per-layer timing of the convolution GEMMs. With profiling on, every
 * matrix-core launch of the network (forward, data-gradient and
 * weight-gradient GEMMs of each convolution) is bracketed by HIP events;
 * deblur_layer_stats waits for the stream, then writes up to `max` records
 * (one per layer and pass, times summed over all launches since profiling
 * was switched on) and their count. Switching profiling on clears them. */
typedef struct {
    char name[24];      /* "inc.1", "down2.2", "up1.T", ... */
    int32_t pass;       /* 0 forward, 1 data gradient, 2 weight gradient */
    int32_t M, N, K;    /* GEMM shape: outputs x pixels x reduction (wgrad: M x N over K pixels) */
    int64_t calls;
    double flops;       /* 2 M N K per call, summed */
    double ms;          /* summed kernel time */
} deblur_layer_stat;
int deblur_set_profiling(deblur_net *net, int enable);
int deblur_layer_stats(fwi_ctx *ctx, deblur_net *net, deblur_layer_stat *out, int32_t max, int32_t *count);

/* Weights (FP32, parameter-vector order) to / from a file with a small
 * header holding the configuration. */
int deblur_save(fwi_ctx *ctx, const deblur_net *net, const char *path);
int deblur_load(fwi_ctx *ctx, deblur_net *net, const char *path);

#ifdef __cplusplus
}
#endif

#endif /* DEBLUR_H */
