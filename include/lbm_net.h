/*
 * liblbm, warm-start network: a convolutional encoder-decoder that predicts the
 * steady density and velocity of a channel from its wall mask, electric force
 * and interaction strength, trained and evaluated by the library's own HIP
 * kernels.  The prediction seeds the lattice through lbm_init_device /
 * lbm_batch_init_device (populations at the equilibrium of eq. (3) of the
 * predicted density and velocity); the lattice Boltzmann steps of eqs. (1)-(10)
 * then decide the result, so a poor prediction costs steps, not accuracy.
 * The network itself is not part of the paper.
 *
 * Network (H and W multiples of 8; periodic in x, zero-padded in y):
 *   e1 = relu(conv(relu(conv(x))))                     cin -> c1 -> c1,   H x W
 *   e2 = the same on avgpool(e1)                        c1 -> c2 -> c2,   H/2
 *   e3 = the same on avgpool(e2)                        c2 -> c3 -> c3,   H/4
 *   b  = the same on avgpool(e3)                        c3 -> c4 -> c4,   H/8
 *   d3 = the same on concat(upsample(b), e3)       c4+c3 -> c3 -> c3
 *   d2 = the same on concat(upsample(d3), e2)      c3+c2 -> c2 -> c2
 *   d1 = the same on concat(upsample(d2), e1)      c2+c1 -> c1 -> c1
 *   y  = conv1x1(d1)                                    c1 -> cout (linear)
 * conv is 3x3 with bias; avgpool averages 2x2; upsample repeats each value 2x2.
 * Loss: mean over fluid nodes and output planes of (y - t)^2.  Optimiser: Adam
 * with bias correction.
 *
 * Parameters: one FP32 vector; for the 15 layers in the order above
 * (e1a, e1b, e2a, e2b, e3a, e3b, b_a, b_b, d3a, d3b, d2a, d2b, d1a, d1b, out),
 * the weights W[cout][cin][ky][kx] then the biases b[cout].
 *
 * Conventions are those of lbm.h: lbm_status return codes, no exceptions, the
 * caller owns every array and the 256-byte aligned device workspace, all GPU
 * work runs on the stream given to lbm_net_create.  Tensors x, y and t are
 * device FP32 arrays [n][planes][H][W] (x fastest); fluid is a device uint8
 * array [n][H][W], nonzero where the loss counts.  Activations are stored in
 * bf16 (act_bf16 = 1) or FP32 (act_bf16 = 0, the checking build).  With bf16
 * activations the forward 3x3 convolutions after the first run on matrix
 * cores with the weights rounded to bf16 and FP32 accumulation, and so do the
 * input-gradient convolutions of the backward pass, with the layer gradient
 * and the weights rounded to bf16, and the weight gradients of those layers,
 * with the layer gradient rounded to bf16 against the bf16 activations;
 * everything else (and the FP32 build throughout) multiplies and sums in
 * FP32.  The loss is reduced in FP64;
 * master weights, gradients and Adam moments are FP32.
 */
#ifndef LBM_NET_H
#define LBM_NET_H

#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t H, W;      /* lattice rows and columns, multiples of 8           */
    int32_t batch;     /* largest n a call may pass, 1..512                  */
    int32_t cin, cout; /* input and output planes, 1..2048                   */
    int32_t chans[4];  /* c1..c4, 1..2048 each; the widest layer (including
                          the concatenations c4 + c3, c3 + c2, c2 + c1) times
                          H x W must be below 2^31                          */
    int32_t act_bf16;  /* 1: bf16 activations, 0: FP32 activations          */
} lbm_net_config;

typedef struct lbm_net lbm_net;

/* Number of FP32 parameters, or -1 for an invalid configuration. */
int64_t lbm_net_param_count(const lbm_net_config *cfg);

/* Device workspace bytes for cfg (activations and gradients for `batch`
 * samples, parameters, Adam moments, scratch), or 0 if cfg is invalid. */
size_t lbm_net_workspace_bytes(const lbm_net_config *cfg);

/* Create a network in the caller's workspace on `stream` (a hipStream_t, NULL
 * for the default stream).  Parameters and Adam moments start at zero: call
 * lbm_net_set_params before use.  LBM_EINVAL for a bad configuration or an
 * unaligned workspace, LBM_ENOMEM if it is too small. */
lbm_status lbm_net_create(lbm_net **net, const lbm_net_config *cfg, void *workspace, size_t bytes, void *stream);

/* Copy `count` host FP32 parameters in (and reset Adam) or out.  Synchronous. */
lbm_status lbm_net_set_params(lbm_net *net, const float *host, int64_t count);
lbm_status lbm_net_get_params(lbm_net *net, float *host, int64_t count);

/* y = network(x) for n samples, 1 <= n <= batch.  Asynchronous. */
lbm_status lbm_net_forward(lbm_net *net, const float *x, float *y, int32_t n);

/* Loss and gradient with respect to the parameters for n samples; the loss is
 * written to *loss and, if grad_host is not NULL, the gradient to grad_host
 * (param_count floats).  The gradient stays on the device for lbm_net_adam.
 * Synchronous. */
lbm_status lbm_net_gradient(lbm_net *net, const float *x, const float *t, const uint8_t *fluid, int32_t n,
                            double *loss, float *grad_host);

/* One Adam step with the last gradient (LBM_ESTATE if there is none).
 * Asynchronous. */
lbm_status lbm_net_adam(lbm_net *net, float lr, float beta1, float beta2, float eps);

/* Gradient then Adam (beta1 0.9, beta2 0.999, eps 1e-8) on n samples; *loss,
 * if not NULL, receives the loss before the update (then the call is
 * synchronous). */
lbm_status lbm_net_train_step(lbm_net *net, const float *x, const float *t, const uint8_t *fluid, int32_t n,
                              float lr, double *loss);

/* Release the handle (not the workspace). */
void lbm_net_free(lbm_net *net);

/* Message of the last error of `net`, or of the last failed create if NULL. */
const char *lbm_net_last_error(const lbm_net *net);

#ifdef __cplusplus
}
#endif
#endif /* LBM_NET_H */
