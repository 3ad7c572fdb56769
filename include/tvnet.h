/*
 * tvnet.h -- C ABI of the warm-start network for the TVLBM solver.
 *
 * A four-layer 3x3 convolutional network (c_in -> width -> width -> width ->
 * c_out, GELU after the first three layers, zero padding) that maps a
 * geometry/parameter canvas to the steady macroscopic fields
 * (rho, ux, uy, T) of a walled channel; its prediction seeds the TVLBM solve
 * in place of a uniform start.  Forward and backward passes run in
 * hand-written bf16 matrix-core (MFMA) kernels with fp32 accumulation; the
 * optimiser is Adam with fp32 master weights.
 *
 * Conventions
 *   - Return TVLBM_OK (0) or a negative TVLBM_E* code (include/tvlbm.h).
 *   - Activations are channels-last: [batch][height][cols][channels].
 *   - Parameters, flat fp32, layer by layer: W[o][c][dy][dx] (3x3 filter of
 *     output channel o over input channel c; tap (dy, dx) reads input pixel
 *     (y + dy - 1, x + dx - 1)), then the bias b[o].
 *   - The library owns the parameters, Adam state, activations and scratch
 *     (sized for max_batch at init); the caller owns inputs and outputs.
 *   - Work runs on the given stream (NULL = default); calls that return
 *     host values synchronise it.  Not thread-safe.
 */
#ifndef TVNET_H
#define TVNET_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tvnet tvnet;

typedef struct tvnet_desc {
  int32_t c_in;       /* input channels, 1..8                                 */
  int32_t width;      /* hidden channels, 32                                  */
  int32_t c_out;      /* output channels, 1..8                                */
  int32_t height;     /* canvas rows                                          */
  int32_t cols;       /* canvas columns                                       */
  int32_t max_batch;  /* largest batch passed to forward/backward             */
  void *stream;       /* hipStream_t or NULL                                  */
} tvnet_desc;

int tvnet_init(const tvnet_desc *desc, tvnet **net);
int tvnet_destroy(tvnet *net);
/* number of parameters (flat layout above) */
int tvnet_num_params(const tvnet *net, int64_t *n);
/* host <-> library parameter copies (fp32, flat); set also resets Adam */
int tvnet_set_params(tvnet *net, const float *params);
int tvnet_get_params(tvnet *net, float *params);
/* y = net(x).  x: device fp32 [batch][height][cols][c_in]; y: device fp32
 * [batch][height][cols][c_out].  Keeps the activations for tvnet_backward. */
int tvnet_forward(tvnet *net, const void *x, void *y, int32_t batch);
/* Masked mean-squared error of the last forward against target (device fp32,
 * same shape as y) with mask (device fp32 [batch][height][cols]):
 * L = sum mask (y - t)^2 / (c_out * mask_sum); loss (host, may be NULL).
 * Back-propagates and stores the parameter gradients.  Synchronises. */
int tvnet_backward(tvnet *net, const void *target, const void *mask,
                   int32_t batch, double mask_sum, double *loss);
/* gradients of the last backward, host fp32 (flat layout) */
int tvnet_get_grads(tvnet *net, float *grads);
/* one Adam step (step counter t >= 1) on the stored gradients */
int tvnet_adam_step(tvnet *net, float lr, float beta1, float beta2, float eps,
                    int32_t t);

#ifdef __cplusplus
}
#endif
#endif /* TVNET_H */
