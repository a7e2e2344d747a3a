/*
 * dnb_surrogate.h -- C ABI of the learned surrogate in libdnb.so.
 *
 * The paper lists coupling the differentiable N-body code with a neural network
 * as future work (Sec. 3).  This part of the library provides what a surrogate
 * of the stream experiment (Sec. 2.2.1) needs on the GPU: the density image of
 * a simulated stream in an orbit-aligned frame, and training / inference of a
 * 4 -> 256 -> 256 -> 256 -> 2048 multilayer perceptron (exact-erf GELU after the
 * first three layers, linear output) with BF16 matrix-core products and FP32
 * accumulation.  The N-body gradient fit of dnb.h remains the reference.
 *
 * Conventions are those of dnb.h: device pointers unless marked "host",
 * asynchronous on `stream`, arguments validated before anything is enqueued,
 * status codes of dnb_status.
 *
 * Parameter vector (FP32, dnb_mlp_param_count() entries): for layer l = 0..3
 * the weight matrix W_l [in_l][out_l] row-major, then the bias b_l [out_l];
 * (in, out) = (4, 256), (256, 256), (256, 256), (256, 2048).  The BF16 copy
 * (uint16 bit patterns, round to nearest even) has the same layout; the
 * matrix products read it, the optimiser updates the FP32 master and rewrites
 * the copy.
 *
 * Rounding points (what a test must emulate): the weights, and the left operand
 * of every product -- the layer inputs in the forward pass and the output
 * gradients in the backward pass -- are BF16; products accumulate in FP32;
 * bias, GELU, its derivative, the loss and the optimiser are FP32.
 */
#ifndef DNB_SURROGATE_H
#define DNB_SURROGATE_H

#include <stdint.h>

#include "dnb.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Number of FP32 parameters of the network (659200). */
int64_t dnb_mlp_param_count(void);

/* Bytes of the per-batch workspace that dnb_mlp_forward fills and
 * dnb_mlp_backward reads (layer inputs in BF16, pre-activations in FP32,
 * gradient buffers).  Returns -1 for batch < 1. */
int64_t dnb_mlp_workspace_bytes(int64_t batch);

/* Round the FP32 parameters to their BF16 copy. */
dnb_status dnb_mlp_to_bf16(int64_t count, const float* params, uint16_t* params_bf16,
                           void* stream);

/* y [batch][2048] = MLP(x [batch][4]).  params: FP32 master (biases are read
 * from it); params_bf16: BF16 copy (weights).  workspace keeps what the backward
 * pass needs.  batch must be a multiple of 16, at most 65536. */
dnb_status dnb_mlp_forward(const float* params, const uint16_t* params_bf16, int64_t batch,
                           const float* x, float* y, void* workspace, void* stream);

/* Gradients of a loss with output cotangent dy [batch][2048] for the batch last
 * passed to dnb_mlp_forward with the same workspace: grads [param_count]
 * (overwritten; NULL skips the parameter gradients) and, if dx is not NULL, the
 * input cotangent dx [batch][4].  At least one of grads and dx is non-null. */
dnb_status dnb_mlp_backward(const uint16_t* params_bf16, int64_t batch, const float* dy,
                            void* workspace, float* grads, float* dx, void* stream);

/* Mean squared error over count values: loss (device scalar, FP64) =
 * mean((y - t)^2) and dy = 2 (y - t) / count. */
dnb_status dnb_mlp_mse(int64_t count, const float* y, const float* t, double* loss, float* dy,
                       void* stream);

/* One Adam step (t >= 1 is the step number, for the bias correction) on the
 * FP32 master parameters with moment buffers m, v; rewrites the BF16 copy. */
dnb_status dnb_mlp_adam(int64_t count, float* params, uint16_t* params_bf16, float* m, float* v,
                        const float* grads, double lr, double beta1, double beta2, double eps,
                        int64_t t, void* stream);

/* Bytes of the workspace of dnb_mlp_invert for a batch of starts. */
int64_t dnb_mlp_invert_workspace_bytes(int64_t batch);

/* Inversion of the network on a target image (the warm start of the fit):
 * iters Adam steps (beta 0.9, 0.999, eps 1e-8, step size lr) on the inputs u
 * [batch][4] (device, updated in place) of mean((MLP(u) - target)^2) over the
 * batch, with target [2048] (device) the same for every row, each step followed
 * by clamping u to [-1, 1].  The same kernels and order as the loop of
 * dnb_mlp_forward, dnb_mlp_mse, dnb_mlp_backward (dx only) and dnb_mlp_adam,
 * issued from the library with no host round trip.  workspace:
 * dnb_mlp_invert_workspace_bytes(batch) bytes (device).  batch must be a
 * multiple of 16, at most 65536. */
dnb_status dnb_mlp_invert(const float* params, const uint16_t* params_bf16, int64_t batch,
                          const float* target, float* u, int64_t iters, double lr,
                          void* workspace, void* stream);

/* Bytes of the workspace of dnb_density_grid. */
int64_t dnb_grid_workspace_bytes(void);

/* Density image grid [32][64] (FP32) of the positions pos [3][n] in the frame
 * given by the HOST array frame9 = (e1, e2, n) (three orthonormal vectors):
 * phi1 = atan2(x.e2, x.e1) in 64 bins over [-pi, pi), phi2 = asin(x.n/|x|) in 32
 * bins over [-0.1, 0.1]; integer counts, then a separable Gaussian blur of
 * sigma = 1 bin (radius 3, periodic in phi1, zero-padded in phi2), normalised to
 * sum 1 (all zeros when no particle falls inside). */
dnb_status dnb_density_grid(int64_t n, const double* pos, const double* frame9, float* grid,
                            void* workspace, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* DNB_SURROGATE_H */
