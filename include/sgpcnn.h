/* Learned warm start for SGP: a small convolutional network that maps an
 * observed image to a start image for the iteration.
 *
 * SGP accepts any non-negative start image (Sect. 3.1 of Prato et al. 2012,
 * where the flat image and the data are the usual choices); the network
 * supplies a better one, and the solver still takes the flat start whenever
 * the network's start has the larger KL divergence (SGP_INIT_WARM in
 * sgpdeconv.h).  The network is not part of the paper.
 *
 * Architecture (all convolutions 5x5 cross-correlations with periodic
 * padding, convolution weights used rounded to bfloat16, biases in FP32,
 * FP32 accumulation):
 *   s  = max(mean(g - b), 1e-3),  x = (g - b) / s
 *   a1 = relu(conv 1->16 (x)),  a2 = relu(conv 16->16 (a1)),
 *   a3 = relu(conv 16->16 (a2)), o = conv 16->1 (a3)
 *   f0 = s * softplus(o)
 * Parameter vector (float32, sgp_cnn_num_params() = 13649 entries):
 *   W1[16][1][5][5], b1[16], W2[16][16][5][5], b2[16], W3[16][16][5][5],
 *   b3[16], W4[1][16][5][5], b4[1], weights indexed [cout][cin][ky][kx];
 *   conv: out[co](y,x) = b[co] + sum W[co][ci][ky][kx] in[ci](y+ky-2, x+kx-2).
 * Training loss on a batch: mean over all pixels of
 *   (sqrt(f0/s + 1e-3) - sqrt(f_target/s + 1e-3))^2,
 * minimised by Adam (beta1 0.9, beta2 0.999, eps 1e-8) on float32 master
 * weights; every step re-rounds the bfloat16 copy the kernels use.
 *
 * Conventions: images are float32 [ny][nx] row-major in device memory,
 * passed as host arrays of n device pointers; ny and nx must be multiples of
 * 16.  b: host array of n constant backgrounds.  The handle owns its device
 * memory (weights, Adam moments, activations sized for the largest batch
 * seen) until sgp_cnn_destroy.  Calls on one handle must not overlap.
 * Errors: SGP_E_INVALID_ARG for NULL pointers, bad sizes or a wrong
 * parameter count; SGP_E_HIP for a failed runtime call; SGP_E_NO_DEVICE.
 * sgp_last_error() gives the message. */
#ifndef SGPCNN_H
#define SGPCNN_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sgp_cnn sgp_cnn;

/* Number of float32 parameters (13649). */
int sgp_cnn_num_params(void);

/* New network on the current device with the given master weights
 * (host array of sgp_cnn_num_params() floats); Adam moments start at 0. */
int sgp_cnn_create(const float* host_params, size_t nparams, sgp_cnn** out);

/* Copies the float32 master weights to host memory. */
int sgp_cnn_get_params(sgp_cnn* h, float* host_out, size_t nparams);

/* f0[i] = network start image of g[i] (all n images ny x nx).  Runs on
 * hip_stream (NULL: the default stream) and returns after it finishes.
 * Inference stores the hidden activations a1..a3 as bfloat16 (nearest, ties
 * to even, after the ReLU) and runs the three layers with 16 input channels
 * on the bf16 matrix cores (FP32 accumulation); training (below) keeps the
 * activations in float32. */
int sgp_cnn_infer(sgp_cnn* h, int n, const float* const* g, const float* b, int ny, int nx, float* const* f0,
                  void* hip_stream);

/* Batch loss and its gradient with respect to the bfloat16-rounded weights;
 * loss (optional) receives the mean, host_grad (optional) the gradient in
 * the parameter layout.  The gradient also stays on the device for
 * sgp_cnn_adam_step. */
int sgp_cnn_loss_grad(sgp_cnn* h, int n, const float* const* g, const float* b, const float* const* f_target,
                      int ny, int nx, double* loss, float* host_grad, void* hip_stream);

/* One Adam step (step count kept by the handle) with the last gradient. */
int sgp_cnn_adam_step(sgp_cnn* h, float lr, void* hip_stream);

/* sgp_cnn_loss_grad followed by sgp_cnn_adam_step. */
int sgp_cnn_train_step(sgp_cnn* h, int n, const float* const* g, const float* b, const float* const* f_target,
                       int ny, int nx, float lr, double* loss, void* hip_stream);

int sgp_cnn_destroy(sgp_cnn* h);

#ifdef __cplusplus
}
#endif
#endif /* SGPCNN_H */
