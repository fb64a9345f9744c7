/* Learned trace surrogate: a small network that maps a medium c^2, sampled on a 16^3 grid of
 * the unit cube, to the receiver traces a BBWADG run produces in it, trained on such runs
 * (data from bbwadg_misfit_gradient's forward pass). The solver stays the reference: it makes
 * the training data and measures the surrogate's error on held-out media, and a caller falls back
 * to it where that error is too large.
 *
 * Network (about 2 million parameters): three 3x3x3 convolutions with stride 2 and padding 1
 * (1 -> 16 -> 32 -> 64 channels, 16^3 -> 8^3 -> 4^3 -> 2^3, ReLU), then fully connected layers
 * 512 -> 256 -> 256 -> 64 (ReLU) -> nout (linear). Every layer is one GEMM on the BF16 matrix
 * cores with FP32 accumulation (convolutions through im2col); master weights, gradients and the
 * Adam state are FP32. Loss: mean squared error over the batch's outputs.
 *
 * Layouts: input x [B][16][16][16] FP32, z-major (x index fastest); output y [B][nout] FP32.
 * Device pointers are the caller's; the context owns its parameters and work buffers (sized for
 * max_batch at create). Calls run on `stream` and return 0 or a negative BBWADG_E* code with
 * bbwadg_last_error() set. Not thread-safe per context. */
#ifndef BBWADG_SURROGATE_H
#define BBWADG_SURROGATE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bbwadg_sur bbwadg_sur;

/* Create a surrogate for nout outputs and batches up to max_batch (1..4096). grid must be 16.
 * Weights are drawn uniform(-a, a) from a counter-based generator (splitmix64 of seed and the
 * parameter index), a = sqrt(6 / fan_in) for ReLU layers and sqrt(3 / fan_in) for the output
 * layer; biases are zero. */
int bbwadg_sur_create(int32_t grid, int32_t nout, int32_t max_batch, uint64_t seed, bbwadg_sur** out);

int bbwadg_sur_destroy(bbwadg_sur* s);

/* Total number of parameters (FP32 values in the flat parameter vector). */
int64_t bbwadg_sur_num_params(const bbwadg_sur* s);

/* Layer l (0..6) of the flat parameter vector, int32[8]: is_conv, fan-in channels (conv) or
 * features (dense), output channels or features, K (27 Cin for a convolution, else fan-in),
 * Kp (K padded to a multiple of 16 for a convolution, else K), relu, weight offset, bias
 * offset. Weights are W[Kp][N] row-major; a convolution's row ((kz*3 + ky)*3 + kx)*Cin + c
 * multiplies input voxel (2o + k - 1) of channel c; rows >= K are zero. EINVAL for a bad l. */
int bbwadg_sur_layout(const bbwadg_sur* s, int32_t layer, int32_t* info);

/* Copy the FP32 parameters to or from host memory [num_params]; set also refreshes the BF16
 * copies and clears the Adam state. */
int bbwadg_sur_get_params(const bbwadg_sur* s, float* host);
int bbwadg_sur_set_params(bbwadg_sur* s, const float* host);

/* y = f(x) for B inputs (1 <= B <= max_batch). */
int bbwadg_sur_forward(bbwadg_sur* s, const float* x, int32_t B, float* y, void* stream);

/* Loss L = mean((f(x) - t)^2) over B * nout values (*loss, host) and its gradient with respect
 * to the parameters, kept in the context; copied to host grad_host [num_params] if not NULL.
 * Synchronises `stream`. */
int bbwadg_sur_loss_grad(bbwadg_sur* s, const float* x, const float* t, int32_t B, double* loss, float* grad_host,
                         void* stream);

/* The loss of bbwadg_sur_loss_grad (*loss, host) and its gradient with respect to the input,
 * dL/dx into dx (device FP32 [B][16][16][16], the layout of x): the network as a
 * differentiable stand-in for the forward solve (the parameter gradient is formed as well and
 * kept in the context). Synchronises `stream`. */
int bbwadg_sur_input_grad(bbwadg_sur* s, const float* x, const float* t, int32_t B, double* loss, float* dx,
                          void* stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on the gradient of
 * bbwadg_sur_loss_grad at (x, t); *loss gets the loss before the step. */
int bbwadg_sur_train_step(bbwadg_sur* s, const float* x, const float* t, int32_t B, float lr, double* loss, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* BBWADG_SURROGATE_H */
