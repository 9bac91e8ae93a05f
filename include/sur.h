/*
 * sur.h -- C ABI of libsur.so: the learned surrogate that advances the
 * macroscopic fields (phi, C, theta, ux, uy) of the diffuse-interface lattice
 * Boltzmann solver by K main steps in one jump, on MI355X (gfx950).
 *
 * Network: 4-level U-Net, 32/64/128/256 channels, two 3x3 convolutions with
 * leaky ReLU (slope 0.1) per level, 2x2 average pooling down, nearest 2x
 * upsampling with skip concatenation up, 1x1 head; it predicts the
 * normalised residual x(t+K) - x(t).  Weights and activations are bfloat16,
 * products accumulate in FP32 on the matrix cores (v_mfma_f32_16x16x32_bf16),
 * master weights, gradients and Adam moments are FP32.
 *
 * Memory: the caller owns the parameter block (sur_param_bytes) and the
 * workspace (sur_workspace_bytes for batch B and H x W; H and W multiples of
 * 8) and the HIP stream.  Field arrays are planar [B][5][H][W], fields in the
 * order (phi, C, theta, ux, uy).  Calls return 0 or a negative code
 * (-1 invalid argument, -2 buffer too small, -3 HIP error);
 * sur_last_error() describes the last failure.
 *
 * Parameter order (FP32 master copy): for each layer of the sequence
 * enc0a enc0b enc1a enc1b enc2a enc2b enc3a enc3b dec2a dec2b dec1a dec1b
 * dec0a dec0b: W[3][3][Cout][Cin_p] then b[Cout], with Cin_p = Cin rounded
 * up to 32 (only enc0a, 5 -> 32, is padded; the padding stays zero); then
 * head W[5][32], b[5].
 */
#ifndef SUR_H
#define SUR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sur_net* sur_handle;

size_t sur_param_count(void);                 /* FP32 parameters incl. padding */
size_t sur_param_bytes(void);                 /* master, grad, m, v, bf16, flipped bf16 */
size_t sur_workspace_bytes(int B, int H, int W);

int sur_create(int B, int H, int W, void* params_dev, size_t param_bytes, void* work_dev,
               size_t work_bytes, void* hip_stream, sur_handle* out);
int sur_destroy(sur_handle h);

/* Parameters as FP32 host arrays of sur_param_count() values (order above);
 * set also refreshes the bf16 copies and zeroes the Adam moments. */
int sur_set_params(sur_handle h, const float* host);
int sur_get_params(sur_handle h, float* host);
int sur_get_grads(sur_handle h, float* host);

/* Normalisation: network input channel c = (field_c - mean[c]) / std[c];
 * the head predicts (x(t+K) - x(t))_c / rstd[c]. */
int sur_set_normalization(sur_handle h, const float* mean5, const float* std5, const float* rstd5);

/* Per-channel weights w of the training loss (default 1 each): loss = sum
 * over samples, pixels and channels c of w_c (prediction - target)^2, divided
 * by b H W 5.  Weights finite and >= 0, at least one positive. */
int sur_set_loss_weights(sur_handle h, const float* w5);

/* Forward pass for b <= B samples.  x: device FP32 [b][5][H][W].  out (may
 * be NULL): device FP64 [b][5][H][W] receiving x + rstd * prediction. */
int sur_forward(sur_handle h, int b, const float* x, double* out);

/* Forward + backward on (x, y = fields K steps later), both device FP32
 * [b][5][H][W]; gradients accumulate from zero; *loss (host) receives the
 * (weighted, see sur_set_loss_weights) mean squared error of the normalised
 * residual.  Synchronises. */
int sur_gradients(sur_handle h, int b, const float* x, const float* y, float* loss);

/* sur_gradients followed by one Adam step (beta1 0.9, beta2 0.999,
 * eps 1e-8) with learning rate lr; step counter kept by the handle. */
int sur_train_step(sur_handle h, int b, const float* x, const float* y, float lr, float* loss);

/* A tensor of conv layer k (0..13, in the parameter order above) as the last
 * forward pass (which 0: the layer's input, 1: its output after the leaky
 * ReLU) or the last sur_gradients call (which 2: the gradient of the layer's
 * pre-activation output, i.e. the dY its weight gradient consumed) left it in
 * the workspace, for checks of single layers against a reference.  host: FP32
 * [B][H >> level][W >> level][C] (NHWC, the workspace's batch B; C = Cin
 * rounded up to 32 for which 0, Cout otherwise), the bf16 values exactly.
 * Synchronises. */
int sur_get_layer_tensor(sur_handle h, int k, int which, float* host);

/* One 16x16x32 bf16 matrix-core product D = A B on the device (A 16x32 and
 * B 32x16 row-major FP32 host arrays rounded to bf16, D 16x16): checks the
 * operand lane layout the convolution kernels assume. */
int sur_mfma_check(const float* A, const float* B, float* D);

/* One 3x3 convolution kernel on host data rounded to bf16, for checks:
 * op 0: Y = conv(X, Wt) (zero bias, no activation), out [B][H][W][Cout];
 * op 1: input gradient of op 0 for dY [B][H][W][Cout], out [B][H][W][Cin];
 * op 2: weight gradient sum_pixels dY X_shift, out [3][3][Cout][Cin] (FP32).
 * X [B][H][W][Cin], Wt [3][3][Cout][Cin]; Cin and Cout multiples of 32.
 * Uses temporary device allocations; synchronous. */
int sur_conv_check(int op, int B, int H, int W, int Cin, int Cout, const float* X, const float* Wt,
                   const float* dY, float* out);

const char* sur_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
