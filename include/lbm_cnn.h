/*
 * lbm_cnn.h - C ABI of the HIP (gfx950) kernels of the learned warm start: a small convolutional
 * network (3x3 convolutions, ReLU) that maps a porous slice, its inlet composition and current
 * density to an initial mole-fraction field for the LBM / Maxwell-Stefan solver.  The method's
 * own steady fields are the training targets; the solver then converges from the prediction.
 *
 * Conventions: tensors are NCHW float32 (or bfloat16 where named), contiguous, device memory
 * owned by the caller; every call is enqueued on `stream` (hipStream_t) and returns 0 or a
 * negative lbm_ms_status code (-1 invalid argument, -4 HIP error).  Convolutions use zero
 * padding of one pixel, so output and input have the same H x W.  Channel counts: C_in <= 32,
 * C_out <= 32.  Weights are [C_out][C_in][3][3], biases [C_out].
 */
#ifndef LBM_CNN_H
#define LBM_CNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* out = act(conv3x3(in * gate, w) + b), act = ReLU if relu != 0.  gate (may be NULL) multiplies
 * each input value by (gate > 0) with gate shaped like in (used to apply a ReLU derivative). */
int lbm_cnn_conv_forward(const float* in, const float* gate, int B, int C_in, int H, int W,
                         const float* w, const float* b, int C_out, int relu, float* out,
                         void* stream);

/* Same convolution with bfloat16 activations and weights (raw uint16 bit patterns), FP32
 * accumulation; b stays float32. */
int lbm_cnn_conv_forward_bf16(const uint16_t* in, int B, int C_in, int H, int W,
                              const uint16_t* w, const float* b, int C_out, int relu,
                              uint16_t* out, void* stream);

/* Gradient of the input of a convolution layer: grad_in = conv3x3(grad_out * (act > 0), w^T)
 * with w^T the transposed, flipped kernel (act = the layer's output if it has a ReLU, else NULL).
 * wt_scratch: C_in*C_out*9 floats. */
int lbm_cnn_conv_backward_data(const float* grad_out, const float* act, int B, int C_out, int H,
                               int W, const float* w, int C_in, float* grad_in, float* wt_scratch,
                               void* stream);

/* Gradients of weights and bias: grad_w = sum over images and pixels of (grad_out * (act > 0)) x
 * im2col(in), grad_b = sum of (grad_out * (act > 0)).  Deterministic: per-workgroup partial sums
 * in partial (at least lbm_cnn_backward_weight_scratch floats), then a fixed-order sum. */
size_t lbm_cnn_backward_weight_scratch(int B, int C_in, int C_out, int H, int W);
int lbm_cnn_conv_backward_weight(const float* in, const float* grad_out, const float* act, int B,
                                 int C_in, int C_out, int H, int W, float* grad_w, float* grad_b,
                                 float* partial, void* stream);

/* Masked mean squared error over fluid pixels: loss = sum m (p - t)^2 / (C sum m), with m =
 * fluid[B][H][W] (1 fluid, 0 solid); grad = d loss / d pred.  loss_out: one float64 on the
 * device; partial: 2 * 1024 + 1 float64 scratch. */
int lbm_cnn_masked_mse(const float* pred, const float* target, const float* fluid, int B, int C,
                       int H, int W, float* grad, double* loss_out, double* partial,
                       void* stream);

/* lbm_cnn_masked_mse without the partial argument, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, outputs and results as lbm_cnn_masked_mse (bitwise: the same kernels in the
 * same order).  Its scratch is a fixed library array of 2 * 1024 + 1 float64 (16 KiB) per
 * device, held until the process ends; the call allocates nothing.  The partial-sum count is
 * set by the grid, at most 1024 workgroups, so every size fits: -8 (LBM_MS_E_NOMEM) would mean
 * the fixed scratch is too small; -1 for null pointers or non-positive sizes, -4 for a HIP
 * error.  All calls on one device share that device's scratch: calls that overlap in time on
 * one device (different streams or host threads) race and must be serialized by the caller. */
int lbm_cnn_masked_mse_noalloc(const float* pred, const float* target, const float* fluid, int B,
                               int C, int H, int W, float* grad, double* loss_out, void* stream);

/* Adam update of n parameters (step t >= 1). */
int lbm_cnn_adam(float* param, const float* grad, float* m, float* v, int64_t n, float lr,
                 float beta1, float beta2, float eps, int t, void* stream);

/* float32 -> bfloat16 (round to nearest even) bit patterns. */
int lbm_cnn_to_bf16(const float* in, uint16_t* out, int64_t n, void* stream);
int lbm_cnn_from_bf16(const uint16_t* in, float* out, int64_t n, void* stream);

/* Input features [B][8][H][W] and the baseline field the prediction corrects.  With phi(x) the
 * fluid fraction of column x (at least 1/H) and prof[B][2][W] the paper's one-dimensional profile
 * (X_1, X_2 along x), the porosity-weighted profile is P_s(x) = X_in,s + sum over x' <= x of
 * (prof_s(x') - prof_s(x' - 1)) / phi(x'), with prof_s(-1) = X_in,s.  Channels: fluid indicator,
 * X_in,1, X_in,2, j / 2 (j in A/cm^2), x / (W - 1), (P_1 - X_in,1) / 0.01, (P_2 - X_in,2) / 0.01,
 * phi(x).  base[B][2][W] (float64) receives P.  solid: [B][H][W] uint8; X_in: [B][3];
 * W <= 2048, B <= 65535. */
int lbm_cnn_features(const uint8_t* solid, const double* X_in, const double* j_A_cm2,
                     const double* prof, int B, int H, int W, float* feat, double* base,
                     void* stream);

/* Initial field from a prediction pred[B][2][H][W] and a baseline prof[B][2][W] (the base output
 * of lbm_cnn_features): X_s = max(prof_s + scale * pred_s, x_min)
 * (s = 1, 2); where X_3 = 1 - X_1 - X_2 would fall below x_min, the parts of X_1 and X_2 above
 * x_min are scaled so that X_3 = x_min.  Written as X[B][3][H][W] float64 (the layout
 * lbm_ms_init / lbm_ms_batch_init take); 0 < x_min < 1/3. */
int lbm_cnn_assemble(const float* pred, const double* prof, int B, int H, int W, float scale,
                     double x_min, double* X, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_CNN_H */
