/* hipipm_mlp — the learned warm start's network on the GPU (C ABI, part of libhipipm.so).
 *
 * The network maps an instance's parameters (d_in values, e.g. start state, target and obstacle
 * spheres of the point-to-point NMPC) to a primal trajectory and equality multipliers (d_out
 * values): d_in -> hidden -> hidden -> hidden -> d_out, GELU after each hidden layer.  It is the
 * warm-start addition the method is extended with: trained on solutions the solver itself
 * produces, judged by the interior-point method (a warm point it cannot use falls back to the
 * cold start).  Products run on the matrix cores with BF16 weights and activations and FP32
 * accumulation; biases, the loss, gradients and the Adam state are FP32.
 *
 * Buffers (all device memory, owned by the caller):
 *   model   FP32 [model_len]: per layer l = 1..4 the weight W_l [out][in] (row major) and the bias
 *           b_l [out]; then the input normalisation in_mu[d_in], in_sd[d_in] and the output
 *           normalisation out_mu[d_out], out_sd[d_out] (x_n = (x - mu) / sd).
 *   w_bf16  BF16 (uint16) [n_weights]: the weights W_1..W_4 in the same order, rounded to nearest
 *           even; refreshed by hipipm_mlp_weights_bf16 and hipipm_mlp_adam.
 *   act     activation workspace of hipipm_mlp_sizes(..., batch, act_bytes) bytes, 16-byte aligned.
 *   grad    FP32 [n_params] in the layout of the model's parameter part.
 * inputs / targets are FP64 row major [rows][d_in] / [rows][d_out]; the loss is the mean squared
 * error of the normalised outputs.
 *
 * Every call returns 0, -1 for an invalid argument, -2 for a HIP launch error; launches are
 * asynchronous on `stream` (NULL: the default stream). */
#ifndef HIPIPM_MLP_H
#define HIPIPM_MLP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Sizes for the given network and batch: model buffer length (floats), trainable parameters,
 * weights, activation workspace bytes.  Any output pointer may be NULL. */
int hipipm_mlp_sizes(int32_t d_in, int32_t hidden, int32_t d_out, int32_t batch, int64_t* model_len,
                     int64_t* n_params, int64_t* n_weights, int64_t* act_bytes);

/* w_bf16 <- BF16(model weights). */
int hipipm_mlp_weights_bf16(int32_t d_in, int32_t hidden, int32_t d_out, const float* model, uint16_t* w_bf16,
                            void* stream);

/* Column means and standard deviations (floored at 1e-6) of `rows` training inputs and targets
 * into the model's normalisation part. */
int hipipm_mlp_normalizer(int32_t d_in, int32_t hidden, int32_t d_out, int64_t rows, const double* inputs,
                          const double* targets, float* model, void* stream);

/* outputs[batch][d_out] (FP64, de-normalised) = network(inputs[batch][d_in]). */
int hipipm_mlp_forward(int32_t d_in, int32_t hidden, int32_t d_out, const float* model, const uint16_t* w_bf16,
                       const double* inputs, double* outputs, int32_t batch, void* act, void* stream);

/* Gradient of the loss over the rows `rows[0..batch)` of inputs/targets (rows NULL: the first
 * `batch` rows) into grad; loss_parts (nullable, FP32 [ceil(batch d_out / 256)]) receives partial
 * sums of the squared normalised errors (their sum / (batch d_out) is the loss). */
int hipipm_mlp_backward(int32_t d_in, int32_t hidden, int32_t d_out, const float* model, const uint16_t* w_bf16,
                        const double* inputs, const double* targets, const int32_t* rows, int32_t batch,
                        void* act, float* grad, float* loss_parts, void* stream);

/* One Adam step (step >= 1 is the update count, for the bias corrections) on the model's
 * parameters with grad, then the BF16 weights. */
int hipipm_mlp_adam(int32_t d_in, int32_t hidden, int32_t d_out, float* model, uint16_t* w_bf16, const float* grad,
                    float* adam_m, float* adam_v, int32_t step, float lr, float beta1, float beta2, float eps,
                    void* stream);

#ifdef __cplusplus
}
#endif

#endif /* HIPIPM_MLP_H */
