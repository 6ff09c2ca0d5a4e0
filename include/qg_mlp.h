/*
 * qg_mlp.h -- C ABI of the learned warm start: a multilayer perceptron that
 * maps a day's bus loads and reserve requirements to an initial point of the
 * solver (voltages, angles and dispatch), trained on solutions the solver
 * itself produced.  The paper names learning as future work (Section V) and
 * notes that the starting point matters (Section III); the network is
 *
 *   h_0 = x,  h_i = gelu(h_{i-1} W_i + b_i)  (i = 1..depth),
 *   y   = h_depth W_out + b_out,
 *
 * with gelu(z) = z Phi(z) (Phi the standard normal distribution function),
 * trained on the mean squared error with Adam.
 *
 * Conventions
 * -----------
 * - Parameters are one FP32 vector: W_1 [d_in][width], b_1 [width], then
 *   W_i [width][width], b_i for i = 2..depth, then W_out [width][d_out],
 *   b_out [d_out]; matrices row-major.  Each array starts at a multiple of
 *   64 floats; qg_mlp_layout gives the offsets.
 * - Batches are row-major [batch][features] FP32.
 * - Device buffers are caller-owned, 256-byte aligned; the workspace is
 *   sized by qg_mlp_sizes for the largest batch that will be used.
 * - Calls only enqueue work on the stream (no synchronisation), except where
 *   noted.  Errors return a qg_status (see qg.h) with qg_last_error() text.
 */
#ifndef QG_MLP_H
#define QG_MLP_H

#include <stddef.h>
#include <stdint.h>

#include "qg.h"

#ifdef __cplusplus
extern "C" {
#endif

#define QG_MLP_MAX_DEPTH 8

typedef struct {
  int32_t d_in, width, depth, d_out;  /* depth = number of hidden layers (1..8) */
} qg_mlp_desc;

typedef struct {
  int64_t n_params;                    /* floats in the parameter vector */
  int64_t w_off[QG_MLP_MAX_DEPTH + 1]; /* offsets of W_1..W_depth, W_out */
  int64_t b_off[QG_MLP_MAX_DEPTH + 1]; /* offsets of b_1..b_depth, b_out */
} qg_mlp_layout;

/* Parameter layout and workspace bytes for batches up to max_batch.
 * Host only.  Errors: ARG. */
qg_status qg_mlp_sizes(const qg_mlp_desc* desc, int32_t max_batch, qg_mlp_layout* layout,
                       size_t* workspace_bytes);

/* y [batch][d_out] = network(x [batch][d_in]) in FP32.  Errors: ARG, DEVICE. */
qg_status qg_mlp_forward(const qg_mlp_desc* desc, const float* d_params, const float* d_x,
                         int32_t batch, float* d_y, void* d_workspace, void* stream);

/* Mean squared error over the batch, L = sum (y - t)^2 / (batch d_out), and
 * its gradient with respect to every parameter (d_grad, n_params floats).
 * *d_loss receives L (device float).  Errors: ARG, DEVICE. */
qg_status qg_mlp_grad(const qg_mlp_desc* desc, const float* d_params, const float* d_x,
                      const float* d_t, int32_t batch, float* d_grad, float* d_loss,
                      void* d_workspace, void* stream);

/* One training step: qg_mlp_grad, then Adam on the parameters (moments m, v,
 * 1-based step iter, learning rate lr, beta1 0.9, beta2 0.999, eps 1e-8).
 * d_grad is scratch of n_params floats.  Errors: ARG, DEVICE. */
qg_status qg_mlp_train_step(const qg_mlp_desc* desc, float* d_params, float* d_m, float* d_v,
                            float* d_grad, const float* d_x, const float* d_t, int32_t batch,
                            int64_t iter, float lr, float* d_loss, void* d_workspace,
                            void* stream);

/* BF16 inference: d_params16 (n_params bf16, as uint16) from the FP32
 * parameters (round to nearest even), then y = network(x) with BF16 operands
 * and FP32 accumulation (activations rounded to BF16 between layers).
 * Errors: ARG, DEVICE. */
qg_status qg_mlp_to_bf16(const qg_mlp_desc* desc, const float* d_params, uint16_t* d_params16,
                         void* stream);
qg_status qg_mlp_forward_bf16(const qg_mlp_desc* desc, const uint16_t* d_params16,
                              const float* d_x, int32_t batch, float* d_y, void* d_workspace,
                              void* stream);

#ifdef __cplusplus
}
#endif
#endif /* QG_MLP_H */
