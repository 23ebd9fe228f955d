/* mlp.h -- C ABI of the learned surrogate's network: a fully connected MLP with GELU hidden layers,
 * BF16 operands and FP32 accumulation on gfx950 matrix cores (MFMA), trained by hand-written
 * forward, backward, loss and Adam kernels.
 *
 * The paper accelerates the convection schemes themselves (arXiv:1711.00289, Algorithms 2-3); this
 * network is an extension trained on (sounding -> tendency) pairs that those schemes generate, with
 * the FP64 schemes kept as the fallback and as the reference for its error.
 *
 * Conventions.
 *   widths[0..n_layers] are the layer widths (input first); each is a multiple of 32, at most 4096.
 *   Layer l maps width widths[l] to widths[l+1] with weight W_l [widths[l+1]][widths[l]] (row-major,
 *   FP32 master copy) and bias b_l [widths[l+1]]; GELU (the erf form) follows every layer but the
 *   last.  Activations are BF16 (stored as uint16_t bit patterns, round-to-nearest-even); the
 *   network output is FP32.  All array pointers are DEVICE pointers; the caller owns them and the
 *   workspace.  Calls only enqueue work on `stream` (no allocation, no host synchronisation).
 *   Return 0 (MLP_OK) or a negative error code; argument errors (MLP_EINVAL) make no HIP call.
 */
#ifndef MLP_H
#define MLP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MLP_OK 0
#define MLP_EINVAL -1
#define MLP_EHIP -3
#define MLP_MAX_LAYERS 8

typedef struct mlp mlp_t; /* opaque host-side handle */

/* Workspace bytes for a network of these widths trained or run on batches of at most max_batch
 * rows (0 on bad arguments). */
size_t mlp_workspace_bytes(const int32_t *widths, int n_layers, int64_t max_batch);

/* Handle over a 256-byte aligned workspace.  Weights are undefined until mlp_set_params. */
int mlp_create(const int32_t *widths, int n_layers, int64_t max_batch, void *workspace,
               size_t ws_bytes, mlp_t **out);

/* The same with a separate, smaller limit for training: inference forwards (keep = 0) and
 * mlp_mse take up to max_batch rows, training forwards (keep != 0), mlp_backward and
 * mlp_train_step up to max_train_batch (1 <= max_train_batch <= max_batch; a larger training
 * batch is rejected with MLP_EINVAL).  Only the activations scale with max_batch; the
 * pre-activations, transposed copies and hidden gradients that training keeps scale with
 * max_train_batch, so a network that infers in large chunks and trains in small batches needs a
 * fraction of mlp_workspace_bytes(widths, n_layers, max_batch).  mlp_create(.., b, ..) is
 * mlp_create_ex(.., b, b, ..). */
size_t mlp_workspace_bytes_ex(const int32_t *widths, int n_layers, int64_t max_batch,
                              int64_t max_train_batch);
int mlp_create_ex(const int32_t *widths, int n_layers, int64_t max_batch, int64_t max_train_batch,
                  void *workspace, size_t ws_bytes, mlp_t **out);
void mlp_destroy(mlp_t *m);

/* Flat FP32 parameter vector layout: for l = 0..n_layers-1, W_l then b_l.  Its length: */
int64_t mlp_param_count(const mlp_t *m);

/* Copies a device FP32 parameter vector into the master weights (and their BF16 copies) and
 * clears the Adam moments and step count. */
int mlp_set_params(mlp_t *m, const float *params, void *stream);
/* Copies the master weights out (device FP32 vector) / the last backward's gradients. */
int mlp_get_params(const mlp_t *m, float *params, void *stream);
int mlp_get_grads(const mlp_t *m, float *grads, void *stream);

/* y[batch][widths[n]] = network(x[batch][widths[0]]).  `keep` != 0 stores the pre-activations and
 * activations for mlp_backward (training; batch <= max_train_batch); 0 runs the lighter inference
 * path (batch <= max_batch). */
int mlp_forward(mlp_t *m, const uint16_t *x, float *y, int64_t batch, int keep, void *stream);

/* Mean squared error over the first n_valid outputs:
 * loss = sum_{b, j < n_valid} (y - t)^2 / (batch * n_valid), written to loss[0] (device FP32), and
 * the output gradient 2 (y - t) / (batch * n_valid) (zero for j >= n_valid) kept for mlp_backward.
 * Sums are taken in a fixed order. */
int mlp_mse(mlp_t *m, const float *y, const float *target, int64_t batch, int n_valid, float *loss,
            void *stream);

/* Gradients of the loss with respect to every weight and bias (FP32, fixed summation order), from
 * the activations of the last mlp_forward with keep != 0 and the gradient of the last mlp_mse. */
int mlp_backward(mlp_t *m, int64_t batch, void *stream);

/* One Adam step (Kingma & Ba) on the master weights with the last gradients: step count t = t+1,
 * m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2, w -= lr (m/(1-b1^t)) / (sqrt(v/(1-b2^t)) + eps);
 * then refreshes the BF16 copies. */
int mlp_adam_step(mlp_t *m, float lr, float beta1, float beta2, float eps, void *stream);

/* One training step in one call: mlp_forward (keep), mlp_mse, mlp_backward and mlp_adam_step on
 * the same stream, with the same results; y [batch][widths[n]] receives the network output and
 * loss[0] the loss.  Returns the first error. */
int mlp_train_step(mlp_t *m, const uint16_t *x, const float *target, int64_t batch, int n_valid,
                   float lr, float beta1, float beta2, float eps, float *y, float *loss,
                   void *stream);

/* The layer kernel on its own, for tests: acc[M][N] = A[M][K] . B[N][K]^T with BF16 operands
 * (row-major, K contiguous, K a multiple of 8, lda/ldb multiples of 8) and FP32 accumulation;
 * mode 0 writes acc + bias as FP32 to c; mode 1 writes bf16(gelu(acc + bias)) to c (uint16_t) and,
 * when z is not NULL, acc + bias as FP32 to z (same leading dimension ldc).  bias may be NULL. */
int mlp_gemm_nt(const uint16_t *a, int64_t lda, const uint16_t *b, int64_t ldb, const float *bias,
                int64_t M, int32_t N, int32_t K, int mode, void *c, int64_t ldc, float *z,
                void *stream);

const char *mlp_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* MLP_H */
