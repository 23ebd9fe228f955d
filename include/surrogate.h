/* surrogate.h -- C ABI of the learned surrogate of one convection step: the MLP of mlp.h applied to
 * the column state, with the FP64 scheme (conv.h) as the fallback where the network leaves the range
 * it was trained on.
 *
 * The paper accelerates the deep and shallow convection schemes (arXiv:1711.00289, Algorithms 1-3);
 * this surrogate is an extension that learns the tendencies of one conv_step (deep, then shallow on
 * the updated state) from pairs that conv_step itself produces.
 *
 * Feature layout for nlev = L levels (one row per column, row-major):
 *   inputs  [w_in >= 3L]:  T[0..L), q[0..L), p_mid[0..L), then zeros;
 *   targets [w_out >= 2L+1]: dTdt[0..L), dqdt[0..L), prec, then zeros, where each tendency is the
 *   sum of the deep and shallow outputs of conv_step.
 * Normalised features are (v - mean) / std per feature; inputs are fed to the network as BF16.
 * All array pointers are DEVICE pointers owned by the caller; calls enqueue work on `stream`.
 * Return 0 or a negative CONV_E* code (conv.h).
 */
#ifndef SURROGATE_H
#define SURROGATE_H

#include <stddef.h>
#include <stdint.h>

#include "conv.h"
#include "mlp.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Raw (unnormalised) FP32 feature rows: out[c][w] for columns 0..ncol-1.  w <= 256. */
int surr_pack_inputs_raw(const conv_state_t *s, int32_t nlev, int64_t ncol, int32_t w_in,
                         float *out, void *stream);
int surr_pack_targets_raw(const conv_deep_out_t *d, const conv_shallow_out_t *sh, int32_t nlev,
                          int64_t ld, int64_t ncol, int32_t w_out, float *out, void *stream);

/* Per-feature mean and standard deviation (population, two passes) of the first n_valid columns of
 * the FP32 matrix a[n][w], accumulated in FP64 in a fixed order.  A feature without spread keeps its
 * mean and gets std 1 (it normalises to 0); features j >= n_valid get mean 0 and std 1.  When `rms`
 * is not NULL it receives every feature's root-mean-square sqrt(var + mean^2).
 * `scratch`: device memory of surr_col_stats_scratch_bytes(w) bytes. */
size_t surr_col_stats_scratch_bytes(int32_t w);
int surr_col_stats(const float *a, int64_t n, int32_t w, int32_t n_valid, float *mean, float *std,
                   float *rms, void *scratch, size_t scratch_bytes, void *stream);

/* (a - mean) / std per feature: in place (FP32), or into BF16 bit patterns when out_bf16 != NULL. */
int surr_normalize(float *a, int64_t n, int32_t w, const float *mean, const float *std,
                   uint16_t *out_bf16, void *stream);

/* Network inputs straight from the state: bf16((v - mean) / std), zeros past 3L. */
int surr_pack_inputs(const conv_state_t *s, int32_t nlev, int64_t ncol, int32_t w_in,
                     const float *mean, const float *std, uint16_t *x, void *stream);

/* ------------------------------------------------------------------ inference with fallback */
typedef struct surr surr_t; /* opaque host-side handle */

/* Workspace for inference over at most max_cols columns in network batches of `chunk` rows (the
 * network's own workspace is separate: mlp_create with max_batch >= chunk). */
size_t surr_workspace_bytes(int32_t nlev, int32_t w_in, int32_t w_out, int64_t max_cols,
                            int64_t chunk);

/* A surrogate over `net` (widths[0] = w_in >= 3L, last width w_out >= 2L+1) with the scheme
 * parameters for the fallback. */
int surr_create(mlp_t *net, int32_t nlev, int32_t w_in, int32_t w_out, int64_t max_cols,
                int64_t chunk, const conv_params_t *params, void *workspace, size_t ws_bytes,
                surr_t **out);
void surr_destroy(surr_t *s);

/* Normalisation (device FP32 arrays: in_mean/in_std [w_in], out_mean/out_std [w_out]) and the
 * trusted range of the predicted precipitation: a column whose prediction lies outside
 * [prec_lo, prec_hi] (kg m-2 s-1) falls back to the scheme.  Copied at the call. */
int surr_set_norm(surr_t *s, const float *in_mean, const float *in_std, const float *out_mean,
                  const float *out_std, double prec_lo, double prec_hi, void *stream);

/* Inference path.  With enable != 0 (the default) a network of hidden width 512, an input width
 * from 64 to 512 that is a multiple of 32 and an output width of 64 runs as one fused kernel (every
 * layer of a 64-column tile on the chip, activations in LDS, no chunks); with enable == 0, and for
 * other networks, inference goes layer by layer through mlp_forward in batches of `chunk` columns.
 * Both give the same bits.  Returns 1 when the next surr_infer takes the fused kernel, 0 when not,
 * CONV_EINVAL for a NULL handle. */
int surr_set_fused(surr_t *s, int enable);

/* Total tendencies of one step for columns 0..ncol-1 (ncol <= max_cols): dTdt, dqdt [L][ld],
 * prec [ld] (FP64).  Predicted precipitation below zero is set to zero.  With fallback != 0 the
 * flagged columns are gathered, stepped by conv_step and scattered back, which waits once on the
 * host for the number of flagged columns (reported in *n_fallback when not NULL); with fallback == 0
 * nothing waits and *n_fallback is not written. */
int surr_infer(surr_t *s, const conv_state_t *state, int64_t ncol, double *dTdt, double *dqdt,
               double *prec, int fallback, int64_t *n_fallback, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SURROGATE_H */
