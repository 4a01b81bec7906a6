/*
 * spdba_proposer.h -- C ABI of the learned activation proposer kernels (gfx950).
 *
 * The proposer predicts, per k-space block, whether the block will be active
 * within the next K steps, so that the exact indicator can skip the blocks
 * predicted inactive (they are passed to spdba_set_skip).  The exact indicator
 * audits every block at the steps closing each K-step window, and the caller
 * falls back to the plain rule after any miss.  The paper has no such
 * component; it plugs into the paper's state-preparation stage (Methods,
 * "Spectral dynamic block activation": the activity measure compared with a
 * threshold) and into periodic full activation (Supplementary S1.3).
 *
 * Network: 8 -> 64 -> 64 -> 1, ReLU, ReLU, sigmoid.  Weights are bf16 for the
 * forward pass with an FP32 master copy for training; every matrix product
 * runs on bf16 MFMA with FP32 accumulation (inputs of each layer rounded to
 * bf16, round-to-nearest-even).
 *
 * Parameter vector (FP32 master and bf16 shadow share the layout, row-major
 * [in][out]): W1 8x64 @0, b1 64 @512, W2 64x64 @576, b2 64 @4672, W3 64 @4736,
 * b3 @4800; SPDBA_MLP_NPARAM = 4801 values.
 *
 * All pointers are HIP device pointers unless stated; stream is a hipStream_t
 * (NULL = default).  Calls are asynchronous.  Errors: SPDBA_EINVAL for bad
 * sizes or NULL required pointers, SPDBA_EDEVICE for launch failures.
 */
#ifndef SPDBA_PROPOSER_H
#define SPDBA_PROPOSER_H

#include <stddef.h>
#include <stdint.h>

#include "spdba.h"

#ifdef __cplusplus
extern "C" {
#endif

#define SPDBA_MLP_NIN 8
#define SPDBA_MLP_NHID 64
#define SPDBA_MLP_NPARAM 4801

/* Forward pass of n samples.  x: n x 8 FP32 features (row-major).  w_bf16:
 * SPDBA_MLP_NPARAM bf16 values (raw 16-bit patterns).  Outputs (NULL skips):
 * prob n FP32 sigmoid outputs, logit n FP32, h1 / h2 n x 64 FP32 post-ReLU
 * activations (kept for the backward pass). */
spdba_status spdba_mlp_forward(const float *x, int64_t n, const uint16_t *w_bf16, float *prob,
                               float *logit, float *h1, float *h2, void *stream);

/* Scratch bytes the backward pass needs for n samples. */
size_t spdba_mlp_backward_scratch(int64_t n);

/* Backward pass: given dlogit (n FP32, dL/dlogit of every sample), the forward
 * activations x, h1, h2 and the FP32 master parameters w (the products use
 * their bf16 rounding, i.e. the forward pass's shadow), writes the gradient of
 * every parameter (SPDBA_MLP_NPARAM FP32, same layout) into grad.  The matrix
 * products dW = act^T delta and delta W^T run on bf16 MFMA (operands rounded
 * to bf16, FP32 accumulation); bias gradients are FP32 column sums.  scratch
 * must hold spdba_mlp_backward_scratch(n) bytes.  Deterministic: fixed-order
 * sums. */
spdba_status spdba_mlp_backward(const float *x, const float *h1, const float *h2,
                                const float *dlogit, int64_t n, const float *w, float *grad,
                                void *scratch, void *stream);

/* Weighted binary cross-entropy on logits, averaged over n:
 * L = -mean[pos_weight y log p + (1 - y) log(1 - p)]; writes dlogit (n) and,
 * if loss != NULL, the FP64 loss to loss[0] (fixed-order reduction).  scratch
 * (device, at least 8 KiB) holds the per-workgroup partial sums. */
spdba_status spdba_mlp_bce(const float *logit, const float *y, int64_t n, float pos_weight,
                           float *dlogit, double *loss, void *scratch, void *stream);

/* One Adam step (step number t >= 1) on the FP32 master w with moments m, v
 * and gradient g (nparam values each); refreshes the bf16 shadow w_bf16. */
spdba_status spdba_mlp_adam(float *w, float *m, float *v, const float *g, uint16_t *w_bf16,
                            int64_t nparam, float lr, float beta1, float beta2, float eps,
                            int64_t t, void *stream);

/* Round an FP32 parameter vector to the bf16 shadow (round to nearest even). */
spdba_status spdba_mlp_to_bf16(const float *w, uint16_t *w_bf16, int64_t nparam, void *stream);

/* Per-block features of the instances of `plan` (8 FP32 per block, all blocks
 * of all instances in the plan's block order), written to x:
 *   0..2  log10(a_b / G) at the three given indicator snapshots (newest first),
 *         clamped to [-40, 0], scaled by 1/40 and shifted by +1
 *   3     mean |k| over the block's modes / |k| at the Nyquist index
 *   4     active face neighbours (periodic block grid) / 6, from mask
 *   5     step fraction (a host scalar)
 *   6     log10(E_b nb / E_tot), E_b = sum over the block of |c_k|^2, clamped to
 *         [-40, 40], scaled by 1/40
 *   7     mask bit
 * ab[j] / G[j] (j = 0..2): device arrays of per-block FP64 indicator values
 * and per-instance FP64 maxima; mask: per-block u8; eb: per-block FP64 block
 * energies (from spdba_set_block_energy); scratch: 520 bytes per instance. */
spdba_status spdba_proposer_features(spdba_plan plan, const double *const ab[3],
                                     const double *const G[3], const uint8_t *mask,
                                     const double *eb, float step_fraction, float *x,
                                     void *scratch, void *stream);

/* Labels for training: y[b] = 1 if any of the n_masks per-block masks
 * (masks + j * total_blocks) marks block b active, else 0 (FP32). */
spdba_status spdba_proposer_labels(const uint8_t *masks, int32_t n_masks, int64_t total_blocks,
                                   float *y, void *stream);

/* Skip set from probabilities: skip[b] = prob[b] < threshold (u8).  gate
 * (device u32, may be NULL): when it holds a non-zero miss count the whole set
 * is cleared instead, so the next window runs the plain rule without a host
 * round trip.  count (device u32, may be NULL) accumulates the number of
 * blocks put in the set.  A NaN threshold is EINVAL. */
spdba_status spdba_proposer_skip(const float *prob, int64_t total_blocks, float threshold,
                                 const uint32_t *gate, uint8_t *skip, uint32_t *count, void *stream);

/* Audit: adds to *count (u32, device) the number of blocks that are in the
 * skip set and active in mask (integer atomics, order-free). */
spdba_status spdba_proposer_miss(const uint8_t *skip, const uint8_t *mask, int64_t total_blocks,
                                 uint32_t *count, void *stream);

/* Per-block energies: while d_eb != NULL, every update that evaluates the
 * indicator on all blocks also writes E_b = sum over the block of |q_k|^2
 * (FP64, both species for Gray-Scott) into d_eb (one double per block of the
 * plan); NULL turns it off. */
spdba_status spdba_set_block_energy(spdba_plan plan, double *d_eb);

#ifdef __cplusplus
}
#endif
#endif /* SPDBA_PROPOSER_H */
