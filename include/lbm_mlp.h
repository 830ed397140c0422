/*
 * lbm_mlp.h - the learned activation proposal of liblbm: a small multilayer
 * perceptron that predicts which inactive blocks the criterion of Eq 13
 * (section 4.2 of arXiv 1510.03560) will request within the next K steps, so
 * that they can be meshed ahead of need.  The criterion still decides every
 * activation the method needs; a block activated early holds the rest state
 * its inactive self stands for, so the fields stay bit-identical.
 *
 * Network: x (12 features) -> standardise -> h1 = relu(W1 x' + b1) (64)
 *          -> h2 = relu(W2 h1 + b2) (64) -> z = w3 . h2 + b3 -> p = 1/(1+e^-z).
 * Parameters, one FP32 vector of LBM_MLP_NPARAMS values in this order:
 *   mean[12], inv_std[12], W1[64][12], b1[64], W2[64][64], b2[64], w3[64], b3[1]
 * (x' = (x - mean) * inv_std; mean and inv_std are not trained).
 * Loss: binary cross-entropy on the logits, averaged over the batch.
 *
 * All pointers are DEVICE pointers owned by the caller; work is enqueued on
 * `stream` (a hipStream_t, NULL for the null stream) and the calls return
 * before it finishes.  Return LBM_OK or LBM_EINVAL / LBM_EHIP (lbm.h).
 */
#ifndef LBM_MLP_H
#define LBM_MLP_H

#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_MLP_IN 12
#define LBM_MLP_HIDDEN 64
#define LBM_MLP_NPARAMS (2 * 12 + 64 * 12 + 64 + 64 * 64 + 64 + 64 + 1)

/* Forward pass: logits[n] for samples x[n][12].  h1, h2 (n x 64 each) receive
 * the hidden activations when non-NULL (the backward pass needs them). */
int lbm_mlp_forward(const float* params, const float* x, int32_t n, float* logits, float* h1, float* h2,
                    void* stream);

/* Gradient of the mean binary cross-entropy of logits against labels y[n]
 * (0 or 1) with respect to the trainable parameters, written into grad
 * (LBM_MLP_NPARAMS values; the mean/inv_std entries are set to 0).  Needs
 * the logits and hidden activations of lbm_mlp_forward on the same x, and a
 * scratch of n x 129 floats.  The per-parameter sums run over the samples in
 * order, so the result does not depend on scheduling.  Also writes the mean
 * loss to loss[0] when loss is non-NULL. */
int lbm_mlp_backward(const float* params, const float* x, const float* y, int32_t n, const float* logits,
                     const float* h1, const float* h2, float* scratch, float* grad, float* loss, void* stream);

/* One Adam step (Kingma and Ba 2015): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), for the
 * trainable parameters (t >= 1 is the step number). */
int lbm_mlp_adam(float* params, const float* grad, float* m, float* v, int32_t t, float lr, float beta1,
                 float beta2, float eps, void* stream);

/* Proposal features of the current state of a handle (progressive mesh):
 * for every inactive block holding fluid with at least one active
 * neighbour (a candidate), 12 values (listed at lbm_set_proposal below)
 * into feat[cap][12] and the block id into block[cap]
 * (device buffers).  Returns the number of candidates (may exceed cap; only
 * cap are written) or a negative error.  Synchronous. */
int lbm_proposal_features(lbm_t* h, float* feat, int32_t* block, int32_t cap);

/* Enables (enable >= 1) or disables (enable <= 0) the proposal inside
 * lbm_step: after the criterion of every step whose index is a multiple of
 * enable, every candidate block whose predicted probability exceeds
 * threshold is activated as well (enable = 1: every step; the network looks
 * K = 20 steps ahead, so running it every few steps loses little).  params: host array of LBM_MLP_NPARAMS
 * values, copied.  Features of candidate N: the means, over the cells of its
 * active neighbours within shell_width cells of N, of rho_1, rho_2, |u_1|,
 * |u_2|, |psi_1 - psi_rest,1|, |psi_2 - psi_rest,2| (Eq 4-7 on the state the
 * criterion sees); the steps since a neighbour of N was last activated; the
 * fraction of N's cells that are fluid; the number of N's 26 neighbours that
 * are active; the mean over them of the unit vector pointing to N. */
int lbm_set_proposal(lbm_t* h, const float* params, float threshold, int32_t enable);

#ifdef __cplusplus
}
#endif
#endif /* LBM_MLP_H */
