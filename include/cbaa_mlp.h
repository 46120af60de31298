/*
 * cbaa_mlp.h -- learned cardinality estimator of libcbaa (an extension of the
 * paper's method, compared against it).
 *
 * The paper estimates a restored host's cardinality from the zero bits of its
 * union column with the eps-corrected linear count of Thm. 2 (from Eq. 1).
 * This interface adds a small network that maps the host's per-array column
 * popcounts ("per-layer" popcounts) to ln(1 + cardinality):
 *     z1 = W1 x + b1, h1 = relu(z1); z2 = W2 h1 + b2, h2 = relu(z2);
 *     y = w3 . h2 + b3;  estimate = exp(y) - 1.
 * Hidden width 64; weights W1, W2, w3 are bfloat16, biases fp32, all
 * accumulation fp32. z1 is computed in fp32 as b1 plus each input's product
 * in input order, and the second layer takes h1 rounded to bfloat16 (round to
 * nearest even), so that its 64 x 64 product is a bf16 contraction: inference
 * runs it on the matrix cores. Training minimises mean (y - t)^2 / 2 with Adam
 * on an fp32 master copy of every parameter; the gradient passes the rounding
 * of h1 unchanged.
 *
 * Parameter vector (fp32 master, P = cbaa_mlp_param_count(F) floats):
 *     W1 [64][F] row-major, b1 [64], W2 [64][64] row-major, b2 [64], w3 [64], b3
 * The bf16 copy d_wbf has the same P entries (uint16 bfloat16 bits); kernels
 * read weights from it and biases from the master.
 *
 * Features (cbaa_mlp_features), fp32 [n][F], in the log domain of the linear
 * count (Eq. 1) so that the network learns a correction of it: for each
 * array a, x[a] = ln(1 + g u_a), u_a = -ln(max(z_a, 1) / g), z_a = g - the
 * popcount of the host's column in array a; with F = n_ra + n_va + 2 also the
 * union column's ln(1 + g u), u = max(0, -ln(max(Z, 1) / (g - g eps))) (Thm. 2),
 * and g eps (Thm. 1); with F = n_ra + n_va + 4 further the union column's
 * ln(1 + g u) with g eps replaced by the sketch's row-aware shared-bit mass
 * M = sum over rows b of prod over arrays a of (columns of a with bit b set)
 * / c(a), and M itself. M extends Thm. 1 to rows that fill unevenly (it is
 * g eps when every row of an array is equally full); the rows fan-in hosts
 * set in almost every column are what it captures. Logarithms in fp64,
 * stored as fp32.
 *
 * Conventions as in cbaa.h: device pointers, caller-owned buffers, stream as
 * void*, CBAA_* return codes, asynchronous enqueue.
 */
#ifndef CBAA_MLP_H
#define CBAA_MLP_H

#include <stdint.h>

#include "cbaa.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Number of parameters for F features (1 <= F <= 8), 0 otherwise. */
uint32_t cbaa_mlp_param_count(uint32_t n_features);

/* He-uniform weights from a counter-based hash of (seed, index), zero biases,
 * and with zero_output != 0 a zero output layer (w3 = 0, b3 = 0: the network
 * then outputs exactly 0); writes the master and its bf16 copy. */
int cbaa_mlp_init(uint32_t n_features, uint32_t seed, int zero_output, float* d_master,
                  uint16_t* d_wbf, void* stream);

/* Per-host features from a cube (see above). n_features is n_ra + n_va,
 * n_ra + n_va + 2 or n_ra + n_va + 4 (at most 8). d_scratch holds
 * cbaa_restore_scratch_bytes(cfg, 0). */
int cbaa_mlp_features(const cbaa_config* h_cfg, const void* d_cube, const uint32_t* d_hosts,
                      uint64_t n, uint32_t n_features, float* d_x, void* d_scratch,
                      uint64_t scratch_bytes, void* stream);

/* d_y[k] = network output (ln(1 + cardinality) estimate) for d_x[k][0..F). */
int cbaa_mlp_forward(uint32_t n_features, const float* d_master, const uint16_t* d_wbf,
                     const float* d_x, uint64_t n, float* d_y, void* stream);

/* Gradient of mean over the n samples of (y - t)^2 / 2 into d_grad (P
 * floats, overwritten) and the loss into d_loss[0]. n >= 1. */
int cbaa_mlp_loss_grad(uint32_t n_features, const float* d_master, const uint16_t* d_wbf,
                       const float* d_x, const float* d_t, uint64_t n, float* d_grad,
                       float* d_loss, void* stream);

/* One Adam step (Kingma and Ba, with bias correction for step >= 1) on the
 * master, refreshing the bf16 copy; d_m and d_v are the moment buffers (P
 * floats each, zero before step 1). */
int cbaa_mlp_adam(uint32_t n_features, float* d_master, uint16_t* d_wbf, const float* d_grad,
                  float* d_m, float* d_v, uint32_t step, float lr, float beta1, float beta2,
                  float eps, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CBAA_MLP_H */
