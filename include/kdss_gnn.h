/*
 * kdss warm-start model -- a small message-passing network on gfx950.
 *
 * The loads r of Frank-Wolfe start from integers r0 (the paper's Algorithm 2
 * leaves "initialize r(u)" open); this model predicts y(u) ~ log1p(r*(u) / T),
 * the per-iteration load a long cold run reaches, from three node features
 * (degree, core number, triangle count), and r0 = round(t0 * expm1(y)).
 * Frank-Wolfe then runs unchanged (kdss_run with d_r0), so the results stay
 * exact; only the number of iterations to a good density changes.
 *
 * Model: x0 = features (n x 8 BF16, columns 3..7 zero);
 *   h1 = ReLU([x0 | mean_N(x0)] W1 + b1)      (K = 16)
 *   h2 = ReLU([h1 | mean_N(h1)] W2 + b2)      (K = 128)
 *   h3 = ReLU([h2 | mean_N(h2)] W3 + b3)      (K = 128)
 *   y  = h3 w + b                             (FP32)
 * Every product runs on the matrix cores with BF16 operands and FP32
 * accumulation (gfx950's v_mfma_f32_32x32x16_bf16, 16 k per instruction);
 * FP32 -> BF16 rounds to nearest even.
 *
 * Conventions as in kdss.h: device pointers are caller-owned, work is
 * enqueued on `stream` (a hipStream_t), status codes are kdss.h's.  Row-major
 * BF16 buffers are uint16_t; leading dimensions count elements and must be
 * multiples of 8; buffers must be 16-byte aligned.
 */
#ifndef KDSS_GNN_H
#define KDSS_GNN_H

#include "kdss.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Device workspace (bytes) that kdss_gnn_features needs for a graph of n nodes
 * and nnz directed edges (row_ptr[n]). */
int kdss_gnn_features_workspace(uint32_t n, uint64_t nnz, size_t *bytes);

/* x0 (device, n x 8 BF16) = [log1p(degree), log1p(core number),
 * log1p(triangles through the node), 0, ...] for the tree's graph (feature_set
 * 0), or the same with the triangle column 0 and no triangle counting
 * (feature_set 1), n = the
 * tree's node count.  d_row_ptr (u64[n + 1]) and d_col (u32[nnz]) are that
 * graph's CSR on the device; edges past nnz and ids >= n are ignored.  Core
 * numbers and the degeneracy order come from the tree's host build and are
 * copied up; on the device the edges are oriented along that order (a DAG
 * with out-degree <= degeneracy), the DAG's row offsets are scanned, and the
 * triangles are counted by intersecting out-neighbour lists.  Enqueued only. */
int kdss_gnn_features(const kdss_sct *s, const uint64_t *d_row_ptr, const uint32_t *d_col, uint64_t nnz,
                      int feature_set, uint16_t *d_x0, void *d_ws, size_t ws_bytes, void *stream);

/* out[u] = mean over neighbours v of h[v] (F = 8, 16, 32 or 64 columns; 0 for isolated nodes). */
int kdss_gnn_aggregate(uint32_t n, const uint64_t *d_row_ptr, const uint32_t *d_col, const uint16_t *d_h,
                       uint32_t F, uint16_t *d_out, void *stream);

/* Transpose of the mean: out[v] = dself[v] + sum over u in N(v) of dagg[u] / deg(u)
 * (dagg and dself have leading dimension ld; out is dense n x F). */
int kdss_gnn_aggregate_backward(uint32_t n, const uint64_t *d_row_ptr, const uint32_t *d_col,
                                const uint16_t *d_dagg, const uint16_t *d_dself, uint32_t F, uint32_t ld,
                                uint16_t *d_out, void *stream);

/* Y[M x 64] (leading dim ldy) = act([A1 | A2] Bt^T + bias): A1 has K1 columns,
 * A2 K2 (multiples of 8, K1 + K2 a multiple of 16 and at most 128; leading
 * dims multiples of 8; A1, A2 and Bt 16-byte aligned), Bt is 64 x (K1 + K2)
 * BF16, bias (nullable) 64 FP32, act = ReLU when relu != 0. */
int kdss_gnn_linear(uint32_t M, const uint16_t *d_a1, uint32_t K1, uint32_t lda1, const uint16_t *d_a2,
                    uint32_t K2, uint32_t lda2, const uint16_t *d_bt, const float *d_bias, int relu,
                    uint16_t *d_y, uint32_t ldy, void *stream);

/* dW[(K1 + K2) x 64] += [A1 | A2]^T dY and db[64] += column sums of dY (FP32,
 * accumulated; db nullable); K1, K2 multiples of 8 with K1 + K2 a multiple of 16
 * and at most 128; dY is M x 64 BF16. */
int kdss_gnn_linear_wgrad(uint32_t M, const uint16_t *d_a1, uint32_t K1, uint32_t lda1, const uint16_t *d_a2,
                          uint32_t K2, uint32_t lda2, const uint16_t *d_dy, float *d_dw, float *d_db,
                          void *stream);

/* dY[i] = 0 where Y[i] <= 0 (ReLU backward on BF16 buffers of `count` elements). */
int kdss_gnn_relu_backward(uint64_t count, const uint16_t *d_y, uint16_t *d_dy, void *stream);

/* pred[u] = sum_c h[u][c] w[c] + w[64]  (h: n x 64 BF16, w: 65 FP32). */
int kdss_gnn_head(uint32_t n, const uint16_t *d_h, const float *d_w, float *d_pred, void *stream);

/* Mean squared error against target: *loss += mean (pred - target)^2; with
 * d = 2 (pred - target) / n: dh = d w (BF16), dw[c] += sum d h[.][c], dw[64] += sum d. */
int kdss_gnn_head_backward(uint32_t n, const uint16_t *d_h, const float *d_w, const float *d_pred,
                           const float *d_target, uint16_t *d_dh, float *d_dw, float *d_loss, void *stream);

/* One Adam step (bias-corrected, step >= 1) on `count` FP32 parameters. */
int kdss_gnn_adam(uint32_t count, float *d_p, const float *d_g, float *d_m, float *d_v, float lr, float b1,
                  float b2, float eps, uint32_t step, void *stream);

/* BF16 copies of a K x 64 FP32 weight: W (K x 64, nullable) and Wt (64 x K, nullable). */
int kdss_gnn_pack_weights(uint32_t K, const float *d_w32, uint16_t *d_w, uint16_t *d_wt, void *stream);

/* r0[u] = round(t0 * expm1(pred[u])) clamped to [0, cap]; *d_rmax = max(*d_rmax, max r0)
 * (clear *d_rmax first). */
int kdss_gnn_warm_start(uint32_t n, const float *d_pred, double t0, uint64_t cap, uint64_t *d_r0,
                        uint64_t *d_rmax, void *stream);

/* ---- the whole model in one call (the start loads of Algorithm 2's
 * "initialize r(u)"; Frank-Wolfe itself is unchanged) ----
 * Parameters: one FP32 array of KDSS_GNN_PARAMS values (device, caller-owned):
 * W1 (16 x 64, row k = input column k: 8 self then 8 neighbour-mean columns),
 * b1, W2 (128 x 64), b2, W3 (128 x 64), b3, then the head w (64) and its bias. */
#define KDSS_GNN_W1 0
#define KDSS_GNN_B1 1024
#define KDSS_GNN_W2 1088
#define KDSS_GNN_B2 9280
#define KDSS_GNN_W3 9344
#define KDSS_GNN_B3 17536
#define KDSS_GNN_HEAD 17600
#define KDSS_GNN_PARAMS 17665

/* Device workspace (bytes) of kdss_gnn_infer (train = 0) or
 * kdss_gnn_train_step (train != 0) on n nodes: BF16 weight copies, per layer
 * the neighbour means and outputs, the prediction, and for training the
 * target, the activation gradients and the parameter gradient. */
int kdss_gnn_model_workspace(uint32_t n, int train, size_t *bytes);

/* Forward pass and warm start: y = head(h3), h_l = ReLU([h_{l-1} | mean_N(h_{l-1})] W_l + b_l),
 * h0 = x0 (n x 8 BF16, 16-byte aligned, from kdss_gnn_features), then
 * r0[u] = round(t0 * expm1(y[u])) clamped to [0, cap] into d_r0 (u64[n]) and
 * max(*d_rmax, max r0) into *d_rmax.  d_pred (nullable, FP32[n]) receives y.
 * d_ws (256-byte aligned) of kdss_gnn_model_workspace(n, 0) bytes.  Enqueued only.
 * Errors: KDSS_EINVAL, KDSS_EWORKSPACE, KDSS_EHIP. */
int kdss_gnn_infer(uint32_t n, const uint64_t *d_row_ptr, const uint32_t *d_col, const uint16_t *d_x0,
                   const float *d_params, double t0, uint64_t cap, void *d_ws, size_t ws_bytes, float *d_pred,
                   uint64_t *d_r0, uint64_t *d_rmax, void *stream);

/* One training step on one graph: the target y = log1p(r / T) from a cold
 * run's loads d_r (u64[n], T iterations), the forward pass, the mean squared
 * error over the nodes (added into *d_loss, device FP32), the backward pass
 * through the head, the three layers and the mean aggregation, and one Adam
 * step (lr, betas 0.9 / 0.999, eps 1e-8, bias correction at `step` >= 1) on
 * the KDSS_GNN_PARAMS parameters with moments d_m, d_v (device FP32, zero
 * before step 1).  d_ws of kdss_gnn_model_workspace(n, 1) bytes.  Enqueued
 * only.  Errors: KDSS_EINVAL, KDSS_EWORKSPACE, KDSS_EHIP. */
int kdss_gnn_train_step(uint32_t n, const uint64_t *d_row_ptr, const uint32_t *d_col, const uint16_t *d_x0,
                        const uint64_t *d_r, uint32_t T, float *d_params, float *d_m, float *d_v, uint32_t step,
                        float lr, void *d_ws, size_t ws_bytes, float *d_loss, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* KDSS_GNN_H */
