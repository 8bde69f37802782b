/*
 * lbmhd_learned.h -- learned correction of the subgrid closure, the
 * filtered-DNS pipeline that trains it, and energy spectra, for the engine of
 * lbmhd.h (Flint & Vahala, arXiv 1705.09807).
 *
 * The analytic closure of Sec. 2.1 / Sec. 3 keeps the first term of the
 * Delta-expansion FilterExampleSmall (filtered product = product of filtered
 * fields + Delta^2/12 products of gradients) and drops the density
 * gradients.  The learned closure adds, per cell, a correction
 * (tau_xx, tau_xy, tau_yy, eps) predicted by a small network from the local
 * resolved fields:
 *   tau_xy            enters M3, tau_xx - tau_yy enters M4,
 *   -3 (tau_xx + tau_yy) enters M7 and M8,
 *   eps               enters the induction moment (E = (u x B)_z + eps),
 * i.e. exactly where the analytic terms enter.  The network is trained on
 * filtered DNS: the exact subgrid terms of the filter's products minus the
 * analytic closure evaluated on the filtered fields.
 *
 * Conventions of lbmhd.h apply (return codes, lbm_last_error, caller-owned
 * 256-byte aligned device buffers, asynchronous on the given stream, natural
 * [plane][y][x] layout).  `hip_stream` is a hipStream_t (NULL = null stream).
 *
 * Network.  Inputs: the 3x3 neighbourhood of seven fields, in this order
 *   0 rho, 1 u_x = m_x / rho, 2 u_y, 3 B_x, 4 B_y,
 *   5 w = D_x u_y - D_y u_x, 6 J_z = D_x B_y - D_y B_x  (central differences),
 * feature k = field * 9 + (dy + 1) * 3 + (dx + 1) for offsets dx, dy in
 * {-1, 0, 1}, k < 63; feature 63 is a zero pad.  Normalised inputs
 *   z_k = (x_k - shift[field]) * scale[field]    (FP32 arithmetic),
 * then z, both hidden activations and all weights are rounded to bfloat16
 * (nearest even) and multiplied on the matrix cores with FP32 accumulation:
 *   h1 = relu(W1^T z + b1), h2 = relu(W2^T h1 + b2), y = W3^T h2 + b3,
 * 63 -> 64 -> 64 -> 4, and the correction is out_scale * y.  A cell with any
 * |z_k| > 6 is out of the training distribution and keeps the analytic
 * closure (correction 0); so does a cell with a non-finite input or output.
 */
#ifndef LBMHD_LEARNED_H
#define LBMHD_LEARNED_H

#include <stddef.h>
#include <stdint.h>

#include "lbmhd.h"

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_MLP_FIELDS 7
#define LBM_MLP_FEATURES 64   /* 63 inputs + one zero pad                      */
#define LBM_MLP_HIDDEN 64
#define LBM_MLP_OUTPUTS 4     /* tau_xx, tau_xy, tau_yy, eps                    */

/* FP32 master parameters, one contiguous array of LBM_MLP_PARAMS floats:
 *   w1[k][i] at LBM_MLP_OFF_W1 + k*64 + i   (input k, hidden i; row 63 is
 *                                             the pad and must stay 0)
 *   b1[i], w2[i][j] (hidden i -> hidden j), b2[j], w3[j][o], b3[o].       */
#define LBM_MLP_OFF_W1 0
#define LBM_MLP_OFF_B1 4096
#define LBM_MLP_OFF_W2 4160
#define LBM_MLP_OFF_B2 8256
#define LBM_MLP_OFF_W3 8320
#define LBM_MLP_OFF_B3 8576
#define LBM_MLP_PARAMS 8580

/* Input and output normalisation (device memory, 128 bytes). */
typedef struct {
  float shift[8];      /* per input field; entry 7 unused                    */
  float scale[8];
  float out_scale[4];  /* correction = out_scale * y                         */
  float pad[12];
} lbm_mlp_norm;

/* Device bytes of a packed network (bfloat16 weights in matrix-core operand
 * order, FP32 biases, the normalisation). */
#define LBM_MLP_PACKED_BYTES 31744

/* Pack FP32 parameters and a normalisation into `packed_dev`
 * (LBM_MLP_PACKED_BYTES): weights rounded to bfloat16, nearest even. */
int lbm_mlp_pack(const float* params_dev, const lbm_mlp_norm* norm_dev, void* packed_dev, void* hip_stream);

/* Network on n >= 0 feature rows x_dev[n][64] (FP32; column 63 ignored):
 * y_dev[n][4] = y (before out_scale); ood_dev[n] (may be NULL) = 1 where any
 * |z_k| > 6 or is not finite, else 0. */
int lbm_mlp_forward(const void* packed_dev, const float* x_dev, int64_t n, float* y_dev, int32_t* ood_dev,
                    void* hip_stream);

/* Normalisation from n >= 2 training rows: shift = mean and scale = 1/std
 * (population std; 1 where it is 0) of each field's centre feature
 * x[:, field*9 + 4]; out_scale = root mean square of each target column
 * t[:, o] (1 where it is 0).  FP64 sums in a fixed order, rounded to FP32.
 * work_dev: >= lbm_mlp_stats_work_bytes(n) bytes. */
size_t lbm_mlp_stats_work_bytes(int64_t n);
int lbm_mlp_feature_stats(const float* x_dev, const float* t_dev, int64_t n, lbm_mlp_norm* norm_dev,
                          void* work_dev, size_t work_bytes, void* hip_stream);

/* One Adam step (Kingma & Ba 2015; beta1 0.9, beta2 0.999, eps 1e-8, bias
 * corrected, step >= 1) on the mean squared error over the batch rows
 * idx_dev[0..batch) of x_dev[n][64] against the normalised targets
 * t_dev[row][o] / out_scale[o].  Gradients of the bfloat16 forward are taken
 * straight through the roundings (FP32 arithmetic, deterministic order).
 * params_dev, adam_m_dev, adam_v_dev (LBM_MLP_PARAMS floats each) are
 * updated in place; loss_dev (1 float, may be NULL) receives the batch loss
 * before the update.  1 <= batch <= 1<<20; row indices are not checked
 * against n: the caller guarantees 0 <= idx < rows of x_dev and t_dev.
 * work_dev: >= lbm_mlp_train_work_bytes(batch) bytes. */
size_t lbm_mlp_train_work_bytes(int32_t batch);
int lbm_mlp_train_step(float* params_dev, float* adam_m_dev, float* adam_v_dev, int64_t step, double lr,
                       const lbm_mlp_norm* norm_dev, const float* x_dev, const float* t_dev,
                       const int32_t* idx_dev, int32_t batch, void* work_dev, size_t work_bytes,
                       float* loss_dev, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight training loops, harnesses that forbid hipMalloc): the same
 * Adam step as lbm_mlp_train_step, with the same kernels and bit-identical
 * results, but no work buffer.  Its work lives in a fixed array of
 * LBM_MLP_TRAIN_NOALLOC_BYTES bytes of device memory that the library holds
 * on every GPU it runs on until the process ends; the call allocates and
 * frees nothing.  1 <= batch <= LBM_MLP_TRAIN_NOALLOC_BATCH; a larger batch
 * returns LBM_EINVAL before any work is enqueued.  hip_stream must belong to
 * the current device.  All calls on one GPU share that GPU's array: calls
 * that overlap on one GPU (other streams or host threads) race and must be
 * serialised by the caller.  Other arguments and rules as for
 * lbm_mlp_train_step. */
#define LBM_MLP_TRAIN_NOALLOC_BATCH 16384
#define LBM_MLP_TRAIN_NOALLOC_BYTES 9437184
int lbm_mlp_train_step_noalloc(float* params_dev, float* adam_m_dev, float* adam_v_dev, int64_t step, double lr,
                               const lbm_mlp_norm* norm_dev, const float* x_dev, const float* t_dev,
                               const int32_t* idx_dev, int32_t batch, float* loss_dev, void* hip_stream);

/* The two halves of lbm_mlp_train_step, for callers that combine gradients
 * (e.g. summed over data-parallel replicas) before the update:
 * lbm_mlp_gradient writes the batch gradient (LBM_MLP_PARAMS floats) to
 * grad_dev and the batch loss to loss_dev (may be NULL); lbm_mlp_adam applies
 * one Adam step with that gradient.  Same arguments, work and rules as
 * lbm_mlp_train_step. */
int lbm_mlp_gradient(const float* params_dev, const lbm_mlp_norm* norm_dev, const float* x_dev, const float* t_dev,
                     const int32_t* idx_dev, int32_t batch, void* work_dev, size_t work_bytes, float* grad_dev,
                     float* loss_dev, void* hip_stream);
int lbm_mlp_adam(float* params_dev, float* adam_m_dev, float* adam_v_dev, const float* grad_dev, int64_t step,
                 double lr, void* hip_stream);

/* Filter and subsample (the convolution of Sec. 1, VelFilter, with a
 * Gaussian of variance delta^2/12: the second moment the expansion of
 * Sec. 2.1 assumes).  Taps w(r) = exp(-r^2 / (2 sigma^2)), |r| <= R =
 * ceil(5 sigma), sigma^2 = delta^2/12, normalised to sum 1, applied along x
 * then y on the periodic nx x ny grid and sampled every `factor` cells:
 *   out[k](X, Y) = sum_{i,j} w(i) w(j) p_k(factor X + i, factor Y + j).
 * mom_dev: 5 FP64 planes rho, m_x, m_y, B_x, B_y (lbm_moments).  out_dev:
 * 12 FP64 planes of (nx/factor) x (ny/factor): p = rho, m_x, m_y, B_x, B_y,
 * m_x m_x / rho, m_x m_y / rho, m_y m_y / rho, B_x B_x, B_x B_y, B_y B_y,
 * (m_x B_y - m_y B_x) / rho.  factor in {1, 2, 4, 8, 16} dividing nx and ny;
 * delta > 0 with R < min(nx, ny) and R <= 127.
 * work_dev: >= lbm_filter_work_bytes(...) bytes (0 = invalid arguments). */
size_t lbm_filter_work_bytes(int32_t nx, int32_t ny, int32_t factor, double delta);
int lbm_filter_subsample(const double* mom_dev, int32_t nx, int32_t ny, int32_t factor, double delta,
                         double* out_dev, void* work_dev, size_t work_bytes, void* hip_stream);

/* Training samples from the 12 filtered planes of an nx x ny (coarse) grid
 * (lbm_filter_subsample): x_dev[n][64] = the network inputs of every cell
 * (FP64 arithmetic, stored FP32), t_dev[n][4] = exact subgrid terms
 *   tau_xx = R_xx + (Q_yy - Q_xx)/2, tau_xy = R_xy - Q_xy,
 *   tau_yy = R_yy + (Q_xx - Q_yy)/2, eps = bar((m x B)_z / rho) - (bar m x bar B)_z / bar rho,
 * with R_ab = bar(m_a m_b / rho) - bar m_a bar m_b / bar rho and
 * Q_ab = bar(B_a B_b) - bar B_a bar B_b, minus the analytic closure of the
 * filtered fields with k2 = delta^2 / 12 (delta in cells of this grid) and
 * the given LBM_STENCIL_*.  Cell c = y * nx + x; nx, ny in [4, 32768]. */
int lbm_closure_samples(const double* coarse_dev, int32_t nx, int32_t ny, double delta, int32_t grad_stencil,
                        float* x_dev, float* t_dev, void* hip_stream);

/* Install a packed network in a context created with closure =
 * LBM_CLOSURE_LEARNED (copied into the context's work buffer; `packed_dev`
 * may be reused afterwards).  lbm_step on such a context returns LBM_ESTATE
 * until a network is installed.  Each step then computes the moments of the
 * state, the network's correction of every cell, and the fused collision
 * with the analytic closure plus the correction. */
int lbm_set_closure_mlp(lbm_ctx* ctx, const void* packed_dev);

/* The correction of the current state: 4 FP32 planes tau_xx, tau_xy,
 * tau_yy, eps (out_scale applied, 0 in out-of-distribution cells) into
 * out_dev (4*nx*ny floats).  The correction that lbm_step holds between
 * evaluations (lbm_set_correction_interval) is left as it is. */
int lbm_closure_correction(lbm_ctx* ctx, float* out_dev);

/* Evaluation cadence of the learned correction (the correction is this
 * library's addition to the closure of Sec. 2.1, so the cadence is its own
 * definition).  With every = K >= 1 (default 1: every step), lbm_step
 * evaluates the network on the state being collided at every step t with
 * t % K == 0 and at the first step after lbm_init_*, lbm_set_state,
 * lbm_set_closure_mlp or this call, and holds that correction (4 FP32 planes
 * in the context's work buffer) for the steps in between, which then launch
 * only the collision sweep.  A run restarted from a saved state at a t that
 * is not a multiple of K evaluates once more than the uninterrupted run.
 * Errors: LBM_ESTATE if the context was not created with the learned
 * closure, LBM_EINVAL if every < 1. */
int lbm_set_correction_interval(lbm_ctx* ctx, int32_t every);

/* Radially binned energy spectra of an n x n periodic field, n a power of
 * two in [8, 16384]: with a_hat(k) = N^-2 sum_x a(x) exp(-2 pi i k.x / N) and
 * integer k_a in [-n/2, n/2),
 *   ek[b] = 1/2 sum_{round(|k|) = b} |u_x_hat|^2 + |u_y_hat|^2  (u = m / rho),
 *   em[b] = the same for B,  b = 0 .. lbm_spectra_bins(n) - 1,
 *   ekx[m] (may be NULL) = 1/2 sum_{|k_x| = m} |u_x_hat|^2 + |u_y_hat|^2,
 *   m = 0 .. n/2,
 * round(r) = floor(r + 1/2).  FP64 FFTs and fixed-order sums.  mom_dev: the
 * 5 FP64 planes of lbm_moments (or the first 5 of lbm_filter_subsample).
 * work_dev: >= lbm_spectra_work_bytes(n) bytes (0 = invalid n): the row
 * transforms (32 n^2 bytes), the per-column bins (16 n lbm_spectra_bins(n))
 * and, beyond n = 4096, the column powers (16 n^2); 0.86 GB at 4096,
 * 18.1 GB at 16384. */
int32_t lbm_spectra_bins(int32_t n);
size_t lbm_spectra_work_bytes(int32_t n);
int lbm_spectra(const double* mom_dev, int32_t n, double* ek_dev, double* em_dev, double* ekx_dev, void* work_dev,
                size_t work_bytes, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LBMHD_LEARNED_H */
