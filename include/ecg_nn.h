/*
 * ecg_nn.h - learned factorised preconditioner M^{-1} = G G^T for the flexibly enlarged CG
 * solver (split preconditioning, Section 4.5, eq. (zsre2): L^{-1} = G^T, L^{-T} = G).
 *
 * G is lower triangular on the pattern of the lower triangle of a 5-point operator on an
 * nx x ny grid in natural order (x fastest): row i holds G_ii, G_i,i-1 (west) and
 * G_i,i-nx (south).  A per-row network maps the local stencil to these three entries:
 *   f_i = (log a_ii, a_iW/a_ii, a_iE/a_ii, a_iS/a_ii, a_iN/a_ii, log(a_WW/a_ii), log(a_SS/a_ii))
 *   with a_WW, a_SS the diagonal entries of the west and south neighbours (0 when absent),
 *   h1 = tanh(W1 f + b1) (32), h2 = tanh(W2 h1 + b2) (32), o = W3 h2 + b3 (3),
 *   G_ii = a_ii^{-1/2} exp(o_0), G_i,i-1 = a_ii^{-1/2} o_1, G_i,i-nx = a_ii^{-1/2} o_2,
 * so G_ii > 0 and G G^T is SPD for every parameter vector.  Training minimises the mean
 * over operators of ||G G^T b - x||_A^2 / ||x||_A^2 (x = A^{-1} b, produced by ecg_solve).
 *
 * Conventions are those of ecg.h (status codes, ecg_last_error, streams: every call
 * enqueues on hip_stream and returns after the work completed).
 *
 * Layouts (all device memory, a batch of nb operators of n = nx*ny rows each):
 *   a5     double [nb][5][n]  stencil: diagonal, west, east, south, north (0 when absent)
 *   g3     double [nb][3][n]  G_ii, G_i,i-1, G_i,i-nx (0 when absent)
 *   b, x   double [nb][n]
 *   params float  [ECG_NN_NPARAM]  W1 (32x7 row-major), b1, W2 (32x32), b2, W3 (3x32), b3
 *   grad, adam moments  double [ECG_NN_NPARAM]
 * Preconditions checked: nx, ny >= 2, nb >= 1, nx*ny*nb < 2^31, every a_ii > 0 is the
 * caller's responsibility (the kernels take its logarithm and inverse square root).
 */
#ifndef ECG_NN_H
#define ECG_NN_H

#include "ecg.h"

#ifdef __cplusplus
extern "C" {
#endif

#define ECG_NN_NPARAM 1411

/* g3 = entries of G predicted by the network for every row of every operator. */
ecg_status ecg_nn_forward(int32_t nx, int32_t ny, int32_t nb, const double* a5, const float* params,
                          double* g3, void* hip_stream);

/* Bytes of device workspace for ecg_nn_loss_grad / ecg_nn_backward with these sizes. */
ecg_status ecg_nn_workspace_size(int32_t nx, int32_t ny, int32_t nb, size_t* bytes);

/* Per operator s: loss[s] = ||G G^T b - x||_A^2 / ||x||_A^2 (device double[nb]) and
 * dg3[s] = d loss[s] / d g3[s] (same layout as g3).  workspace: >= ecg_nn_workspace_size. */
ecg_status ecg_nn_loss_grad(int32_t nx, int32_t ny, int32_t nb, const double* a5, const double* g3,
                            const double* b, const double* x, double* loss, double* dg3, void* workspace,
                            size_t ws_bytes, void* hip_stream);

/* grad = scale * sum over operators and rows of the backpropagation of dg3 through the
 * network (the network is re-evaluated from a5 and params).  Deterministic order. */
ecg_status ecg_nn_backward(int32_t nx, int32_t ny, int32_t nb, const double* a5, const float* params,
                           const double* dg3, double scale, double* grad, void* workspace, size_t ws_bytes,
                           void* hip_stream);

/* One Adam step (Kingma and Ba, bias-corrected; step counts from 1) on params (float) with
 * moments m, v (double) and gradient grad (double). */
ecg_status ecg_nn_adam(int32_t nparam, float* params, const double* grad, double* m, double* v, int32_t step,
                       double lr, double beta1, double beta2, double eps, void* hip_stream);

/* The classical factor on the same pattern, as the baseline of the network (factorised sparse
 * approximate inverse, Kolotilina and Yeremin): g3 = the G that minimises the Kaporin condition
 * number of G^T A G among lower-triangular G on the pattern, in closed form for a 5-point
 * operator (column j of G is A_C^{-1} e_1 scaled to unit A-norm, C = {j, j+1, j+nx}).  a5, g3
 * as above; every Schur complement a_jj - a_jE^2/a_EE - a_jN^2/a_NN must be positive (true for
 * SPD A; not checked). */
ecg_status ecg_nn_fsai(int32_t nx, int32_t ny, int32_t nb, const double* a5, double* g3, void* hip_stream);

/* CSR of G for one operator (g3 holds [3][n]): rowptr int64[n+1], colind int32[nnz],
 * vals double[nnz] with nnz = 3n - ny - nx, each row sorted with the diagonal last (the
 * layout ecg_precond_create_factor expects).  All device pointers. */
ecg_status ecg_nn_factor_csr(int32_t nx, int32_t ny, const double* g3, int64_t* rowptr, int32_t* colind,
                             double* vals, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* ECG_NN_H */
