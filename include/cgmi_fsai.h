/*
 * cgmi_fsai.h -- learned factored sparse-approximate-inverse preconditioner.
 *
 * Not part of the paper (which solves with unpreconditioned CG, Section 3.1):
 * a preconditioned form of the same solver.  M^-1 = G^T G with G lower
 * triangular on the pattern of tril(A).  For 5-point operators in x-fastest
 * order a row i of G has the slots C (column i), W (i-1) and S (i-nx).  A
 * multilayer perceptron 12 -> 64 -> 64 -> 5 (ReLU; bfloat16 weights and
 * activations, float32 accumulation on the matrix cores) maps 12 features of
 * row i of A_hat = D^-1/2 A D^-1/2 to outputs o = [o_C, o_W, o_E, o_S, o_N]:
 *
 *   features: a_ij / sqrt(d_i d_j), log(d_j / d_i), and 1 if absent, for the
 *             neighbours j = W, E, S, N (0 when absent);
 *   factor:   G~_ii = softplus(o_C) + 1e-3, G~_iW = o_W, G~_iS = o_S,
 *             G = G~ D^-1/2   (o_E, o_N unused).
 *
 * Training minimises L = (1/|S|) sum_{i in S} sum_j ((G A G^T)_ij - delta_ij)^2
 * over sampled rows S of generated systems, with Adam on float32 master
 * weights.  Parameters are a flat float32 vector of CG_FSAI_NPARAMS values:
 * W1 (64 x 12, row-major), b1 (64), W2 (64 x 64), b2 (64), W3 (5 x 64), b3 (5).
 *
 * Conventions as in cgmi.h (host CSR arrays are copied, return codes,
 * cg_last_error).  The operators must be 5-point (at most one entry per
 * stencil slot), symmetric, with a positive diagonal; otherwise CG_EINVAL.
 */
#ifndef CGMI_FSAI_H
#define CGMI_FSAI_H

#include <stdint.h>

#include "cgmi.h"

#ifdef __cplusplus
extern "C" {
#endif

#define CG_FSAI_NPARAMS 5317

/* Install the learned factor on a GPU-only solver: features, network
 * inference (matrix cores) and the assembly of G and G^T all run on the
 * device from the handle's matrix.  theta: host, CG_FSAI_NPARAMS floats.
 * Afterwards cg_opts.precond = CG_PC_FSAI makes cg_solve run PCG with
 * z = G^T (G r).  Blocking. */
int cg_fsai_setup(cg_handle *h, const float *theta);

/* Install an explicit factor G (host CSR, lower triangular, n x n, copied);
 * G^T is formed by the library.  For non-learned factors (identity, Jacobi,
 * classic FSAI) and for checking the preconditioned solve. */
int cg_set_fsai(cg_handle *h, int64_t nnz, const int32_t *g_row_ptr, const int32_t *g_col,
                const double *g_val);

/* Install the classic (non-learned) FSAI factor of Kolotilina and Yeremin
 * on the pattern of tril(A), the reference a learned factor is compared
 * with: row i of G holds the solution g of A[P_i, P_i] g = e_i over its
 * pattern P_i (the columns of row i of tril(A), i last), scaled by
 * 1 / sqrt(g_i), so that G A G^T has a unit diagonal.  Each local system is
 * solved by a Cholesky factorisation on host threads.  Any SPD matrix whose
 * tril(A) rows have at most CG_FSAI_CLASSIC_MAX_ROW entries; CG_EINVAL for a
 * longer row, a row without a diagonal entry, or a local system that is not
 * positive definite.  GPU-only handles.  Blocking. */
#define CG_FSAI_CLASSIC_MAX_ROW 8
int cg_fsai_classic(cg_handle *h);

/* Read back the installed factor's values (host, float64, nnz of G in CSR
 * order of the tril(A) pattern for a learned factor). */
int cg_fsai_factor_info(const cg_handle *h, int64_t *nnz);
int cg_fsai_read_factor(const cg_handle *h, int32_t *g_row_ptr, int32_t *g_col, double *g_val);

/* ---- training ----------------------------------------------------------- */
typedef struct cg_fsai_trainer cg_fsai_trainer;

/* Upload nsys training systems (host CSR arrays, copied), precompute their
 * features on the device, and start from the parameters theta0 (host). */
int cg_fsai_trainer_create(int32_t nsys, const int32_t *n, const int64_t *nnz,
                           const int32_t *const *row_ptr, const int32_t *const *col,
                           const double *const *val, const float *theta0,
                           cg_fsai_trainer **out);
void cg_fsai_trainer_destroy(cg_fsai_trainer *t);

/* Loss and gradient for the current parameters (or theta, if not NULL) on the
 * sampled rows: nsel systems sys[0..nsel), rows_per_sys local row indices each
 * in rows[s * rows_per_sys + r].  Writes loss (host double) and grad (host,
 * CG_FSAI_NPARAMS floats; may be NULL).  outputs (may be NULL): the network
 * outputs of system sys[0], n x 5 floats row-major. */
int cg_fsai_loss_grad(cg_fsai_trainer *t, const float *theta, int32_t nsel, const int32_t *sys,
                      int32_t rows_per_sys, const int32_t *rows, double *loss, float *grad,
                      float *outputs);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on the
 * loss of the sampled rows; writes the loss before the step. */
int cg_fsai_train_step(cg_fsai_trainer *t, int32_t nsel, const int32_t *sys,
                       int32_t rows_per_sys, const int32_t *rows, double lr, double *loss);

/* Current float32 master parameters (host, CG_FSAI_NPARAMS floats). */
int cg_fsai_get_params(const cg_fsai_trainer *t, float *theta);

/* The whole optimiser state, for checkpoints: the float32 master parameters,
 * Adam's first and second moment estimates (CG_FSAI_NPARAMS floats each,
 * host) and the number of Adam steps taken (the next step is step + 1).
 * Any of the arrays may be NULL (not read / not written).  set: step >= 0.
 * A trainer restored from a checkpoint continues as the one that wrote it
 * (the next step uses step + 1 in the bias correction); the loss gradients
 * are summed in 64-bit fixed point (order-independent), so a resumed run and
 * an uninterrupted one over the same samples agree bit for bit. */
int cg_fsai_get_state(const cg_fsai_trainer *t, float *theta, float *m, float *v, int32_t *step);
int cg_fsai_set_state(cg_fsai_trainer *t, const float *theta, const float *m, const float *v, int32_t step);

/* Features of system sys as the device computed them (host, n x 12 floats,
 * each already rounded to bfloat16). */
int cg_fsai_features(const cg_fsai_trainer *t, int32_t sys, float *feats);

#ifdef __cplusplus
}
#endif
#endif /* CGMI_FSAI_H */
