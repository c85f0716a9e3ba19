/*
 * libgmres, learned sparse approximate inverse (SPAI) for flexible GMRES.
 *
 * Algorithm 1 of Lindquist, Luszczek, Dongarra (arXiv 2011.01850) takes a
 * preconditioner M^-1 ~ A^-1 as an input; its experiments use ILU(0).  Here
 * M is produced by a small message-passing network over the stored entries
 * ("edges") of A and has A's own sparsity pattern; gmres_set_preconditioner
 * applies it on the right in flexible GMRES.  The network is this project's
 * definition (the paper prescribes none):
 *
 *   d_i = |a_ii| (1 if 0), sigma_i = sign(a_ii), ahat_ij = a_ij / sqrt(d_i d_j)
 *   edge input  f_ij = [ahat_ij, ahat_ji (0 if not stored), [i == j]]
 *   node input  x_i  = [sum_{j!=i} ahat_ij, sum_{j!=i} |ahat_ij|, sum_{j!=i} ahat_ji]
 *   h_i = relu(Wn x_i + bn), e_ij = relu(We f_ij + be)              (width 32)
 *   3 layers: u_ij = [h_i, h_j, e_ij]; m_ij = relu(W_l u_ij + b_l);
 *             h_i += (1/deg_i) sum_j m_ij; e_ij = m_ij
 *   s_ij = wo . [h_i, h_j, e_ij] + bo;  M_ij = (sigma_i [i==j] + s_ij) / sqrt(d_i d_j)
 *
 * so a zero decoder gives Jacobi.  Training minimises
 *   L = (1/K) sum_k ||A M z_k - z_k||^2 / ||z_k||^2
 * over residuals z_k that the solver itself produces.
 *
 * Parameters: one flat vector of SPAI_NPARAMS values in the order
 * Wn[32x3] bn[32] We[32x3] be[32] W1[32x96] b1[32] W2[32x96] b2[32]
 * W3[32x96] b3[32] wo[96] bo[1] (matrices row-major, output x input).  The
 * network reads them as bfloat16 (uint16 bit patterns); products of the
 * message layers run on the matrix cores (bfloat16 inputs, float32
 * accumulation); everything else is float32.  Optimiser state and master
 * weights are float32.
 *
 * Conventions: array arguments are DEVICE pointers; return values are the
 * GMRES_* codes of gmres.h (0 = OK, negative = error).  Each handle owns a
 * non-blocking stream of default priority, waits for the caller's stream
 * (given at creation, NULL = null stream) before reading caller memory and
 * returns after its own stream drains.  One host thread per handle.
 */
#ifndef SPAI_H_
#define SPAI_H_

#include <stddef.h>
#include <stdint.h>

#include "gmres.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { SPAI_NPARAMS = 9665, SPAI_HIDDEN = 32 };

typedef struct spai_ctx* spai_handle;

/* Network instance for one sparsity pattern (CSR row_ptr int32[n+1],
 * col_idx int32[nnz], no duplicate entries).  kmax = the largest number
 * of residual vectors one spai_loss call will take.  Builds the transposed
 * pattern on the host once.  Errors: EINVAL (n <= 0, kmax < 1, bad or
 * duplicated pattern), ENOMEM, EHIP. */
int spai_create(spai_handle* out, int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                int32_t kmax, void* hip_stream);

/* Values of A on the pattern (float64[nnz], CSR order): computes the
 * network inputs and a float32 copy of A for the loss. */
int spai_set_values(spai_handle h, const double* vals);

/* Forward pass: params (uint16 bfloat16 bits [SPAI_NPARAMS]) -> M values
 * (float32[nnz], A's storage order).  Keeps the activations for
 * spai_backward.  Requires spai_set_values. */
int spai_forward(spai_handle h, const uint16_t* params, float* m_out);

/* Loss of M (float32[nnz]) on K residuals Z (float32, K vectors of n
 * values, vector k at Z + k n), K <= kmax: *loss_out (host) = L as above,
 * and, if dm_out is not NULL, dL/dM on the pattern (float32[nnz]).  A zero
 * vector z_k is an error (EINVAL, detected on the device). */
int spai_loss(spai_handle h, const float* m_vals, const float* Z, int32_t K, double* loss_out, float* dm_out);

/* Backward pass of the last spai_forward (same params): given dL/dM
 * (float32[nnz]) writes dL/dparams (float32[SPAI_NPARAMS]) into grad, or
 * adds to it when accumulate != 0.  Reductions are in a fixed order
 * (deterministic). */
int spai_backward(spai_handle h, const uint16_t* params, const float* dm, float* grad, int32_t accumulate);

/* *same_out = 1 if (n, nnz, row_ptr, col_idx) (device CSR) is the
 * network's pattern, else 0 (compared on the device). */
int spai_same_pattern(spai_handle h, int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                      int32_t* same_out);

int spai_destroy(spai_handle h);

/* One Adam step (Kingma & Ba) on float32 master weights theta[count],
 * moments m1, m2 (float32[count]), step t >= 1 (bias correction), then
 * params_bf16 = round-to-nearest-even bfloat16(theta).  grad is scaled by
 * grad_scale first.  Runs on hip_stream and synchronises it. */
int spai_adam_step(int64_t count, float* theta, uint16_t* params_bf16, const float* grad, float grad_scale,
                   float* m1, float* m2, float lr, float beta1, float beta2, float eps, int32_t t,
                   void* hip_stream);

/* Inference for a solver handle (single system, created with
 * precond = GMRES_PRECOND_SPAI): runs the network on the handle's own
 * matrix and installs M (as gmres_set_preconditioner does).  If m_out is
 * not NULL the M values are also copied there (float32[nnz]).
 * param_bytes must be SPAI_NPARAMS * 2. */
int gmres_spai_infer(gmres_handle h, const void* params, size_t param_bytes, float* m_out);

/* The same with a caller-owned network instance `net` created for this
 * handle's pattern (checked on the device: ESTATE if it differs), so a
 * family of matrices with one pattern pays the pattern setup once; the
 * per-solve cost is the network inputs and one forward pass. */
int gmres_spai_infer_with(gmres_handle h, spai_handle net, const void* params, size_t param_bytes, float* m_out);

#ifdef __cplusplus
}
#endif

#endif /* SPAI_H_ */
