/*
 * gmcp_mlp.h - C ABI of the learned warm start: a per-vertex MLP
 * 9 -> 128 -> 128 -> 128 -> 3 with SiLU activations, run on the MI355X
 * matrix cores (bf16 operands, float32 accumulation), with its training
 * kernels (backward pass, mean-squared loss, Adam).  The network predicts
 * the correction d = x* - (x_t + dt v_t) of an implicit step from each
 * vertex's position, velocity and previous correction; the Newton solve
 * (gmcp_fem.h + gmcp.h) starts from x_t + dt v_t + d after the contact
 * step-bound filter, and its converged solution judges the prediction.
 *
 * Tensors are float32 device arrays.  Inputs are padded to 16 features and
 * outputs to 16 columns (zeros beyond the real 9 / 3).  Parameters are one
 * contiguous float32 array (gmcp_mlp_param_count entries):
 *   W1 [16][128], b1 [128], W2 [128][128], b2 [128], W3 [128][128], b3 [128],
 *   W4 [128][16], b4 [16];  layer l computes Z = H W + b, H' = SiLU(Z).
 * All calls enqueue on `stream` (a hipStream_t) and are deterministic.
 */
#ifndef GMCP_MLP_H
#define GMCP_MLP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

int64_t gmcp_mlp_param_count(void);

/* Scratch bytes gmcp_mlp_backward needs for a batch of B rows. */
size_t gmcp_mlp_work_bytes(int64_t B);

/* y [B][16] = MLP(x [B][16]); act [B][768] receives Z1|H1|Z2|H2|Z3|H3
 * (nullable: inference; the backward pass reads it).  One fused launch:
 * each wave runs all four layers on 32 rows with the activations in
 * registers and the weights staged once per block in LDS as bf16. */
int gmcp_mlp_forward(const float *params, const float *x, int64_t B, float *y, float *act, void *stream);

/* grad [param_count] = d(loss)/d(params) given dy [B][16] = d(loss)/dy and
 * the activations of the forward pass on the same x. */
int gmcp_mlp_backward(const float *params, const float *x, const float *act, const float *dy, int64_t B,
                      float *grad, void *work, size_t work_bytes, void *stream);

/* loss (one device float) = mean over B rows and the first n_out columns of
 * (y - t)^2; dy = its gradient (0 on the padding).  work >= 4 * ceil(16 B / 256) bytes. */
int gmcp_mlp_mse(const float *y, const float *t, int64_t B, int n_out, float *loss, float *dy, void *work,
                 size_t work_bytes, void *stream);

/* The same loss and gradient as gmcp_mlp_mse for callers that cannot
 * allocate device memory (code under HIP graph capture, tight training
 * loops, harnesses that forbid allocation): no work argument, and no
 * allocation of any kind.  Its per-block partial sums live in a static
 * device array of 4 MiB that every GPU the library runs on holds until the
 * process ends, so B is limited to gmcp_mlp_mse_noalloc_max_rows() rows
 * (larger B: GMCP_E_ARG, nothing enqueued).  `stream` must belong to the
 * current device (else GMCP_E_ARG).  All calls on one GPU share that array:
 * calls that overlap on one GPU (other streams, other threads) race. */
int gmcp_mlp_mse_noalloc(const float *y, const float *t, int64_t B, int n_out, float *loss, float *dy,
                         void *stream);

/* Largest B that gmcp_mlp_mse_noalloc accepts (host only). */
int64_t gmcp_mlp_mse_noalloc_max_rows(void);

/* One Adam step (bias-corrected, step >= 1) on n parameters. */
int gmcp_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t n, float lr, float beta1,
                  float beta2, float eps, int step, void *stream);

/* C [M][N] (ldc) = op(A) op(B) on the matrix cores, bf16 operands, float32
 * accumulation; op(A) = A^T if transA (A stored [K][M]), same for B. */
int gmcp_gemm_bf16(const float *A, int lda, int transA, const float *B, int ldb, int transB, int M, int N, int K,
                   float *C, int ldc, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GMCP_MLP_H */
