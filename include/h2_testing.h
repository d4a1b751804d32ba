/*
 * h2_testing.h -- test hooks of the MI355X H2 library (not for production use).
 *
 * They expose the batched dense primitives of the construction and the weak
 * (sibling-block) factors of the most recent h2_build on this thread, so tests
 * can compare each stage with an independent CPU computation.  All arrays are
 * host, column-major, FP64; the hooks allocate, copy, run on the null stream
 * and synchronise.  Return value: h2_status.
 */
#ifndef H2_MI355X_TESTING_H
#define H2_MI355X_TESTING_H

#include "h2.h"

#ifdef __cplusplus
extern "C" {
#endif

/* C = alpha op(A) op(B) + beta C (op = transpose when t* != 0); C in/out */
h2_status h2_test_gemm(int ta, int tb, int M, int N, int K, double alpha, const double* A, int lda,
                       const double* B, int ldb, double beta, double* C, int ldc);
/* Householder QR of A (m x n): Q (m x min(m,n)), R (min(m,n) x n); either may be NULL */
h2_status h2_test_qr(int m, int n, const double* A, double* Q, double* R);
/* tall QR, m >= n: Q (m x n) and R (n x n); mode 0: one TSQR (n <= 96);
   1: block Gram-Schmidt over 64-column panels with TSQR panels; 2: the
   kernel chosen by shape (Q and R); 3: the same, R only (Q is not written) */
h2_status h2_test_cholqr(int m, int n, const double* A, double* Q, double* R, int mode);
/* one-sided Jacobi SVD of A (m x n, m >= n): sigma (n), U (m x n), V (n x n) */
h2_status h2_test_svd(int m, int n, const double* A, double* sigma, double* U, double* V);
/* raw accumulator of one 16x16 matrix-core product (kind 0: f64 16x16x4,
   1: f32 16x16x4, 2: bf16 16x16x16) of known operands; out[lane*4 + reg]
   (256 values) -- pins the operand and result lane layouts the kernels use */
h2_status h2_test_mfma_layout(int kind, double* out);
/* out[lane] = the wave-wide sum of in[0..63] as the kernels' reduction returns
   it to each lane of one 64-lane wave (host arrays of 64 doubles) */
h2_status h2_test_wave_sum(const double* in, double* out);
/* polls a workgroup of the multi-workgroup Jacobi SVD makes before it stops
   waiting for the blocks of its round (then the call's singular values are
   NaN); negative: 0.  Restore the default with 4194304. */
void h2_test_svd_spin_limit(int polls);
/* y = A x (FP64, user order, ld n, device pointers) with the matrix-core tile
   width fixed to nt (1, 2, 4 sixteen-vector tiles per workgroup; 0: tuned) */
h2_status h2_test_gemv_tile(const h2_matrix* A, int nv, const double* x, double* y, int nt);
/* the tile width the autotuner chose for FP64 products with nv vectors on
   A's tree (0: not tuned yet) */
int h2_test_tuned_tile(const h2_matrix* A, int nv);
/* groups per far list that h2_gemv's coupling stage uses for nv vectors on A
   (1: no split) */
int h2_test_gemv_split_groups(const h2_matrix* A, int nv);
/* the one-sided Jacobi SVD for `count` matrices in one batched call: matrix i
   is m[i] x n[i] (m[i] >= n[i]); A and U are the column-major matrices stored
   one after the other, sigma the n[i] values one after the other, V the
   n[i] x n[i] factors one after the other */
h2_status h2_test_svd_batch(int count, const int* m, const int* n, const double* A, double* sigma,
                            double* U, double* V);
/* keep the weak factors of subsequent h2_build calls on this thread (1) or not (0) */
void h2_test_keep_factors(int on);
/* factors of level l of the last kept build: ranks (2^(l-1)) and F (n x K, K = max rank) */
h2_status h2_test_factors(int level, int32_t* ranks_out, int* K_out, double* F_out);

#ifdef __cplusplus
}
#endif
#endif
