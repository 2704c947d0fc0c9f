/*
 * hqr_oracle.h -- plain sequential FP64 reference of the in-place Householder
 * QR least-squares path (TEST INFRASTRUCTURE ONLY).
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may call this code.  The product library never links it, and it
 * shares no source with the HIP path.
 *
 * Storage contract (paper, Section 3, Alg. 2, and the stored pair of Alg. 3):
 *   column-major, A is m x n with m >= n, leading dimension lda >= max(1, m).
 *   After oracle_qr_factor:
 *     - the upper triangle of A (diagonal included) holds R;
 *     - below the diagonal, column k holds the tail of reflector k exactly as
 *       it was when the reflector was generated;
 *     - up[k] holds the reflector's leading component (the paper's
 *       global_up_array); up[k] == 0 means H_k = I;
 *     - b_k = up[k] * R[k][k] is derived, never stored (global_b_array).
 *   H_k = I + v_k v_k^T / b_k, with v_k = (0, .., 0, up[k], A[k+1:m, k]).
 */
#ifndef HQR_ORACLE_H
#define HQR_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Factor A in place.  Returns 0, or -i when argument i is invalid. */
int oracle_qr_factor(int64_t m, int64_t n, double *A, int64_t lda, double *up);

/* The same factorization under the paper's barrier schedule on nthreads
 * threads (one barrier after each reflector's generation and after its
 * application); bitwise the result of oracle_qr_factor.  For timing the
 * paper's CPU baseline only. */
int oracle_qr_factor_barrier(int64_t m, int64_t n, double *A, int64_t lda,
                             double *up, int nthreads);

/* B (m x nrhs) <- Q^T B = H_{n-1} ... H_0 B (reflectors in ascending order). */
int oracle_apply_qt(int64_t m, int64_t n, int64_t nrhs, const double *A,
                    int64_t lda, const double *up, double *B, int64_t ldb);

/* B (m x nrhs) <- Q B = H_0 ... H_{n-1} B (reflectors in descending order). */
int oracle_apply_q(int64_t m, int64_t n, int64_t nrhs, const double *A,
                   int64_t lda, const double *up, double *B, int64_t ldb);

/* B[0:n] <- R^{-1} B[0:n].  If some R[k][k] == 0, *info = smallest such k+1
 * and B is left untouched; otherwise *info = 0. */
int oracle_backsolve(int64_t n, int64_t nrhs, const double *A, int64_t lda,
                     double *B, int64_t ldb, int *info);

/* B[0:n] <- R^{-T} B[0:n] (forward substitution with R^T). */
int oracle_backsolve_t(int64_t n, int64_t nrhs, const double *A, int64_t lda,
                       double *B, int64_t ldb, int *info);

/* Scaled Euclidean norm of x[0:len]. */
double oracle_norm2(int64_t len, const double *x);

/* Factor, apply Q^T, record resnorm[j] = ||(Q^T B)[n:m, j]||, back-substitute.
 * x ends in B[0:n].  resnorm may be NULL. */
int oracle_lsq_solve(int64_t m, int64_t n, int64_t nrhs, double *A, int64_t lda,
                     double *up, double *B, int64_t ldb, double *resnorm,
                     int *info);

/* Extended-precision reference: refine the least-squares solution x (n) and
 * residual r (m) of min ||b - A0 x|| by `steps` augmented-system correction
 * steps whose residuals are accumulated in long double.  Af/up is the
 * oracle's factorization of A0.  Returns 0 or a negative argument error. */
int oracle_lsq_refine_ext(int64_t m, int64_t n, const double *A0, int64_t lda0,
                          const double *Af, int64_t ldaf, const double *up,
                          const double *b, double *x, double *r, int steps);

/* Equality-constrained least squares min ||A x - b|| s.t. C x = d
 * (C p x n, p <= n, m >= n - p) by the null-space method on the routines
 * above.  x: n outputs.  info: 0, k+1 for a zero pivot of C's R, p+k+1 for
 * a zero pivot of the reduced problem.  Returns 0 or -i. */
int oracle_lse_solve(int64_t m, int64_t n, int64_t p, const double *A,
                     int64_t lda, const double *C, int64_t ldc,
                     const double *b, const double *d, double *x, int *info);

/* Cholesky S = R^T R (upper triangle of S overwritten by R).  info = j+1
 * at the first non-positive pivot, else 0.  Returns 0 or -i. */
int oracle_cholesky(int64_t n, double *S, int64_t lds, int *info);

/* R'^T R' = R^T R + v v^T by plane rotations (v overwritten).  Returns 0
 * or -i. */
int oracle_chol_update(int64_t n, double *R, int64_t ldr, double *v);

#ifdef __cplusplus
}
#endif

#endif
