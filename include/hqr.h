/*
 * hqr.h -- C ABI of libhqr: in-place Householder QR least squares on MI355X.
 *
 * The operation (Chatterjee et al., "Efficient Task Graph Scheduling for
 * Parallel QR Factorization in SLSQP"):
 *   - qr_factor transforms A into upper-triangular form in place, one
 *     reflector per column (Section 3, Alg. 2), keeping each reflector's
 *     leading component `up` and its tail below the diagonal (the pair
 *     (up, b) of Alg. 3, with b = up * R[k][k]);
 *   - qr_apply_qt and qr_apply_q apply Q^T or Q to right-hand sides with
 *     those stored reflectors, without forming Q (Section 1); qr_form_q
 *     forms leading columns of Q explicitly;
 *   - qr_backsolve back-substitutes with R (abstract; Section 6 names the
 *     triangular solve as a kernel of the same solver);
 *   - qr_lsq_solve chains the three; qr_lsq_refine solves again with a
 *     stored factorization and refines against the original matrix.
 *
 * Conventions shared by every entry point:
 *   - Matrices are FP64, column-major, leading dimension >= max(1, rows).
 *   - Every matrix/vector pointer is a DEVICE pointer (HBM of the current
 *     HIP device).  Arrays of shapes in the batched call are HOST arrays.
 *   - Calls are asynchronous on `stream` (0 = the null stream); outputs are
 *     valid after the stream is synchronized.  Calls never synchronize the
 *     host except where stated.
 *   - Calls on different streams may run concurrently from different host
 *     threads: the library keeps its per-stream state (the look-ahead's side
 *     stream and events, the batched descriptor staging buffer) per caller
 *     stream.  Calls on one stream from several host threads must be
 *     serialized by the caller.  The tuning and profiling calls change
 *     process-global state and are not thread-safe.
 *   - The caller owns every buffer.  `work`/`lwork` is an optional device
 *     workspace of at least hqr_workspace_size() bytes; with work == NULL the
 *     library takes a stream-ordered allocation (hipMallocAsync) and frees it
 *     on the same stream before returning.
 *   - Return value (host): 0 on success; -i when argument i (1-based) is
 *     invalid, checked before any work is enqueued; or one of the HQR_E*
 *     codes below.  Data-dependent outcomes go to the DEVICE int `*info`.
 *   - Reflector storage after qr_factor: R in the upper triangle (diagonal
 *     included); below the diagonal, column k holds reflector k's tail as it
 *     was when the reflector was generated; up[k] its leading component.
 *     H_k = I + v v^T / b_k with v = (0..0, up[k], A[k+1:m, k]) and
 *     b_k = up[k] * R[k][k]; up[k] == 0 means H_k = I (the tail below the
 *     pivot was exactly zero, which includes the last column when m == n).
 *     R[k][k] = -sgn(x_0) ||x|| with sgn(0) = +1, x = A[k:m, k] at step k.
 *   - NaN/Inf inputs are not checked; they propagate.
 */
#ifndef HQR_H
#define HQR_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Host status codes (besides 0 and -i). */
#define HQR_ENOMEM   (-1001) /* workspace too small or allocation failed     */
#define HQR_EDEVICE  (-1002) /* a HIP call failed                             */
#define HQR_ENOTSUP  (-1003) /* shape/option combination not supported        */

/* Device info codes (besides 0 and k+1 for a zero R[k][k]). */
#define HQR_INFO_TIMEOUT (-2001) /* a bounded cross-workgroup wait expired;
                                     outputs are invalid                   */
#define HQR_INFO_NOCONV  (1 << 29) /* refinement did not converge: the FP64
                                      fallback was used and its result
                                      returned (OR-ed into info together
                                      with any k+1), or, with
                                      HQR_OPT_NO_FALLBACK, x is the last
                                      refinement iterate                   */

/* Precision of the trailing-update contractions. */
#define HQR_PREC_FP64  0 /* everything FP64                                  */
#define HQR_PREC_MIXED 1 /* trailing update on FP32 MFMA with FP32
                            accumulation, subtracted into FP64 storage;
                            reflector generation, R's diagonal, Q^T b and
                            the back-substitution stay FP64, then
                            refinement of the semi-normal equations with
                            FP64 residuals of the original matrix          */

/* hqr_opts.flags */
#define HQR_OPT_NO_FALLBACK 1 /* refinement (mixed qr_lsq_solve, qr_lsq_refine):
                                 never wait on the host; when some
                                 right-hand side does not converge,
                                 HQR_INFO_NOCONV is ORed into info on the
                                 device and x is the last iterate (no FP64
                                 fallback: the caller decides)           */
#define HQR_OPT_TSQR_PANEL  2 /* blocked path (FP64 and mixed qr_lsq_solve):
                                 every 64-column panel by TSQR (a reduction
                                 tree of row-block Householder QRs) with
                                 Householder reconstruction, stable at any
                                 panel conditioning; the default CholeskyQR2
                                 panel hands a panel whose Gram pivots fall
                                 below 1e-15 of its column norms to the exact
                                 one-workgroup loop instead (Section 6 names
                                 tiled and communication-avoiding QR as the
                                 way forward).  A caller's work area must
                                 then have hqr_workspace_size_opts() bytes
                                 (HQR_PANEL=tsqr in the environment selects
                                 the TSQR panel for every call, and
                                 hqr_workspace_size then includes it)    */

typedef struct hqr_opts {
    int precision;   /* HQR_PREC_FP64 or HQR_PREC_MIXED                      */
    double tol;      /* refinement: converged when ||dx|| <= tol * ||x||
                        (<= 0: 1e-13)                                        */
    int max_iter;    /* refinement step limit (< 0: 10)                       */
    int flags;       /* HQR_OPT_* bits (0: none)                              */
} hqr_opts;

/* Bytes of device workspace the calls below need for an m x n problem with
 * nrhs right-hand sides at the given precision.  Returns a negative status on
 * invalid arguments. */
int64_t hqr_workspace_size(int64_t m, int64_t n, int64_t nrhs, int precision);

/* The same for qr_lsq_solve with options: opt->precision and the buffers of
 * the TSQR tree when opt->flags has HQR_OPT_TSQR_PANEL (opt NULL: FP64, no
 * flags).  Returns a negative status on invalid arguments. */
int64_t hqr_workspace_size_opts(int64_t m, int64_t n, int64_t nrhs, const hqr_opts *opt);

/* In-place factorization (Alg. 2 with the storage of Alg. 3).
 *   m >= n >= 0; A: m x n (lda >= max(1,m)), overwritten by R and the
 *   reflector tails; up: n doubles (out); info: one device int (out):
 *   0, or HQR_INFO_TIMEOUT. */
int qr_factor(int64_t m, int64_t n, double *A, int64_t lda, double *up,
              void *work, int64_t lwork, int *info, hipStream_t stream);

/* B (m x nrhs, ldb >= max(1,m)) <- Q^T B = H_{n-1} ... H_0 B, using the
 * output of qr_factor.  Rows 0..n-1 of B then hold the coefficients for the
 * back-substitution, rows n..m-1 the residual components. */
int qr_apply_qt(int64_t m, int64_t n, int64_t nrhs, const double *A,
                int64_t lda, const double *up, double *B, int64_t ldb,
                void *work, int64_t lwork, hipStream_t stream);

/* B (m x nrhs, ldb >= max(1,m)) <- Q B = H_0 H_1 ... H_{n-1} B, using the
 * output of qr_factor: the stored reflectors applied last to first (Section
 * 1: SLSQP applies Q as well as Q^T from the stored reflectors, never forming
 * Q).  Same arguments, workspace and errors as qr_apply_qt. */
int qr_apply_q(int64_t m, int64_t n, int64_t nrhs, const double *A,
               int64_t lda, const double *up, double *B, int64_t ldb,
               void *work, int64_t lwork, hipStream_t stream);

/* Explicit Q: Q (m x k, 0 <= k <= m, ldq >= max(1,m), device) <- the leading
 * k columns of Q = H_0 ... H_{n-1} from qr_factor's output (k = n: the thin
 * Q with A = Q[:, 0:n] R; k = m: the full orthogonal Q).  Q is overwritten
 * (its input is ignored).  Workspace: hqr_workspace_size(m, n, k, FP64)
 * bytes, or NULL.  Returns 0 or -i (argument i invalid: m < 0, n outside
 * [0, m], k outside [0, m], lda < m, ldq < m, null pointers). */
int qr_form_q(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda,
              const double *up, double *Q, int64_t ldq, void *work,
              int64_t lwork, hipStream_t stream);

/* B[0:n] (n x nrhs, ldb >= max(1,n)) <- R^{-1} B[0:n], R = upper triangle
 * of A (lda >= max(1,n)).  If some R[k][k] == 0, *info = smallest such k+1
 * and B is left unchanged; otherwise *info = 0. */
int qr_backsolve(int64_t n, int64_t nrhs, const double *A, int64_t lda,
                 double *B, int64_t ldb, int *info, hipStream_t stream);

/* Least squares min ||B[:,j] - A x_j|| for every column j:
 * factor A in place, B <- Q^T B, resnorm[j] <- ||(Q^T B)[n:m, j]|| (if
 * resnorm != NULL; device array of nrhs doubles), then back-substitute so
 * x_j ends in B[0:n, j].
 *   opt == NULL or opt->precision == HQR_PREC_FP64: plain FP64.
 *   opt->precision == HQR_PREC_MIXED: A_orig must point to an unmodified
 *     FP64 copy of A (same m x n, leading dimension lda_orig) used for the
 *     FP64 residuals of the refinement; resnorm is then ||b - A x||.
 *   info: device int (0, k+1 for a zero R[k][k], HQR_INFO_* flags);
 *   iters: device int or NULL, refinement steps taken (0 for FP64).
 *   Refinement (opt->tol, opt->max_iter) of every right-hand side: a column
 *   is converged when ||dx|| <= tol ||x||, or when ||dx|| stops halving at or
 *   below 3e-11 ||x|| (the rounding floor); corrections that stop halving
 *   above that floor twice in a row, or max_iter steps without convergence,
 *   mean no convergence.  A converged column's x is left as it is.
 *   The mixed form synchronizes `stream` with the host once, after the
 *   refinement, to read whether every column converged; without
 *   convergence the problem is solved again by the FP64 path from the
 *   restored inputs (A_orig, the original B) and HQR_INFO_NOCONV is ORed
 *   into the info that solve reports.  With HQR_OPT_NO_FALLBACK in
 *   opt->flags nothing waits on the host and there is no fallback (see
 *   there).  qr_lsq_refine behaves the same way. */
int qr_lsq_solve(int64_t m, int64_t n, int64_t nrhs, double *A, int64_t lda,
                 double *up, double *B, int64_t ldb, double *resnorm,
                 const hqr_opts *opt, const double *A_orig, int64_t lda_orig,
                 void *work, int64_t lwork, int *info, int *iters,
                 hipStream_t stream);

/* Equality-constrained least squares: x = argmin ||A x - b|| subject to
 * C x = d (A m x n, C p x n, 0 <= p <= n, m >= n - p), the form of SLSQP's
 * least-squares subproblem with its linearized equality constraints
 * (Section 1), solved by the null-space method on this library's QR:
 *   C^T = Q [R; 0] (qr_factor of C^T), R^T y1 = d, A Q = (Q^T A^T)^T,
 *   y2 = argmin ||(A Q)[:, p:n] y2 - (b - (A Q)[:, 0:p] y1)|| (the
 *   least-squares solve above), x = Q [y1; y2].
 * A (lda >= max(1,m)) is overwritten by A Q and then by the reduced
 * problem's factorization; b (m) is overwritten; C (ldc >= max(1,p)) and d
 * (p) are read only; x (n, device) is the output.  Requires rank(C) = p and
 * the reduced problem of full column rank: info (device int) = k+1 when
 * C^T's R_kk == 0, p + k + 1 when the reduced problem's R_kk == 0, else 0.
 * Workspace: hqr_lse_workspace_size(m, n, p) bytes, or NULL.  Returns 0 or
 * -i (argument i invalid; -3 also when m < n - p). */
int64_t hqr_lse_workspace_size(int64_t m, int64_t n, int64_t p);
int qr_lse_solve(int64_t m, int64_t n, int64_t p, double *A, int64_t lda,
                 double *C, int64_t ldc, double *b, const double *d,
                 double *x, void *work, int64_t lwork, int *info,
                 hipStream_t stream);

/* Cholesky factorization S = R^T R of a symmetric positive definite n x n
 * matrix (SLSQP keeps its Hessian approximation in this factored form;
 * Section 6 names Cholesky as a further kernel of the solver).  Only the
 * upper triangle of S (lds >= max(1,n), device) is read and it is
 * overwritten by R (positive diagonal); the strict lower triangle is not
 * touched.  Right-looking by 64-column blocks on FP64 MFMA.  info (device
 * int): 0, or j+1 for the first pivot that is not positive (S not positive
 * definite; R is then partial).  Workspace: 32768 bytes, or NULL.  Returns
 * 0 or -i. */
int hqr_cholesky(int64_t n, double *S, int64_t lds, void *work, int64_t lwork,
                 int *info, hipStream_t stream);

/* Rank-one update of a triangular factor: R (n x n upper, ldr >= max(1,n),
 * device) becomes R' with R'^T R' = R^T R + v v^T, by one plane rotation per
 * row, keeping the sign of each diagonal entry.  For a Cholesky factor this
 * is the factor of the updated matrix; for the R of a QR factorization
 * (qr_factor's upper triangle, read in place with lda) it is the R of the
 * matrix with the row v^T appended.  v (n, device) is overwritten.  One
 * workgroup; n <= 4096 (else HQR_ENOTSUP).  Returns 0 or -i. */
int hqr_chol_update(int64_t n, double *R, int64_t ldr, double *v,
                    hipStream_t stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): qr_lsq_solve in FP64
 * (opt == NULL) that allocates nothing.  Its workspace is a device array of
 * HQR_STATIC_SCRATCH_BYTES inside the library, one per GPU, held until the
 * process ends; problems needing more (hqr_workspace_size(m, n, nrhs,
 * HQR_PREC_FP64) > HQR_STATIC_SCRATCH_BYTES; 8192 x 4096 with up to 8
 * right-hand sides fits) return HQR_ENOMEM before anything is enqueued.
 * The look-ahead side stream is not used (everything runs on `stream`), so
 * nothing is created either.  Arguments, outputs and info as qr_lsq_solve.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (on different streams, or from different threads) race and must be
 * serialized by the caller. */
#define HQR_STATIC_SCRATCH_BYTES (80ll << 20)
int qr_lsq_solve_static(int64_t m, int64_t n, int64_t nrhs, double *A,
                        int64_t lda, double *up, double *B, int64_t ldb,
                        double *resnorm, int *info, hipStream_t stream);

/* Solve again with a stored factorization (qr_factor's output, from either
 * precision, e.g. a previous mixed-precision qr_lsq_solve), then refine:
 * B (m x nrhs) <- Q^T B, back-substitute, and correct x with the
 * semi-normal equations using FP64 residuals of A_orig, the unmodified FP64
 * A (r = b - A_orig x, A_orig^T r, R^T z = A_orig^T r, R dx = z), as the
 * mixed form of qr_lsq_solve does (opt->tol, opt->max_iter; opt may be
 * NULL).  x ends in B[0:n]; resnorm (device, nrhs doubles, or NULL) gets
 * ||b - A_orig x||.  A and up are never modified.  Convergence rule, host
 * synchronization and HQR_OPT_NO_FALLBACK as for the mixed qr_lsq_solve;
 * the FP64 fallback works on a copy of A_orig (a stream-ordered allocation
 * of m*n doubles).  A zero R[k][k] gives info = k+1.  iters (device int or
 * NULL): steps taken (max_iter without convergence). */
int qr_lsq_refine(int64_t m, int64_t n, int64_t nrhs, const double *A,
                  int64_t lda, const double *up, double *B, int64_t ldb,
                  double *resnorm, const hqr_opts *opt, const double *A_orig,
                  int64_t lda_orig, void *work, int64_t lwork, int *info,
                  int *iters, hipStream_t stream);

/* Many independent least-squares problems of uneven size in ONE persistent
 * launch (a batch of the per-iteration subproblems an SLSQP-like solver
 * produces).  Arrays of length `count` are HOST arrays; A[i], up[i], B[i],
 * resnorm[i] are device pointers.  Instance i: m[i] x n[i] (n[i] <= m[i] <=
 * 4096), nrhs[i] right-hand sides (n[i] + nrhs[i] <= 2048); A[i] is factored
 * in place exactly as by qr_factor's one-reflector-at-a-time definition,
 * B[i] becomes (Q^T B) with x in rows 0..n-1, resnorm[i] (if resnorm and
 * resnorm[i] are non-NULL, nrhs[i] doubles) gets ||(Q^T B)[n:m]||, and
 * info[i] (device int array of `count`) gets 0 or the smallest k+1 with
 * R[k][k] == 0.  Instances are scheduled longest-first; each result depends
 * only on its own instance, never on the rest of the batch.
 * Workspace: hqr_batched_workspace_size(count) bytes (or NULL). */
int64_t hqr_batched_workspace_size(int count);
int qr_lsq_solve_batched(int count, const int64_t *m, const int64_t *n,
                         const int64_t *nrhs, double *const *A,
                         const int64_t *lda, double *const *up,
                         double *const *B, const int64_t *ldb,
                         double *const *resnorm, int *info, void *work,
                         int64_t lwork, hipStream_t stream);

/* The same persistent launch over a mix of new and already-factored
 * problems (factor reuse across successive solves): factored[i] (HOST int
 * array) nonzero means A[i] and up[i] already hold qr_factor's output for
 * instance i, which is then only applied to B[i] (Q^T B, residual norms,
 * back-substitution; A[i], up[i] untouched); zero means factor as in
 * qr_lsq_solve_batched.  Other arguments as there. */
int qr_lsq_batched_mixed(int count, const int64_t *m, const int64_t *n,
                         const int64_t *nrhs, double *const *A,
                         const int64_t *lda, double *const *up,
                         double *const *B, const int64_t *ldb,
                         double *const *resnorm, const int *factored,
                         int *info, void *work, int64_t lwork,
                         hipStream_t stream);

/* Tuning rules that choose kernels (the autotuner's output is loaded through
 * these).  A rule applies to problems with m_lo <= m <= m_hi and
 * n_lo <= n <= n_hi at `precision`; the first rule added that matches wins.
 *   op HQR_TUNE_SINGLE: path of one qr_factor / qr_apply_qt / qr_lsq_solve
 *     problem: choice -1 = the blocked multi-kernel path, choice i >= 0 = the
 *     one-workgroup kernel variant i (ignored where it cannot hold the
 *     problem).  Without a rule, problems with n <= 128 that a variant holds
 *     use the smallest such variant.
 *   op HQR_TUNE_BATCHED: variant i of a batched launch, matched on the
 *     largest m and n among the batch's instances that the one-workgroup
 *     kernel takes (m <= 1024, n * nrhs within the smallest staging area);
 *     only variants with 256 threads qualify (they share one arithmetic, so
 *     results do not depend on the batch); without a rule, the smallest such
 *     variant that holds the largest m.
 *   op HQR_TUNE_OCCUPANCY: workgroups per CU of the batched launch (choice
 *     1..8, capped by what the variant's LDS allows), matched like
 *     HQR_TUNE_BATCHED; without a rule, min(2, that cap).
 * Host-side state, process-global, not thread-safe.  Returns 0 or -i. */
#define HQR_TUNE_SINGLE    0
#define HQR_TUNE_BATCHED   1
#define HQR_TUNE_OCCUPANCY 2
int hqr_tune_set(int op, int64_t m_lo, int64_t m_hi, int64_t n_lo,
                 int64_t n_hi, int precision, int choice);
int hqr_tune_clear(void);
/* Number of one-workgroup variants, and the name of variant i ("wgNTxQM"
 * or "wgNTxQMpP": NT threads holding QM rows each, so m <= NT*QM, and P
 * 16-row blocks loaded together in the trailing update, 4 when not given),
 * or NULL. */
int hqr_tune_variants(void);
const char *hqr_tune_variant_name(int i);

/* Kernel timing for measurement.  hqr_profile_begin() starts recording: every
 * kernel the library launches afterwards (on any stream) is bracketed by a
 * pair of HIP events on that stream, grouped by kernel class.
 * hqr_profile_end() stops recording, synchronizes on the recorded events and
 * adds each class's summed elapsed milliseconds and launch count into
 * ms[0..nclass) and count[0..nclass) (either may be NULL).  It returns the
 * number of classes the library knows (or a negative status); class names
 * come from hqr_profile_class().  Process-global and not thread-safe; the
 * events add launch overhead, so time throughput with profiling off. */
int hqr_profile_begin(void);
int hqr_profile_end(int nclass, double *ms, int64_t *count);
const char *hqr_profile_class(int cls);

/* Text of a host status or device info code (static storage). */
const char *hqr_status_string(int status);

/* Library version string. */
const char *hqr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HQR_H */
