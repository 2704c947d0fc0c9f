/*
 * hqr_oracle.c -- plain, slow, sequential FP64 reference of the in-place
 * Householder QR least-squares path.
 *
 * TEST INFRASTRUCTURE ONLY: called by the tests, by the smoke check and by
 * the CPU-baseline leg of the benchmark.  It is built with -ffp-contract=off
 * (no fused multiply-add), shares no code with the HIP library, and does no
 * blocking, reordering or fusion beyond what the definitions below state.
 *
 * What it follows:
 *   - Householder mathematics: paper Section 2.2, Alg. 1 (pivot vector x,
 *     reflected value, reflector vector u = x - s e_0, W = I - 2uu^T/|u|^2).
 *   - In-place storage and the two row-level kernels: paper Section 3, Alg. 2
 *     (update_pivot_row returns the pair (up, b); update_trailing_non_pivot_row
 *     applies it to one trailing vector) and Alg. 3 (the pair is kept in the
 *     global up/b arrays; an undefined reflector is skipped).
 *   - Applying Q^T without forming Q: paper Section 1 (stored reflectors are
 *     reused to apply Q or Q^T), with Q = H_0 H_1 ... so Q^T b applies the
 *     reflectors in ascending order.
 *   - Back-substitution on R: paper abstract and Section 6.
 *
 * Readings where the paper is loose (listed in the design notes as well):
 *   - Sign: the printed alpha/u formulas of Alg. 1 are garbled; this code
 *     takes s = -sgn(x_0) ||x|| with sgn(0) = +1 and u = x - s e_0 (no
 *     cancellation in u_0 = up).
 *   - Identity reflector: when the part of x below the pivot is exactly zero
 *     (this includes the last column of a square matrix), up = 0, H = I and
 *     the pivot stays as it is (Alg. 3 "undefined -> continue").
 *   - Norm: scaled by max |x_i| before squaring.
 *   - Singular R: the back-substitution reports the smallest k with
 *     R[k][k] == 0 (info = k+1) and leaves its right-hand side untouched.
 *
 * Parity: pinned (closed-form worked examples, library R and tau, exact
 * rational normal equations on tiny inputs, Householder invariants).
 */
#include "hqr_oracle.h"

#include <math.h>
#include <stddef.h>
#include <stdlib.h>

#define AT(M, i, j, ld) ((M)[(size_t)(i) + (size_t)(j) * (size_t)(ld)])

double oracle_norm2(int64_t len, const double *x)
{
    double c = 0.0;
    for (int64_t i = 0; i < len; ++i) {
        double a = fabs(x[i]);
        if (a > c) c = a;
    }
    if (c == 0.0) {
        /* all zero, or NaN entries that never compared greater */
        double s = 0.0;
        for (int64_t i = 0; i < len; ++i) s += x[i] * x[i];
        return s == 0.0 ? 0.0 : sqrt(s);
    }
    double s = 0.0;
    for (int64_t i = 0; i < len; ++i) {
        double t = x[i] / c;
        s += t * t;
    }
    return c * sqrt(s);
}

/*
 * update_pivot_row (Alg. 2 / Alg. 3): generate reflector k from
 * x = A[k:m, k].  Writes R[k][k] = s into A[k][k] and the leading component
 * up = x_0 - s into *up_k; the tail A[k+1:m, k] is left unchanged and is the
 * rest of the reflector vector.  Returns 0 for the identity (skipped)
 * reflector, 1 otherwise.
 */
static int update_pivot_row(int64_t m, int64_t k, double *A, int64_t lda,
                            double *up_k)
{
    int tail_nonzero = 0;
    for (int64_t i = k + 1; i < m; ++i) {
        if (AT(A, i, k, lda) != 0.0) { /* NaN != 0 counts as nonzero */
            tail_nonzero = 1;
            break;
        }
    }
    if (!tail_nonzero) {
        *up_k = 0.0;
        return 0;
    }
    double nu = oracle_norm2(m - k, &AT(A, k, k, lda));
    double x0 = AT(A, k, k, lda);
    double s = (x0 >= 0.0) ? -nu : nu;
    *up_k = x0 - s;
    AT(A, k, k, lda) = s;
    return 1;
}

/*
 * update_trailing_non_pivot_row (Alg. 2 / Alg. 4): apply H_k to the vector y
 * (rows k..m-1 are touched).  With v = (up, A[k+1:m, k]) and b = up * s:
 *   w = (up * y_k + sum_{i>k} A[i][k] y_i) / b   (ascending i),
 *   y_k += w * up,  y_i += w * A[i][k]  (i > k).
 */
static void update_trailing(int64_t m, int64_t k, const double *A, int64_t lda,
                            double up, double s, double *y)
{
    double b = up * s;
    double w = up * y[k];
    for (int64_t i = k + 1; i < m; ++i) w += AT(A, i, k, lda) * y[i];
    w = w / b;
    y[k] += w * up;
    for (int64_t i = k + 1; i < m; ++i) y[i] += w * AT(A, i, k, lda);
}

int oracle_qr_factor(int64_t m, int64_t n, double *A, int64_t lda, double *up)
{
    if (m < 0) return -1;
    if (n < 0 || n > m) return -2;
    if (lda < (m > 1 ? m : 1)) return -4;
    if (n == 0) return 0;
    if (!A) return -3;
    if (!up) return -5;
    for (int64_t k = 0; k < n; ++k) {
        if (!update_pivot_row(m, k, A, lda, &up[k])) continue;
        double s = AT(A, k, k, lda);
        for (int64_t j = k + 1; j < n; ++j)
            update_trailing(m, k, A, lda, up[k], s, &AT(A, 0, j, lda));
    }
    return 0;
}

/*
 * The paper's multi-threaded "barrier" schedule (Section 3.2): for each
 * pivot k, one thread generates reflector k, all threads wait, then the
 * trailing columns are shared among the threads and each applies reflector
 * k to its columns, and all threads wait again before pivot k+1.  Every
 * column sees exactly the arithmetic of oracle_qr_factor in the same order,
 * so the result is bitwise the sequential one; only the wall time differs.
 * Used to time the paper's own CPU baseline; never a parity reference.
 */
int oracle_qr_factor_barrier(int64_t m, int64_t n, double *A, int64_t lda,
                             double *up, int nthreads)
{
    if (m < 0) return -1;
    if (n < 0 || n > m) return -2;
    if (lda < (m > 1 ? m : 1)) return -4;
    if (nthreads < 1) return -6;
    if (n == 0) return 0;
    if (!A) return -3;
    if (!up) return -5;
    int reflect = 0;
#pragma omp parallel num_threads(nthreads)
    {
        for (int64_t k = 0; k < n; ++k) {
#pragma omp single
            reflect = update_pivot_row(m, k, A, lda, &up[k]);
            /* implicit barrier after the single construct; every thread
             * reaches the loop's barrier, skipped reflector or not, so no
             * thread's next `single` can overwrite `reflect` before all have
             * read it */
#pragma omp for schedule(static)
            for (int64_t j = k + 1; j < n; ++j)
                if (reflect) update_trailing(m, k, A, lda, up[k], AT(A, k, k, lda), &AT(A, 0, j, lda));
            /* implicit barrier after the loop */
        }
    }
    return 0;
}

static int check_apply(int64_t m, int64_t n, int64_t nrhs, const double *A,
                       int64_t lda, const double *up, const double *B,
                       int64_t ldb)
{
    if (m < 0) return -1;
    if (n < 0 || n > m) return -2;
    if (nrhs < 0) return -3;
    if (lda < (m > 1 ? m : 1)) return -5;
    if (ldb < (m > 1 ? m : 1)) return -8;
    if (n > 0 && nrhs > 0) {
        if (!A) return -4;
        if (!up) return -6;
        if (!B) return -7;
    }
    return 0;
}

int oracle_apply_qt(int64_t m, int64_t n, int64_t nrhs, const double *A,
                    int64_t lda, const double *up, double *B, int64_t ldb)
{
    int e = check_apply(m, n, nrhs, A, lda, up, B, ldb);
    if (e) return e;
    for (int64_t c = 0; c < nrhs; ++c)
        for (int64_t k = 0; k < n; ++k)
            if (up[k] != 0.0)
                update_trailing(m, k, A, lda, up[k], AT(A, k, k, lda),
                                &AT(B, 0, c, ldb));
    return 0;
}

int oracle_apply_q(int64_t m, int64_t n, int64_t nrhs, const double *A,
                   int64_t lda, const double *up, double *B, int64_t ldb)
{
    int e = check_apply(m, n, nrhs, A, lda, up, B, ldb);
    if (e) return e;
    for (int64_t c = 0; c < nrhs; ++c)
        for (int64_t k = n - 1; k >= 0; --k)
            if (up[k] != 0.0)
                update_trailing(m, k, A, lda, up[k], AT(A, k, k, lda),
                                &AT(B, 0, c, ldb));
    return 0;
}

static int first_zero_diag(int64_t n, const double *A, int64_t lda)
{
    for (int64_t k = 0; k < n; ++k)
        if (AT(A, k, k, lda) == 0.0) return (int)(k + 1);
    return 0;
}

int oracle_backsolve(int64_t n, int64_t nrhs, const double *A, int64_t lda,
                     double *B, int64_t ldb, int *info)
{
    if (n < 0) return -1;
    if (nrhs < 0) return -2;
    if (lda < (n > 1 ? n : 1)) return -4;
    if (ldb < (n > 1 ? n : 1)) return -6;
    if (!info) return -7;
    *info = 0;
    if (n == 0 || nrhs == 0) return 0;
    if (!A) return -3;
    if (!B) return -5;
    *info = first_zero_diag(n, A, lda);
    if (*info) return 0;
    for (int64_t c = 0; c < nrhs; ++c) {
        double *x = &AT(B, 0, c, ldb);
        for (int64_t i = n - 1; i >= 0; --i) {
            double t = x[i];
            for (int64_t j = i + 1; j < n; ++j) t -= AT(A, i, j, lda) * x[j];
            x[i] = t / AT(A, i, i, lda);
        }
    }
    return 0;
}

int oracle_backsolve_t(int64_t n, int64_t nrhs, const double *A, int64_t lda,
                       double *B, int64_t ldb, int *info)
{
    if (n < 0) return -1;
    if (nrhs < 0) return -2;
    if (lda < (n > 1 ? n : 1)) return -4;
    if (ldb < (n > 1 ? n : 1)) return -6;
    if (!info) return -7;
    *info = 0;
    if (n == 0 || nrhs == 0) return 0;
    if (!A) return -3;
    if (!B) return -5;
    *info = first_zero_diag(n, A, lda);
    if (*info) return 0;
    for (int64_t c = 0; c < nrhs; ++c) {
        double *z = &AT(B, 0, c, ldb);
        for (int64_t i = 0; i < n; ++i) {
            double t = z[i];
            for (int64_t j = 0; j < i; ++j) t -= AT(A, j, i, lda) * z[j];
            z[i] = t / AT(A, i, i, lda);
        }
    }
    return 0;
}

int oracle_lsq_solve(int64_t m, int64_t n, int64_t nrhs, double *A, int64_t lda,
                     double *up, double *B, int64_t ldb, double *resnorm,
                     int *info)
{
    if (!info) return -10;
    *info = 0;
    int e = oracle_qr_factor(m, n, A, lda, up);
    if (e) return e;
    e = oracle_apply_qt(m, n, nrhs, A, lda, up, B, ldb);
    if (e) return e;
    if (resnorm)
        for (int64_t c = 0; c < nrhs; ++c)
            resnorm[c] = oracle_norm2(m - n, &AT(B, n, c, ldb));
    return oracle_backsolve(n, nrhs, A, lda, B, ldb, info);
}

/*
 * Augmented-system correction (Bjorck's refinement of least-squares
 * solutions): the system [[I, A], [A^T, 0]] [r; x] = [b; 0] is corrected with
 * residuals f = b - r - A x and g = -A^T r formed in long double, and the
 * correction solved with the existing factors:
 *   d = Q^T f,  R^T z = g,  R dx = d[0:n] - z,  dr = Q [z; d[n:m]].
 */
int oracle_lsq_refine_ext(int64_t m, int64_t n, const double *A0, int64_t lda0,
                          const double *Af, int64_t ldaf, const double *up,
                          const double *b, double *x, double *r, int steps)
{
    if (m < 0) return -1;
    if (n < 0 || n > m) return -2;
    if (lda0 < (m > 1 ? m : 1)) return -4;
    if (ldaf < (m > 1 ? m : 1)) return -6;
    if (steps < 0) return -11;
    if (n == 0) return 0;
    double *f = (double *)malloc(sizeof(double) * (size_t)m);
    double *g = (double *)malloc(sizeof(double) * (size_t)n);
    if (!f || !g) {
        free(f);
        free(g);
        return -100;
    }
    int info = 0;
    /* initial residual r = b - A0 x in long double */
    for (int64_t i = 0; i < m; ++i) {
        long double t = (long double)b[i];
        for (int64_t j = 0; j < n; ++j)
            t -= (long double)AT(A0, i, j, lda0) * (long double)x[j];
        r[i] = (double)t;
    }
    for (int it = 0; it < steps; ++it) {
        for (int64_t i = 0; i < m; ++i) {
            long double t = (long double)b[i] - (long double)r[i];
            for (int64_t j = 0; j < n; ++j)
                t -= (long double)AT(A0, i, j, lda0) * (long double)x[j];
            f[i] = (double)t;
        }
        for (int64_t j = 0; j < n; ++j) {
            long double t = 0.0L;
            for (int64_t i = 0; i < m; ++i)
                t -= (long double)AT(A0, i, j, lda0) * (long double)r[i];
            g[j] = (double)t;
        }
        oracle_apply_qt(m, n, 1, Af, ldaf, up, f, m);    /* f <- d = Q^T f */
        oracle_backsolve_t(n, 1, Af, ldaf, g, n, &info); /* g <- z */
        if (info) break;
        for (int64_t j = 0; j < n; ++j) {
            double zj = g[j];
            g[j] = f[j] - zj; /* d1 - z */
            f[j] = zj;        /* [z; d2] */
        }
        oracle_backsolve(n, 1, Af, ldaf, g, n, &info); /* g <- dx */
        if (info) break;
        oracle_apply_q(m, n, 1, Af, ldaf, up, f, m); /* f <- dr */
        for (int64_t j = 0; j < n; ++j) x[j] += g[j];
        for (int64_t i = 0; i < m; ++i) r[i] += f[i];
    }
    free(f);
    free(g);
    return info ? (int)info : 0;
}

/*
 * Equality-constrained least squares, min ||A x - b|| subject to C x = d
 * (A m x n, C p x n, p <= n), by the null-space method (Golub and Van Loan,
 * Matrix Computations, Section 6.2) built from the routines above:
 *   1. C^T = Q [R; 0]              (the in-place Householder QR of C^T)
 *   2. R^T y1 = d                  (forward substitution)
 *   3. A Q = (Q^T A^T)^T           (Q^T applied to the columns of A^T)
 *   4. b1 = b - (A Q)[:, 0:p] y1
 *   5. y2 = argmin ||(A Q)[:, p:n] y2 - b1||   (the least-squares solve above)
 *   6. x = Q [y1; y2]
 * Every x with C x = d is x = Q [y1; y2] for some y2, so step 5 minimizes
 * over exactly the feasible set.  x (n) is the output; A, C, b, d are left
 * unchanged.  info: 0; k+1 (k < p) when R_kk == 0 (C rank deficient);
 * p + k + 1 when the reduced problem's R_kk == 0.  Returns 0 or -i.
 * SLSQP's least-squares subproblem is of this form with the linearized
 * equality constraints (paper, Section 1).
 */
int oracle_lse_solve(int64_t m, int64_t n, int64_t p, const double *A,
                     int64_t lda, const double *C, int64_t ldc,
                     const double *b, const double *d, double *x, int *info)
{
    if (m < 0) return -1;
    if (n < 0) return -2;
    if (p < 0 || p > n) return -3;
    if (lda < (m > 1 ? m : 1)) return -5;
    if (ldc < (p > 1 ? p : 1)) return -7;
    if (m < n - p) return -1;
    if (!info) return -11;
    *info = 0;
    if (n == 0) return 0;
    if (!x) return -10;
    int64_t nr = n - p;
    double *Ct = (double *)malloc(sizeof(double) * (size_t)n * (size_t)(p > 0 ? p : 1));
    double *upc = (double *)malloc(sizeof(double) * (size_t)(p > 0 ? p : 1));
    double *At = (double *)malloc(sizeof(double) * (size_t)n * (size_t)(m > 0 ? m : 1));
    double *Ar = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1) * (size_t)(nr > 0 ? nr : 1));
    double *upr = (double *)malloc(sizeof(double) * (size_t)(nr > 0 ? nr : 1));
    double *b1 = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    double *res = (double *)malloc(sizeof(double) * 1);
    int rc = 0;
    if (!Ct || !upc || !At || !Ar || !upr || !b1 || !res) {
        rc = -100;
        goto done;
    }
    /* 1. C^T (n x p) and its QR */
    for (int64_t i = 0; i < p; ++i)
        for (int64_t j = 0; j < n; ++j) AT(Ct, j, i, n) = AT(C, i, j, ldc);
    if (p > 0) oracle_qr_factor(n, p, Ct, n, upc);
    /* 2. R^T y1 = d, y1 in x[0:p] */
    for (int64_t i = 0; i < p; ++i) x[i] = d[i];
    if (p > 0) {
        int inf = 0;
        oracle_backsolve_t(p, 1, Ct, n, x, p > 1 ? p : 1, &inf);
        if (inf) {
            *info = inf;
            goto done;
        }
    }
    /* 3. A^T (n x m), then Q^T A^T */
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) AT(At, j, i, n) = AT(A, i, j, lda);
    if (p > 0) oracle_apply_qt(n, p, m, Ct, n, upc, At, n);
    /* 4. b1 = b - (A Q)[:, 0:p] y1, with (A Q)[i][j] = At[j][i] */
    for (int64_t i = 0; i < m; ++i) {
        double t = b[i];
        for (int64_t j = 0; j < p; ++j) t -= AT(At, j, i, n) * x[j];
        b1[i] = t;
    }
    /* 5. the reduced least-squares problem on (A Q)[:, p:n] */
    for (int64_t j = 0; j < nr; ++j)
        for (int64_t i = 0; i < m; ++i) AT(Ar, i, j, m) = AT(At, p + j, i, n);
    if (nr > 0) {
        int inf = 0;
        oracle_lsq_solve(m, nr, 1, Ar, m > 1 ? m : 1, upr, b1, m > 1 ? m : 1, res, &inf);
        if (inf) {
            *info = (int)p + inf;
            goto done;
        }
        for (int64_t j = 0; j < nr; ++j) x[p + j] = b1[j];
    }
    /* 6. x = Q [y1; y2] */
    if (p > 0) oracle_apply_q(n, p, 1, Ct, n, upc, x, n);
done:
    free(Ct);
    free(upc);
    free(At);
    free(Ar);
    free(upr);
    free(b1);
    free(res);
    return rc;
}

/*
 * Cholesky factorization S = R^T R of a symmetric positive definite n x n
 * matrix (upper triangle of S read, R written over it; the strict lower
 * triangle is left as it is), the textbook column-by-column definition:
 *   R[j][j] = sqrt(S[j][j] - sum_{k<j} R[k][j]^2),
 *   R[j][i] = (S[j][i] - sum_{k<j} R[k][j] R[k][i]) / R[j][j]   (i > j),
 * sums in ascending k.  info = j+1 at the first pivot that is not positive
 * (S not positive definite; R is then partial), else 0.  SLSQP keeps its
 * Hessian approximation as such a factorization (paper, Section 6 names
 * Cholesky as a further kernel of the solver).
 */
int oracle_cholesky(int64_t n, double *S, int64_t lds, int *info)
{
    if (n < 0) return -1;
    if (lds < (n > 1 ? n : 1)) return -3;
    if (!info) return -4;
    *info = 0;
    if (n == 0) return 0;
    if (!S) return -2;
    for (int64_t j = 0; j < n; ++j) {
        double t = AT(S, j, j, lds);
        for (int64_t k = 0; k < j; ++k) t -= AT(S, k, j, lds) * AT(S, k, j, lds);
        if (!(t > 0.0)) {
            *info = (int)(j + 1);
            return 0;
        }
        double rjj = sqrt(t);
        AT(S, j, j, lds) = rjj;
        for (int64_t i = j + 1; i < n; ++i) {
            double u = AT(S, j, i, lds);
            for (int64_t k = 0; k < j; ++k) u -= AT(S, k, j, lds) * AT(S, k, i, lds);
            AT(S, j, i, lds) = u / rjj;
        }
    }
    return 0;
}

/*
 * Rank-one update of a triangular factor: R (n x n upper, ldr) becomes R'
 * with R'^T R' = R^T R + v v^T, by one plane rotation per row (Golub and
 * Van Loan, Matrix Computations, Section 6.5.4): for k = 0..n-1,
 *   r = sgn(R[k][k]) hypot(R[k][k], v[k])  (sgn(0) = +1, keeping the sign
 *       convention of R's diagonal), c = R[k][k] / r, s = v[k] / r
 *       (c = 1, s = 0 when r = 0),
 *   R[k][k] = r; for j > k: (R[k][j], v[j]) <- (c R[k][j] + s v[j],
 *                                               -s R[k][j] + c v[j]).
 * The same operation updates the R of a QR factorization when a row v^T is
 * appended to the matrix.  v is overwritten (it ends as zeros).
 */
int oracle_chol_update(int64_t n, double *R, int64_t ldr, double *v)
{
    if (n < 0) return -1;
    if (ldr < (n > 1 ? n : 1)) return -3;
    if (n == 0) return 0;
    if (!R) return -2;
    if (!v) return -4;
    for (int64_t k = 0; k < n; ++k) {
        double rkk = AT(R, k, k, ldr);
        double h = hypot(rkk, v[k]);
        double r = (rkk >= 0.0) ? h : -h;
        double c = 1.0, s = 0.0;
        if (r != 0.0) {
            c = rkk / r;
            s = v[k] / r;
        }
        AT(R, k, k, ldr) = r;
        v[k] = 0.0;
        for (int64_t j = k + 1; j < n; ++j) {
            double a = AT(R, k, j, ldr), b = v[j];
            AT(R, k, j, ldr) = c * a + s * b;
            v[j] = -s * a + c * b;
        }
    }
    return 0;
}
