// hqr_cqr.hpp -- panel factorization with a constant number of grid-wide
// steps: CholeskyQR2 followed by Householder reconstruction.
//
// For a panel A_p (m_p x bw, bw <= 64) the Householder reflectors of the
// paper's per-column loop (Section 3, Alg. 2 / Alg. 3, restated for a block
// of alpha pivots) are recovered without a reduction per column:
//   1. G = A_p^T A_p, R1 = chol(G)                    (pass 1)
//   2. Q1 = A_p R1^{-1}, G2 = Q1^T Q1, R2 = chol(G2)  (pass 2), R = R2 R1
//   3. Q = A_p R^{-1} has orthonormal columns.  Householder QR of Q gives the
//      same reflectors as Householder QR of A_p (each pivot vector of Q is a
//      positive multiple of the corresponding pivot vector of A_p, and a
//      reflector with the sign rule R_kk = -sgn(x_0)||x|| does not change
//      when x is scaled by a positive factor).  For orthonormal Q that
//      factorization is an LU factorization without pivoting of Q - [S; 0],
//      S = diag(s_k), s_k = -sgn(pivot of step k) with sgn(0) = +1:
//          Q - [S; 0] = Y U,  T_Y = -U S Y_1^{-T},  R_house = S R,
//      where Y is unit lower trapezoidal (the normalized reflectors), Y_1 its
//      top bw x bw block and H_0 ... H_{bw-1} = I - Y T_Y Y^T.
//   4. Convert to the stored form: tau_k = T_Y[k][k], up_k = -tau_k R_kk,
//      stored tail = Y[k+1:, k] * up_k, and T for v = up*y:
//      T_V[i][j] = T_Y[i][j] / (up_i up_j).
//   The bottom rows of Y are Q_bot U^{-1} = A_bot (R^{-1} U^{-1}).
//
// Panels for which this is not the stored factorization of the one-reflector
// loop, or not accurate, go to an exact one-workgroup Householder panel
// (panel_exact_kernel) instead:
//   - a column whose part below the pivot row is exactly zero (the loop then
//     keeps H_k = I; this includes an empty tail when m_p == bw);
//   - a Cholesky pivot whose squared ratio to the column's norm falls below
//     CQR_RATIO (conditioning beyond what two CholeskyQR passes repair, or
//     rank deficiency).
// The decision is taken on the device; `flag` then makes the remaining
// CholeskyQR kernels of the panel return at once and the exact kernel run.
#pragma once

#include "hqr_device.hpp"
#include "hqr_blocked.hpp"

namespace hqr {

constexpr int CQR_ROWS = 128;          // rows per workgroup in the Gram kernels
constexpr double CQR_RATIO = 1e-15;    // smallest accepted pivot^2 / G_kk
constexpr int LD65 = NB + 1;

// ------------------------------------------------------------------ helpers
// out = A * B for 64 x 64 LDS matrices (row-major, stride 65), FP64 MFMA.
// 256 threads; wave w computes row tile w.  out must not alias A or B.
HQR_DEV void mm64(double (*out)[LD65], const double (*A)[LD65], const double (*B)[LD65], int lane, int w)
{
    f64x4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int k0 = 0; k0 < NB; k0 += 4) {
        const int kr = k0 + (lane >> 4);
        const double a = A[16 * w + (lane & 15)][kr];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, B[kr][16 * t + (lane & 15)], acc[t], 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) out[16 * w + 4 * r + (lane >> 4)][16 * t + (lane & 15)] = acc[t][r];
}

// Sum over the four lanes 4c..4c+3 of a column group (same wave).
HQR_DEV double quad_sum(double v)
{
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    return v;
}

// Inverse of the upper-triangular n x n block of U into X (upper, zeros
// below, identity beyond n).  Column j belongs to lanes 4j..4j+3 of one wave
// (256 threads); lane q keeps X[q + 4t][j], t < 16, in registers.  Rows are
// produced bottom-up; the 16 entries of U's row each lane needs are loaded
// unconditionally (so the loads pipeline), products are selected, not
// branched, and the four partial sums are added across the lanes.
HQR_DEV void inv_upper64(double (*X)[LD65], const double (*U)[LD65], int n, int tid, double *dinv)
{
    const int j = tid >> 2, q = tid & 3;
    if (tid < NB) dinv[tid] = (tid < n) ? 1.0 / U[tid][tid] : 1.0;
    __syncthreads();
    double x[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) x[t] = (q + 4 * t == j) ? dinv[j] : 0.0;
    if (j < n) {
        for (int i = j - 1; i >= 0; --i) {
            double u[16];
#pragma unroll
            for (int t = 0; t < 16; ++t) u[t] = U[i][q + 4 * t];
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int t = 0; t < 16; t += 2) {
                const int l0 = q + 4 * t, l1 = l0 + 4;
                s0 += (l0 > i && l0 <= j) ? u[t] * x[t] : 0.0;
                s1 += (l1 > i && l1 <= j) ? u[t + 1] * x[t + 1] : 0.0;
            }
            const double xi = -quad_sum(s0 + s1) * dinv[i];
#pragma unroll
            for (int t = 0; t < 16; ++t) x[t] = (q + 4 * t == i) ? xi : x[t];
        }
    }
#pragma unroll
    for (int t = 0; t < 16; ++t) X[q + 4 * t][j] = x[t];
    __syncthreads();
}

// Inverse of the unit lower triangle (strict lower entries of L, unit
// diagonal implied) into X (lower, unit diagonal, zeros above); same layout,
// rows produced top-down.
HQR_DEV void inv_unit_lower64(double (*X)[LD65], const double (*L)[LD65], int n, int tid)
{
    const int j = tid >> 2, q = tid & 3;
    double x[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) x[t] = (q + 4 * t == j) ? 1.0 : 0.0;
    if (j < n) {
        for (int i = j + 1; i < n; ++i) {
            double u[16];
#pragma unroll
            for (int t = 0; t < 16; ++t) u[t] = L[i][q + 4 * t];
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int t = 0; t < 16; t += 2) {
                const int l0 = q + 4 * t, l1 = l0 + 4;
                s0 += (l0 >= j && l0 < i) ? u[t] * x[t] : 0.0;
                s1 += (l1 >= j && l1 < i) ? u[t + 1] * x[t + 1] : 0.0;
            }
            const double xi = -quad_sum(s0 + s1);
#pragma unroll
            for (int t = 0; t < 16; ++t) x[t] = (q + 4 * t == i) ? xi : x[t];
        }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 16; ++t) X[q + 4 * t][j] = x[t];
    __syncthreads();
}

// Register of a 16-entry array picked by a runtime index (select chain, so
// the array stays in registers).
HQR_DEV double pick16(const double (&v)[16], int t)
{
    double r = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) r = (q == t) ? v[q] : r;
    return r;
}

// In-place upper Cholesky G = R^T R of the n x n block (R in the upper part,
// zeros below, identity beyond n).  Thread (column j = tid & 63, row group
// rg = tid >> 6) keeps G[rg + 4t][j], t < 16, in registers.  Row k is
// broadcast through a double-buffered LDS row written by its owners after
// their step-(k-1) update, so each step needs one barrier.  *bad reports a
// pivot^2 below ratio * G_kk.
HQR_DEV void chol64(double (*G)[LD65], int n, int tid, double ratio, double *gdiag, double *rdiag, int *bad,
                    double (*rowbuf)[NB])
{
    const int j = tid & 63, rg = tid >> 6;
    double g[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) g[t] = G[rg + 4 * t][j];
    if (tid < NB) gdiag[tid] = (tid < n) ? G[tid][tid] : 1.0;
    if (tid == 0) *bad = 0;
    if (rg == 0) rowbuf[0][j] = g[0];
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        const double *rk = rowbuf[k & 1];
        const double piv = rk[k];
        const double inv = 1.0 / piv;
        const double rkj = rk[j];
        const double rkk = sqrt(fmax(piv, 0.0));
        double rkv[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) rkv[t] = rk[rg + 4 * t];
        const double coef = rkj * inv;
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const int i = rg + 4 * t;
            g[t] = (i > k && i <= j && j < n) ? g[t] - rkv[t] * coef : g[t];
        }
        // row k of R
        if (rg == (k & 3)) G[k][j] = (j > k && j < n) ? rkj / rkk : ((j == k) ? rkk : 0.0);
        if (tid == 0) {
            rdiag[k] = rkk;
            if (!(piv > ratio * gdiag[k])) *bad = 1;
        }
        const int kn = k + 1;
        if (kn < n && rg == (kn & 3)) rowbuf[kn & 1][j] = pick16(g, kn >> 2);
        __syncthreads();
    }
    for (int idx = tid; idx < NB * NB; idx += 256) {
        const int i = idx / NB, c = idx % NB;
        if (i > c || i >= n || c >= n) G[i][c] = (i == c && i >= n) ? 1.0 : 0.0;
    }
    __syncthreads();
}

// In place: M (n x n, top block of Q) becomes L (strict lower, unit diagonal
// implied) and U (upper) of the LU factorization without pivoting of
// M - S, with s_k = -sgn(pivot k) (sgn(0) = +1) chosen at step k.  Same
// register layout as chol64; column k reaches the wave's lanes by readlane.
HQR_DEV void lu_sign64(double (*M)[LD65], int n, int tid, double *sgn, double *udiag, double (*rowbuf)[NB])
{
    const int j = tid & 63, rg = tid >> 6;
    double mv[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) mv[t] = M[rg + 4 * t][j];
    if (rg == 0) rowbuf[0][j] = mv[0];
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        const double *rk = rowbuf[k & 1];
        const double q = rk[k];
        const double s = (q >= 0.0) ? -1.0 : 1.0;
        const double ukk = q - s;
        const double ukj = rk[j] / ukk;
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const int i = rg + 4 * t;
            const double lik = readlane_f64(mv[t], k); // column k, row i
            mv[t] = (i > k && i < n && j > k && j < n) ? mv[t] - lik * ukj : mv[t];
        }
        if (tid == 0) {
            sgn[k] = s;
            udiag[k] = ukk;
        }
        const int kn = k + 1;
        if (kn < n && rg == (kn & 3)) rowbuf[kn & 1][j] = pick16(mv, kn >> 2);
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const int i = rg + 4 * t;
        double v = mv[t];
        if (i < n && j < n) {
            if (i > j) v = v / udiag[j];
            else if (i == j) v = udiag[j];
        }
        M[i][j] = v;
    }
    __syncthreads();
}

// ------------------------------------------------------------ Gram kernel
struct CqrArgs {
    double *A;
    int64_t lda;
    int64_t m;
    int c0, bw;
    int pass;                 // 1: G of A_p (and zero-tail masks); 2: G of A_p R1^{-1}
    int ngroups;              // workgroups (row chunks of CQR_ROWS rows)
    double *gpart;            // [ngroups][NB][NB]
    unsigned long long *mask; // [ngroups] bit k: column k nonzero below its pivot row
    const double *r1inv;      // [NB][NB] row-major (pass 2)
    int *flag;                // nonzero: this panel takes the exact path
};

__global__ void __launch_bounds__(256) cqr_gram_kernel(CqrArgs p)
{
    __shared__ double X[NB][LD65];   // [row][col] chunk of 64 rows
    __shared__ double Y[NB][LD65];
    __shared__ double Ri[NB][LD65];
    __shared__ unsigned long long msk;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (p.pass == 2 && *((volatile int *)p.flag)) return;
    const int64_t r_begin = (int64_t)p.c0 + (int64_t)blockIdx.x * CQR_ROWS;
    const int64_t r_end = min<int64_t>(p.m, r_begin + CQR_ROWS);
    if (tid == 0) msk = 0ull;
    if (p.pass == 2)
        for (int idx = tid; idx < NB * NB; idx += 256) Ri[idx / NB][idx % NB] = p.r1inv[idx];

    f64x4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
    unsigned long long mymask = 0ull;

    for (int64_t r0 = r_begin; r0 < r_end; r0 += 64) {
        __syncthreads();
        for (int idx = tid; idx < 64 * NB; idx += 256) {
            const int c = idx / 64, r = idx % 64;
            const int64_t gi = r0 + r;
            double v = 0.0;
            if (gi < r_end && c < p.bw) {
                v = HQR_AT(p.A, gi, p.c0 + c, p.lda);
                if (p.pass == 1 && gi > (int64_t)p.c0 + c && v != 0.0) mymask |= (1ull << c);
            }
            X[r][c] = v;
        }
        __syncthreads();
        double (*Z)[LD65] = X;
        if (p.pass == 2) {
            mm64(Y, X, Ri, lane, w);
            __syncthreads();
            Z = Y;
        }
        // acc += Z^T Z : wave w owns output rows [16w, 16w+16)
#pragma unroll 4
        for (int k0 = 0; k0 < 64; k0 += 4) {
            const int kr = k0 + (lane >> 4);
            const double a = Z[kr][16 * w + (lane & 15)];
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Z[kr][16 * t + (lane & 15)], acc[t], 0, 0, 0);
        }
    }
    double *out = p.gpart + (size_t)blockIdx.x * NB * NB;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) out[(16 * w + 4 * r + (lane >> 4)) * NB + 16 * t + (lane & 15)] = acc[t][r];
    if (p.pass == 1) {
        if (mymask) atomicOr(&msk, mymask);
        __syncthreads();
        if (tid == 0) p.mask[blockIdx.x] = msk;
    }
}

// ----------------------------------------------- partial Gram reduction
// G[e] = sum_q gpart[q][e] in a fixed order: 64 workgroups of 256 threads;
// thread (entry e, quarter g4) sums q = g4, g4+4, ..; quarters added 0..3.
// Workgroup 0 also ORs the zero-tail masks.
struct GredArgs {
    const double *gpart;
    int ngroups;
    double *G;
    const unsigned long long *mask;
    unsigned long long *mask_all;
    int with_mask;
    const int *flag;
};

__global__ void __launch_bounds__(256) gram_reduce_kernel(GredArgs p)
{
    __shared__ double part[4][64];
    const int tid = threadIdx.x, e = blockIdx.x * 64 + (tid & 63), g4 = tid >> 6;
    if (*((volatile int *)p.flag)) return;
    double s = 0.0;
#pragma unroll 4
    for (int q = g4; q < p.ngroups; q += 4) s += p.gpart[(size_t)q * NB * NB + e];
    part[g4][tid & 63] = s;
    __syncthreads();
    if (tid < 64) p.G[e] = ((part[0][tid] + part[1][tid]) + part[2][tid]) + part[3][tid];
    if (p.with_mask && blockIdx.x == 0 && tid == 64) {
        unsigned long long all = 0ull;
        for (int q = 0; q < p.ngroups; ++q) all |= p.mask[q];
        *p.mask_all = all;
    }
}

// --------------------------------------------------------- Cholesky kernel
struct CholArgs {
    double *A;
    int64_t lda;
    int64_t m;
    int c0, bw;
    int pass;
    const double *G;                    // reduced Gram
    const unsigned long long *mask_all; // ORed zero-tail masks (pass 1)
    double *r1;         // [NB][NB]  (pass 1 out, pass 2 in)
    double *r1inv;      // [NB][NB]  (pass 1 out, pass 2 in)
    double *winv;       // [NB][NB]  (pass 2 out) R^{-1} U^{-1} diag(up)
    double *T;          // [NB][NB]  (pass 2 out) T for the stored vectors
    double *up;         // global up (pass 2 out)
    int *flag;
    long long *tstamp;  // optional per-phase timestamps (thread 0), may be null
};

// One workgroup, 256 threads.
__global__ void __launch_bounds__(256) cqr_chol_kernel(CholArgs p)
{
    __shared__ double M0[NB][LD65];
    __shared__ double M1[NB][LD65];
    __shared__ double M2[NB][LD65];
    __shared__ double M3[NB][LD65];
    __shared__ double gdiag[NB], rdiag[NB], sgn[NB], upv[NB], rh[NB];
    __shared__ double rowbuf[2][NB];
    __shared__ int bad;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int bw = p.bw;
    if (p.pass == 2 && *((volatile int *)p.flag)) return;
    int tsi = 0;
#define HQR_TS()                                                                 \
    do {                                                                         \
        if (p.tstamp && tid == 0) p.tstamp[tsi] = (long long)wall_clock64();     \
        ++tsi;                                                                   \
    } while (0)
    HQR_TS();

    for (int idx = tid; idx < NB * NB; idx += 256) {
        const int i = idx / NB, j = idx % NB;
        M0[i][j] = (i < bw && j < bw) ? p.G[idx] : 0.0;
    }
    int structural = 0;
    if (p.pass == 1 && tid == 0) {
        const unsigned long long all = *p.mask_all;
        const unsigned long long need = (bw == 64) ? ~0ull : ((1ull << bw) - 1ull);
        structural = ((all & need) != need);
    }
    __syncthreads();
    HQR_TS();
    chol64(M0, bw, tid, CQR_RATIO, gdiag, rdiag, &bad, rowbuf);
    HQR_TS();
    if (tid == 0 && (bad || structural)) atomicExch(p.flag, 1);
    __syncthreads();
    if (bad || __hip_atomic_load(p.flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;

    if (p.pass == 1) {
        inv_upper64(M1, M0, bw, tid, gdiag);
        for (int idx = tid; idx < NB * NB; idx += 256) {
            p.r1[idx] = M0[idx / NB][idx % NB];
            p.r1inv[idx] = M1[idx / NB][idx % NB];
        }
        return;
    }

    // ---- pass 2: M0 = R2
    inv_upper64(M1, M0, bw, tid, gdiag);                // M1 = R2^{-1}
    HQR_TS();
    for (int idx = tid; idx < NB * NB; idx += 256) M2[idx / NB][idx % NB] = p.r1inv[idx];
    __syncthreads();
    mm64(M3, M2, M1, lane, w);                          // M3 = R^{-1} = R1^{-1} R2^{-1}
    __syncthreads();
    for (int idx = tid; idx < NB * NB; idx += 256) M2[idx / NB][idx % NB] = p.r1[idx];
    __syncthreads();
    mm64(M1, M0, M2, lane, w);                          // M1 = R = R2 R1
    __syncthreads();
    // Q_top = A_top R^{-1}
    for (int idx = tid; idx < NB * NB; idx += 256) {
        const int c = idx / NB, r = idx % NB;
        M2[r][c] = (r < bw && c < bw) ? HQR_AT(p.A, (int64_t)p.c0 + r, p.c0 + c, p.lda) : 0.0;
    }
    __syncthreads();
    mm64(M0, M2, M3, lane, w);                          // M0 = Q_top
    __syncthreads();
    HQR_TS();
    // modified LU of Q_top - S (in place in M0)
    lu_sign64(M0, bw, tid, sgn, rdiag, rowbuf);
    HQR_TS();
    // R_house = S R: write the upper triangle of the panel's top block
    for (int idx = tid; idx < bw * bw; idx += 256) {
        const int c = idx / bw, r = idx % bw;
        if (r <= c) HQR_AT(p.A, (int64_t)p.c0 + r, p.c0 + c, p.lda) = sgn[r] * M1[r][c];
    }
    if (tid < bw) {
        const double rkk = sgn[tid] * M1[tid][tid];
        const double tau = -M0[tid][tid] * sgn[tid];      // = 1 + |pivot|
        rh[tid] = rkk;
        upv[tid] = -tau * rkk;
    }
    __syncthreads();
    // W^{-1} = R^{-1} U^{-1}, scaled by up per column
    {
        // M2 = U^{-1} from the upper part of M0 (diagonal = U_kk)
        for (int idx = tid; idx < NB * NB; idx += 256) {
            const int i = idx / NB, j = idx % NB;
            M1[i][j] = (i <= j && i < bw && j < bw) ? M0[i][j] : ((i == j) ? 1.0 : 0.0);
        }
        __syncthreads();
        inv_upper64(M2, M1, NB, tid, gdiag);
        HQR_TS();
        mm64(M1, M3, M2, lane, w);                      // M1 = R^{-1} U^{-1}
        __syncthreads();
        for (int idx = tid; idx < NB * NB; idx += 256) {
            const int i = idx / NB, j = idx % NB;
            p.winv[idx] = (j < bw) ? M1[i][j] * upv[j] : 0.0;
        }
    }
    // T_Y = -(U S) L^{-T};  T_V = T_Y / (up_i up_j)
    __syncthreads();
    HQR_TS();
    inv_unit_lower64(M2, M0, bw, tid);                  // M2 = L^{-1}
    HQR_TS();
    for (int idx = tid; idx < NB * NB; idx += 256) {
        const int i = idx / NB, l = idx % NB;
        M1[i][l] = (i <= l && l < bw) ? M0[i][l] * sgn[l] : 0.0; // U S
        M3[l][i] = M2[i][l];                                     // L^{-T}
    }
    __syncthreads();
    mm64(M2, M1, M3, lane, w);
    __syncthreads();
    for (int idx = tid; idx < NB * NB; idx += 256) {
        const int i = idx / NB, j = idx % NB;
        p.T[idx] = (i <= j && j < bw) ? -M2[i][j] / (upv[i] * upv[j]) : 0.0;
    }
    // stored tails of the top block: L[i][j] * up_j (strict lower)
    for (int idx = tid; idx < bw * bw; idx += 256) {
        const int c = idx / bw, r = idx % bw;
        if (r > c) HQR_AT(p.A, (int64_t)p.c0 + r, p.c0 + c, p.lda) = M0[r][c] * upv[c];
    }
    if (tid < bw) p.up[p.c0 + tid] = upv[tid];
    HQR_TS();
#undef HQR_TS
}

// ------------------------------------------ bottom rows: Y_bot * diag(up)
struct FinArgs {
    double *A;
    int64_t lda;
    int64_t m;
    int c0, bw;
    const double *winv;
    const int *flag;
};

__global__ void __launch_bounds__(256) cqr_finish_kernel(FinArgs p)
{
    __shared__ double X[NB][LD65];
    __shared__ double Wi[NB][LD65];
    __shared__ double Y[NB][LD65];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (*((volatile int *)p.flag)) return;
    const int64_t r0 = (int64_t)p.c0 + p.bw + (int64_t)blockIdx.x * 64;
    for (int idx = tid; idx < NB * NB; idx += 256) Wi[idx / NB][idx % NB] = p.winv[idx];
    for (int idx = tid; idx < 64 * NB; idx += 256) {
        const int c = idx / 64, r = idx % 64;
        const int64_t gi = r0 + r;
        X[r][c] = (gi < p.m && c < p.bw) ? HQR_AT(p.A, gi, p.c0 + c, p.lda) : 0.0;
    }
    __syncthreads();
    mm64(Y, X, Wi, lane, w);
    __syncthreads();
    for (int idx = tid; idx < 64 * NB; idx += 256) {
        const int c = idx / 64, r = idx % 64;
        const int64_t gi = r0 + r;
        if (gi < p.m && c < p.bw) HQR_AT(p.A, gi, p.c0 + c, p.lda) = Y[r][c];
    }
}

// ------------------------------------------------- exact one-workgroup panel
// The one-reflector-at-a-time loop on the panel (same arithmetic as the
// per-pivot launches), streamed from global memory by one workgroup of 1024
// threads, followed by T from V^T V.  Runs only when `flag` is set.
struct ExactArgs {
    double *A;
    int64_t lda;
    int64_t m;
    int c0, bw;
    double *up;
    double *T;
    const int *flag;
};

__global__ void __launch_bounds__(1024) panel_exact_kernel(ExactArgs p)
{
    __shared__ double red[16][PW];
    __shared__ double wsh[NB];
    __shared__ double sc[4];
    __shared__ double G[NB][LD65];
    __shared__ double Ts[NB][LD65];
    __shared__ double tau[NB], tmp[NB];
    const int tid = threadIdx.x, j = tid & 63, g = tid >> 6; // 16 row groups
    if (!*((volatile int *)p.flag)) return;
    const int bw = p.bw, c0 = p.c0;
    const int64_t m = p.m;
    for (int k = 0; k < bw; ++k) {
        const int64_t pr = (int64_t)c0 + k;
        // partial dots x . a_j over rows > pr, plus max|x| and #nonzero
        double acc = 0.0, mx = 0.0, nz = 0.0;
        for (int64_t i = pr + 1 + g; i < m; i += 16) {
            const double xi = HQR_AT(p.A, i, c0 + k, p.lda);
            if (j >= k && j < bw) acc += xi * HQR_AT(p.A, i, c0 + j, p.lda);
            mx = fmax(mx, fabs(xi));
            nz += (xi != 0.0) ? 1.0 : 0.0;
        }
        red[g][j] = acc;
        if (j == 0) {
            red[g][NB] = mx;
            red[g][NB + 1] = nz;
        }
        __syncthreads();
        if (tid < PW) {
            double v = 0.0;
            if (tid == NB) {
                for (int q = 0; q < 16; ++q) v = fmax(v, red[q][NB]);
            } else {
                for (int q = 0; q < 16; ++q) v += red[q][tid];
            }
            red[0][tid] = v;
        }
        __syncthreads();
        if (tid == 0) {
            const double x0 = HQR_AT(p.A, pr, c0 + k, p.lda);
            double upk, sk;
            if (red[0][NB + 1] == 0.0) {
                upk = 0.0;
                sk = x0;
            } else {
                const double c = fmax(fabs(x0), red[0][NB]);
                double nu;
                if (norm_fast_path_ok(c)) {
                    nu = sqrt(x0 * x0 + red[0][k]);
                } else {
                    double t = 0.0;
                    for (int64_t i = pr + 1; i < m; ++i) {
                        const double y = HQR_AT(p.A, i, c0 + k, p.lda) / c;
                        t += y * y;
                    }
                    const double x0c = x0 / c;
                    nu = c * sqrt(x0c * x0c + t);
                }
                sk = (x0 >= 0.0) ? -nu : nu;
                upk = x0 - sk;
            }
            sc[0] = upk;
            sc[1] = sk;
            p.up[c0 + k] = upk;
        }
        __syncthreads();
        const double upk = sc[0], sk = sc[1];
        if (upk != 0.0) {
            const double bk = upk * sk;
            if (tid < NB) wsh[tid] = (tid > k && tid < bw) ? (upk * HQR_AT(p.A, pr, c0 + tid, p.lda) + red[0][tid]) / bk : 0.0;
            __syncthreads();
            if (j > k && j < bw) {
                const double wj = wsh[j];
                for (int64_t i = pr + g; i < m; i += 16) {
                    const double v = (i == pr) ? upk : HQR_AT(p.A, i, c0 + k, p.lda);
                    HQR_AT(p.A, i, c0 + j, p.lda) += wj * v;
                }
            }
        }
        __syncthreads();
        if (tid == 0) HQR_AT(p.A, pr, c0 + k, p.lda) = sk;
        __syncthreads();
    }
    // G = V^T V (V masked: up on the diagonal), then T by the recurrence
    for (int e = tid; e < NB * NB; e += 1024) {
        Ts[e / NB][e % NB] = 0.0;
        const int a = e / NB, b = e % NB;
        if (a > b) continue;
        double s = 0.0;
        if (b < bw) {
            const int64_t lo = (int64_t)c0 + b;
            s = p.up[c0 + b] * ((a == b) ? p.up[c0 + a] : HQR_AT(p.A, lo, c0 + a, p.lda));
            for (int64_t i = lo + 1; i < m; ++i) s += HQR_AT(p.A, i, c0 + a, p.lda) * HQR_AT(p.A, i, c0 + b, p.lda);
        }
        G[a][b] = s;
        G[b][a] = s;
    }
    if (tid < NB) {
        double t = 0.0;
        if (tid < bw) {
            const double u = p.up[c0 + tid];
            t = (u == 0.0) ? 0.0 : -1.0 / (u * HQR_AT(p.A, (int64_t)c0 + tid, c0 + tid, p.lda));
        }
        tau[tid] = t;
    }
    __syncthreads();
    for (int jj = 0; jj < bw; ++jj) {
        if (tid < jj) {
            double s = 0.0;
            for (int l = tid; l < jj; ++l) s += Ts[tid][l] * G[l][jj];
            tmp[tid] = s;
        }
        __syncthreads();
        if (tid < jj) Ts[tid][jj] = -tau[jj] * tmp[tid];
        if (tid == jj) Ts[jj][jj] = tau[jj];
        __syncthreads();
    }
    for (int e = tid; e < NB * NB; e += 1024) p.T[e] = Ts[e / NB][e % NB];
}

} // namespace hqr
