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

constexpr int CQR_ROWS = 64;           // rows per workgroup in the Gram kernels
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






// ------------------------------------------- 16 x 16 blocks on MFMA
// FP64 MFMA 16x16x4 layouts: A[i][k] at lane i + 16k, B[k][j] at lane
// j + 16k, D[i][j] at lane j + 16 (i % 4), register i / 4.  A product D
// feeds the next MFMA as its B operand directly: register q is the B operand
// of the k-chunk 4q..4q+3.

// acc += MA[ar:ar+16][ac:ac+16] * MB[br:br+16][bc:bc+16]
HQR_DEV f64x4 mma_blk(f64x4 acc, const double (*MA)[LD65], int ar, int ac, const double (*MB)[LD65], int br, int bc,
                      int lane)
{
    const int i = lane & 15, kk = lane >> 4;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int k = 4 * q + kk;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(MA[ar + i][ac + k], MB[br + k][bc + i], acc, 0, 0, 0);
    }
    return acc;
}

// acc += MA[ar:ar+16][ac:ac+16] * D  (D a 16 x 16 block in D layout)
HQR_DEV f64x4 mma_blk_reg(f64x4 acc, const double (*MA)[LD65], int ar, int ac, f64x4 d, int lane)
{
    const int i = lane & 15, kk = lane >> 4;
#pragma unroll
    for (int q = 0; q < 4; ++q)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(MA[ar + i][ac + 4 * q + kk], d[q], acc, 0, 0, 0);
    return acc;
}

HQR_DEV void st_blk(double (*M)[LD65], int r0, int c0, f64x4 d, double scale, int lane)
{
#pragma unroll
    for (int r = 0; r < 4; ++r) M[r0 + 4 * r + (lane >> 4)][c0 + (lane & 15)] = scale * d[r];
}

// X = U^{-1} for the upper-triangular n x n block of U (identity beyond n;
// U's entries outside that block must be zero off the diagonal), by the 4
// waves of the workgroup: wave w inverts diagonal block w (lane j < 16
// solves for its column), then the blocks above the diagonal follow by their
// distance from it, X_ij = -X_ii sum_{k=i+1..j} U_ik X_kj, as MFMA products.
// Starts and ends with a barrier.
HQR_DEV void inv_upper64_blk(double (*X)[LD65], const double (*U)[LD65], int n, int lane, int w)
{
    __syncthreads();
    {
        const int b0 = 16 * w, j = lane & 15;
        double x[16];
#pragma unroll
        for (int i = 15; i >= 0; --i) {
            const int gi = b0 + i;
            double s = (i == j) ? 1.0 : 0.0;
#pragma unroll
            for (int l = i + 1; l < 16; ++l) s = fma(-U[gi][b0 + l], x[l], s);
            x[i] = (i > j) ? 0.0 : ((gi < n) ? s / U[gi][gi] : ((i == j) ? 1.0 : 0.0));
        }
        if (lane < 16) {
#pragma unroll
            for (int i = 0; i < 16; ++i) X[b0 + i][b0 + j] = x[i];
        }
        for (int idx = lane; idx < 16 * b0; idx += 64) X[b0 + idx / b0][idx % b0] = 0.0;
    }
    __syncthreads();
    if (w < 3) { // distance 1
        const int i = w, j = w + 1;
        f64x4 t = mma_blk(f64x4{0.0, 0.0, 0.0, 0.0}, U, 16 * i, 16 * j, X, 16 * j, 16 * j, lane);
        st_blk(X, 16 * i, 16 * j, mma_blk_reg(f64x4{0.0, 0.0, 0.0, 0.0}, X, 16 * i, 16 * i, t, lane), -1.0, lane);
    }
    __syncthreads();
    if (w < 2) { // distance 2
        const int i = w, j = w + 2;
        f64x4 t = mma_blk(f64x4{0.0, 0.0, 0.0, 0.0}, U, 16 * i, 16 * (i + 1), X, 16 * (i + 1), 16 * j, lane);
        t = mma_blk(t, U, 16 * i, 16 * j, X, 16 * j, 16 * j, lane);
        st_blk(X, 16 * i, 16 * j, mma_blk_reg(f64x4{0.0, 0.0, 0.0, 0.0}, X, 16 * i, 16 * i, t, lane), -1.0, lane);
    }
    __syncthreads();
    if (w == 0) { // distance 3
        f64x4 t = mma_blk(f64x4{0.0, 0.0, 0.0, 0.0}, U, 0, 16, X, 16, 48, lane);
        t = mma_blk(t, U, 0, 32, X, 32, 48, lane);
        t = mma_blk(t, U, 0, 48, X, 48, 48, lane);
        st_blk(X, 0, 48, mma_blk_reg(f64x4{0.0, 0.0, 0.0, 0.0}, X, 0, 0, t, lane), -1.0, lane);
    }
    __syncthreads();
}

// X = L^{-1} for the unit lower triangle whose strict lower entries are L's
// (n x n block; L's entries outside it must be zero), same scheme: diagonal
// blocks by forward substitution, then X_ij = -X_ii sum_{k=j..i-1} L_ik X_kj.
// Starts and ends with a barrier.
HQR_DEV void inv_unit_lower64_blk(double (*X)[LD65], const double (*L)[LD65], int n, int lane, int w)
{
    __syncthreads();
    {
        const int b0 = 16 * w, j = lane & 15;
        double x[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int gi = b0 + i;
            double s = (i == j) ? 1.0 : 0.0;
#pragma unroll
            for (int l = 0; l < i; ++l) s = fma(-L[gi][b0 + l], x[l], s);
            x[i] = (i < j) ? 0.0 : ((i == j) ? 1.0 : ((gi < n && b0 + j < n) ? s : 0.0));
        }
        if (lane < 16) {
#pragma unroll
            for (int i = 0; i < 16; ++i) X[b0 + i][b0 + j] = x[i];
        }
        const int c1 = b0 + 16, wid = NB - c1;
        for (int idx = lane; idx < 16 * wid; idx += 64) X[b0 + idx / wid][c1 + idx % wid] = 0.0;
    }
    __syncthreads();
    if (w < 3) { // distance 1: X_{j+1, j}
        const int j = w, i = w + 1;
        f64x4 t = mma_blk(f64x4{0.0, 0.0, 0.0, 0.0}, L, 16 * i, 16 * j, X, 16 * j, 16 * j, lane);
        st_blk(X, 16 * i, 16 * j, mma_blk_reg(f64x4{0.0, 0.0, 0.0, 0.0}, X, 16 * i, 16 * i, t, lane), -1.0, lane);
    }
    __syncthreads();
    if (w < 2) { // distance 2: X_{j+2, j}
        const int j = w, i = w + 2;
        f64x4 t = mma_blk(f64x4{0.0, 0.0, 0.0, 0.0}, L, 16 * i, 16 * j, X, 16 * j, 16 * j, lane);
        t = mma_blk(t, L, 16 * i, 16 * (j + 1), X, 16 * (j + 1), 16 * j, lane);
        st_blk(X, 16 * i, 16 * j, mma_blk_reg(f64x4{0.0, 0.0, 0.0, 0.0}, X, 16 * i, 16 * i, t, lane), -1.0, lane);
    }
    __syncthreads();
    if (w == 0) { // distance 3: X_{3, 0}
        f64x4 t = mma_blk(f64x4{0.0, 0.0, 0.0, 0.0}, L, 48, 0, X, 0, 0, lane);
        t = mma_blk(t, L, 48, 16, X, 16, 0, lane);
        t = mma_blk(t, L, 48, 32, X, 32, 0, lane);
        st_blk(X, 48, 0, mma_blk_reg(f64x4{0.0, 0.0, 0.0, 0.0}, X, 48, 48, t, lane), -1.0, lane);
    }
    __syncthreads();
}

// 16 x 16 LDS block in D layout (to accumulate an MFMA update onto it)
HQR_DEV f64x4 ld_blk(const double (*M)[LD65], int r0, int c0, int lane)
{
    f64x4 d;
#pragma unroll
    for (int r = 0; r < 4; ++r) d[r] = M[r0 + 4 * r + (lane >> 4)][c0 + (lane & 15)];
    return d;
}

// In-place upper Cholesky G = R^T R of the n x n block of G (R in the upper
// part, zeros below, identity beyond n; G's entries outside the block must
// be zero), by 16-column block steps.  In block step kb ONE wave computes
// rows 16kb .. 16kb+15 of R (lane t owning column 16kb + t, right-looking
// within the block: the pivot from lane i by readlane, then the rank-1
// update of the block's remaining rows with the other columns' entries by
// readlane); then all waves subtract R_p^T R_p from the trailing upper
// blocks on MFMA.  gdiag gets G's original
// diagonal, rdiag R's; *bad is set when a pivot^2 falls below ratio * G_kk.
// Starts and ends with a barrier.
HQR_DEV void chol64_blk(double (*G)[LD65], int n, int lane, int w, double ratio, double *gdiag, double *rdiag,
                        int *bad)
{
    const int tid = 64 * w + lane;
    __syncthreads();
    if (tid < NB) gdiag[tid] = (tid < n) ? G[tid][tid] : 1.0;
    if (tid == 0) *bad = 0;
    __syncthreads();
#pragma unroll 1
    for (int kb = 0; kb < 4; ++kb) {
        const int b0 = 16 * kb;
        if (w == 0) {
            // lane t holds column c = b0 + t of the block row; right-looking
            // within the block, other columns' entries by readlane
            const int c = b0 + lane;
            const bool act = c < NB;
            double g[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) g[i] = act ? G[b0 + i][c] : 0.0;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int gi = b0 + i;
                const double piv = readlane_f64(g[i], i);
                const double rii = (gi < n) ? sqrt(fmax(piv, 0.0)) : 1.0;
                if (lane == 0 && gi < n && !(piv > ratio * gdiag[gi])) *bad = 1;
                double v;
                if (gi >= n) v = (c == gi) ? 1.0 : 0.0;
                else if (lane < i) v = 0.0;
                else if (lane == i) v = rii;
                else v = (c < n) ? g[i] / rii : 0.0;
#pragma unroll
                for (int i2 = i + 1; i2 < 16; ++i2) g[i2] = fma(-readlane_f64(v, i2), v, g[i2]);
                g[i] = v;
            }
            if (act) {
#pragma unroll
                for (int i = 0; i < 16; ++i) G[b0 + i][c] = g[i];
            }
        }
        __syncthreads();
        // trailing upper blocks (ib <= jb): G_ij -= R_p,i^T R_p,j, R_p = rows b0..b0+15
        const int rem = 3 - kb;
        const int nblk = rem * (rem + 1) / 2;
        for (int bidx = w; bidx < nblk; bidx += 4) {
            int ib = 0, jb = 0, cnt = 0;
            for (int a = kb + 1; a <= 3; ++a)
                for (int b = a; b <= 3; ++b) {
                    if (cnt == bidx) { ib = a; jb = b; }
                    ++cnt;
                }
            f64x4 acc = ld_blk(G, 16 * ib, 16 * jb, lane);
            const int i16 = lane & 15, kk = lane >> 4;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = b0 + 4 * q + kk;
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-G[k][16 * ib + i16], G[k][16 * jb + i16], acc, 0, 0, 0);
            }
            st_blk(G, 16 * ib, 16 * jb, acc, 1.0, lane);
        }
        __syncthreads();
    }
    for (int idx = tid; idx < NB * NB; idx += 256) {
        const int i = idx / NB, c = idx % NB;
        if (i > c) G[i][c] = 0.0;
    }
    if (tid < NB) rdiag[tid] = G[tid][tid];
    __syncthreads();
}

// In place: M (n x n block; entries outside it zero) becomes L (strict
// lower, unit diagonal implied) and U (upper, diagonal U_kk) of the LU
// factorization without pivoting of M - S, s_k = -sgn(pivot k) (sgn(0) = +1)
// chosen at step k; entries outside the block stay zero.  Block steps of 16:
// ONE wave computes U's block row and L's block column (lane t owning column
// 16kb + t of U and row 16kb + t of L, right-looking within the block with
// the other lanes' entries by readlane), then all waves subtract L_p U_p
// from the trailing blocks on MFMA.  Starts and
// ends with a barrier.
HQR_DEV void lu_sign64_blk(double (*M)[LD65], int n, int lane, int w, double *sgn, double *udiag)
{
    __syncthreads();
#pragma unroll 1
    for (int kb = 0; kb < 4; ++kb) {
        const int b0 = 16 * kb;
        if (w == 0) {
            // lane t holds column t over the block rows (cv) and row t over the
            // block columns (rv); the diagonal block is in both copies, which
            // receive identical updates; other lanes' entries by readlane
            const int t = b0 + lane;
            const bool act = t < NB;
            double cv[16], rv[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                cv[i] = act ? M[b0 + i][t] : 0.0;
                rv[i] = act ? M[t][b0 + i] : 0.0;
            }
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int gi = b0 + i;
                const double q = readlane_f64(cv[i], i);
                const double sg = (q >= 0.0) ? -1.0 : 1.0;
                const double ukk = q - sg;
                const double u = (lane > i) ? cv[i] : ((lane == i) ? ukk : 0.0);   // U[gi][t]
                const double l = (lane > i) ? rv[i] / ukk : 0.0;                   // L[t][gi]
#pragma unroll
                for (int i2 = i + 1; i2 < 16; ++i2) {
                    cv[i2] = fma(-readlane_f64(l, i2), u, cv[i2]);
                    rv[i2] = fma(-l, readlane_f64(u, i2), rv[i2]);
                }
                cv[i] = u;
                rv[i] = l;
                if (lane == 0 && gi < n) {
                    sgn[gi] = sg;
                    udiag[gi] = ukk;
                }
            }
            if (act && t < n) {
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int gi = b0 + i;
                    if (gi < n && lane >= i) M[gi][t] = cv[i];
                    if (gi < n && lane > i) M[t][gi] = rv[i];
                }
            }
        }
        __syncthreads();
        // trailing blocks: M_ij -= L_p,i U_p,j over the block's 16 pivots
        const int rem = 3 - kb;
        for (int bidx = w; bidx < rem * rem; bidx += 4) {
            const int ib = kb + 1 + bidx / rem, jb = kb + 1 + bidx % rem;
            f64x4 acc = ld_blk(M, 16 * ib, 16 * jb, lane);
            const int i16 = lane & 15, kk = lane >> 4;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = b0 + 4 * q + kk;
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-M[16 * ib + i16][k], M[k][16 * jb + i16], acc, 0, 0, 0);
            }
            st_blk(M, 16 * ib, 16 * jb, acc, 1.0, lane);
        }
        __syncthreads();
    }
}

// out (global, row-major 64 x 64) = (A * B) diag(cs) on columns < bw, zero
// beyond; A, B in LDS; 256 threads, wave w computes row tile w.
HQR_DEV void mm64_to_global(double *out, const double (*A)[LD65], const double (*B)[LD65], const double *cs,
                            int bw, int lane, int w)
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
    for (int t = 0; t < 4; ++t) {
        const int c = 16 * t + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) out[(16 * w + 4 * r + (lane >> 4)) * NB + c] = (c < bw) ? acc[t][r] * cs[c] : 0.0;
    }
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
    // pass 2 reads R1^{-1}, R1 and A's top block late: load them now, so the
    // loads overlap the Cholesky factorization
    double pf_r1inv[16], pf_r1[16], pf_at[16];
    if (p.pass == 2) {
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const int idx = tid + 256 * t;
            const int c = idx / NB, r = idx % NB;
            pf_r1inv[t] = p.r1inv[idx];
            pf_r1[t] = p.r1[idx];
            pf_at[t] = (r < bw && c < bw) ? HQR_AT(p.A, (int64_t)p.c0 + r, p.c0 + c, p.lda) : 0.0;
        }
    }

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
    chol64_blk(M0, bw, lane, w, CQR_RATIO, gdiag, rdiag, &bad);
    HQR_TS();
    if (tid == 0 && (bad || structural)) atomicExch(p.flag, 1);
    __syncthreads();
    if (bad || __hip_atomic_load(p.flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;

    if (p.pass == 1) {
        for (int idx = tid; idx < NB * NB; idx += 256) p.r1[idx] = M0[idx / NB][idx % NB];
        inv_upper64_blk(M1, M0, bw, lane, w);
        for (int idx = tid; idx < NB * NB; idx += 256) p.r1inv[idx] = M1[idx / NB][idx % NB];
        return;
    }

    // ---- pass 2: M0 = R2
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const int idx = tid + 256 * t;
        M2[idx / NB][idx % NB] = pf_r1inv[t];
    }
    inv_upper64_blk(M1, M0, bw, lane, w);                // M1 = R2^{-1}
    HQR_TS();
    mm64(M3, M2, M1, lane, w);                          // M3 = R^{-1} = R1^{-1} R2^{-1}
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const int idx = tid + 256 * t;
        M2[idx / NB][idx % NB] = pf_r1[t];
    }
    __syncthreads();
    mm64(M1, M0, M2, lane, w);                          // M1 = R = R2 R1
    __syncthreads();
    // Q_top = A_top R^{-1}
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const int idx = tid + 256 * t;
        M2[idx % NB][idx / NB] = pf_at[t];
    }
    __syncthreads();
    mm64(M0, M2, M3, lane, w);                          // M0 = Q_top
    __syncthreads();
    HQR_TS();
    // modified LU of Q_top - S (in place in M0)
    lu_sign64_blk(M0, bw, lane, w, sgn, rdiag);
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
    // U^{-1} and L^{-1} from the LU in M0
    inv_upper64_blk(M2, M0, bw, lane, w);
    inv_unit_lower64_blk(M1, M0, bw, lane, w);
    HQR_TS();
    // W^{-1} = R^{-1} U^{-1} diag(up), straight to global
    mm64_to_global(p.winv, M3, M2, upv, bw, lane, w);
    __syncthreads();
    // T_Y = -(U S) L^{-T};  T_V = T_Y / (up_i up_j)
    for (int idx = tid; idx < NB * NB; idx += 256) {
        const int i = idx / NB, l = idx % NB;
        M2[i][l] = (i <= l && l < bw) ? M0[i][l] * sgn[l] : 0.0; // U S
        M3[l][i] = M1[i][l];                                     // L^{-T}
    }
    __syncthreads();
    mm64(M1, M2, M3, lane, w);
    __syncthreads();
    for (int idx = tid; idx < NB * NB; idx += 256) {
        const int i = idx / NB, j = idx % NB;
        p.T[idx] = (i <= j && j < bw) ? -M1[i][j] / (upv[i] * upv[j]) : 0.0;
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
