// hqr_chol.hpp -- Cholesky factorization S = R^T R of a symmetric positive
// definite matrix (the factored form in which SLSQP keeps its Hessian
// approximation) and the rank-one update R'^T R' = R^T R + v v^T (which is
// also the update of a QR factorization's R when a row is appended).
//
// Factorization, right-looking by 64-column blocks k:
//   chol_diag_kernel   one workgroup: R_kk = chol(S_kk) and R_kk^{-1} (LDS)
//   chol_panel_kernel  R_kj = R_kk^{-T} S_kj for the block row (FP64 MFMA)
//   chol_syrk_kernel   S_ij -= R_ki^T R_kj on the trailing upper blocks
// Only the upper triangle of S is read or written.
#pragma once

#include "hqr_args.hpp"

namespace hqr {

constexpr int CH_LD = 65;

// out[i][j] = sum_k (TA ? A[k][i] : A[i][k]) B[k][j] for 64 x 64 LDS
// matrices (row-major, stride 65), FP64 MFMA; 256 threads, wave w computes
// rows 16w..16w+15.  Returned in D layout: acc[t][r] = out[16w + 4r + l/16][16t + l%16].
template <bool TA>
HQR_DEV void ch_mm64(f64x4 (&acc)[4], const double (*A)[CH_LD], const double (*B)[CH_LD], int lane, int w)
{
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int k0 = 0; k0 < 64; k0 += 4) {
        const int kr = k0 + (lane >> 4), i = 16 * w + (lane & 15);
        const double a = TA ? A[kr][i] : A[i][kr];
#pragma unroll
        for (int t = 0; t < 4; ++t)
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, B[kr][16 * t + (lane & 15)], acc[t], 0, 0, 0);
    }
}

struct CholArgsS {
    double *S;
    int64_t lds;
    int64_t n;
    int64_t k0;       // first row/column of the diagonal block
    int bw;           // block width (<= 64)
    double *rinv;     // [64][64] row-major R_kk^{-1}
    int *info;        // 0, or j+1 at the first non-positive pivot
};

// One workgroup.  Loads the upper triangle of S_kk (symmetric fill), factors
// it column by column (thread j < bw owns column j: at step p it reads the
// pivot row p published in LDS), inverts R_kk by column-oriented back
// substitution, writes R_kk over S_kk's upper triangle and R_kk^{-1} to rinv.
// A non-positive pivot sets *info = k0 + p + 1 and skips the rest.
__global__ void __launch_bounds__(256) chol_diag_kernel(CholArgsS a)
{
    __shared__ double M[64][CH_LD];
    __shared__ double X[64][CH_LD];
    __shared__ int bad;
    const int tid = threadIdx.x, bw = a.bw;
    if (*((volatile int *)a.info) != 0) return;
    if (tid == 0) bad = 0;
    for (int e = tid; e < 64 * 64; e += 256) {
        const int r = e & 63, c = e >> 6;
        double v = 0.0;
        if (r < bw && c < bw) {
            const int rr = r <= c ? r : c, cc = r <= c ? c : r;
            v = HQR_AT(a.S, a.k0 + rr, a.k0 + cc, a.lds);
        } else if (r == c) {
            v = 1.0;
        }
        M[r][c] = v;
        X[r][c] = 0.0;
    }
    __syncthreads();
    // right-looking unblocked Cholesky of the 64 x 64 block (identity beyond bw)
    for (int p = 0; p < 64; ++p) {
        const double piv = M[p][p];
        if (!(piv > 0.0)) {
            if (tid == 0 && p < bw) bad = p + 1;
            break;
        }
        const double rpp = sqrt(piv);
        __syncthreads();
        // row p of R: R[p][c] = M[p][c] / rpp for c >= p
        if (tid >= p && tid < 64) M[p][tid] = (tid == p) ? rpp : M[p][tid] / rpp;
        __syncthreads();
        // trailing update M[i][j] -= R[p][i] R[p][j] (upper part, i, j > p)
        for (int e = tid; e < 64 * 64; e += 256) {
            const int i = e >> 6, j = e & 63;
            if (i > p && j >= i) M[i][j] -= M[p][i] * M[p][j];
        }
        __syncthreads();
    }
    __syncthreads();
    if (bad) {
        if (tid == 0) atomicExch(a.info, (int)(a.k0 + bad));
        return;
    }
    // X = R^{-1}: thread c < 64 solves column c of R X = I by back substitution
    if (tid < 64) {
        const int c = tid;
        for (int i = c; i >= 0; --i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int l = i + 1; l <= c; ++l) s -= M[i][l] * X[l][c];
            X[i][c] = s / M[i][i];
        }
    }
    __syncthreads();
    for (int e = tid; e < 64 * 64; e += 256) {
        const int r = e >> 6, c = e & 63;
        a.rinv[e] = X[r][c];
        if (r < bw && c < bw && r <= c) HQR_AT(a.S, a.k0 + r, a.k0 + c, a.lds) = M[r][c];
    }
}

// grid: ceil((n - k0 - bw) / 64) column tiles j of the block row:
// R_kj = R_kk^{-T} S_kj (64 x 64 each), written over S_kj.
__global__ void __launch_bounds__(256) chol_panel_kernel(CholArgsS a)
{
    __shared__ double Ri[64][CH_LD];
    __shared__ double Sk[64][CH_LD];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (*((volatile int *)a.info) != 0) return;
    const int64_t c0 = a.k0 + a.bw + (int64_t)blockIdx.x * 64;
    const int nc = (int)min<int64_t>(64, a.n - c0);
    for (int e = tid; e < 64 * 64; e += 256) {
        const int r = e >> 6, c = e & 63;
        Ri[r][c] = a.rinv[e];
        const int rr = e & 63, cc = e >> 6;
        Sk[rr][cc] = (rr < a.bw && cc < nc) ? HQR_AT(a.S, a.k0 + rr, c0 + cc, a.lds) : 0.0;
    }
    __syncthreads();
    f64x4 acc[4];
    ch_mm64<true>(acc, Ri, Sk, lane, w);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 16 * w + 4 * r + (lane >> 4), j = 16 * t + (lane & 15);
            if (i < a.bw && j < nc) HQR_AT(a.S, a.k0 + i, c0 + j, a.lds) = acc[t][r];
        }
}

// grid: (T, T) over the trailing column tiles (T = ceil((n - k0 - bw)/64));
// tiles below the diagonal return.  S_ij -= R_ki^T R_kj; on diagonal tiles
// only the upper triangle is written.
__global__ void __launch_bounds__(256) chol_syrk_kernel(CholArgsS a)
{
    __shared__ double Ri[64][CH_LD];
    __shared__ double Rj[64][CH_LD];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (blockIdx.x > blockIdx.y) return;
    if (*((volatile int *)a.info) != 0) return;
    const int64_t t0 = a.k0 + a.bw;
    const int64_t ri = t0 + (int64_t)blockIdx.x * 64, cj = t0 + (int64_t)blockIdx.y * 64;
    const int ni = (int)min<int64_t>(64, a.n - ri), nj = (int)min<int64_t>(64, a.n - cj);
    for (int e = tid; e < 64 * 64; e += 256) {
        const int k = e & 63, c = e >> 6;
        Ri[k][c] = (k < a.bw && c < ni) ? HQR_AT(a.S, a.k0 + k, ri + c, a.lds) : 0.0;
        Rj[k][c] = (k < a.bw && c < nj) ? HQR_AT(a.S, a.k0 + k, cj + c, a.lds) : 0.0;
    }
    __syncthreads();
    f64x4 acc[4];
    ch_mm64<true>(acc, Ri, Rj, lane, w);
    const bool diag = blockIdx.x == blockIdx.y;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 16 * w + 4 * r + (lane >> 4), j = 16 * t + (lane & 15);
            if (i < ni && j < nj && (!diag || i <= j)) HQR_AT(a.S, ri + i, cj + j, a.lds) -= acc[t][r];
        }
}

// ------------------------------------------------------------ rank-one update
// One workgroup of 1024 threads; thread t owns columns t, t + 1024, ..
// (CPT of them).  Rotation k is formed by the owner of column k from R[k][k]
// and its running v_k and published in LDS (double-buffered, one barrier per
// step); every owner of a column j > k then rotates (R[k][j], v_j).  Rows
// are staged CHOL_UCH at a time in registers (each column is walked
// downwards).  n <= 1024 CPT.
constexpr int CHOL_UCH = 8;
template <int CPT>
__global__ void __launch_bounds__(1024) chol_update_kernel(double *R, int64_t ldr, double *v, int64_t n)
{
    __shared__ double cs[2][2];
    const int tid = threadIdx.x;
    double vj[CPT];
    int64_t col[CPT];
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        col[q] = tid + 1024 * (int64_t)q;
        vj[q] = (col[q] < n) ? v[col[q]] : 0.0;
    }
    for (int64_t k0 = 0; k0 < n; k0 += CHOL_UCH) {
        const int kn = (int)min<int64_t>(CHOL_UCH, n - k0);
        double rk[CPT][CHOL_UCH];
#pragma unroll
        for (int q = 0; q < CPT; ++q)
#pragma unroll
            for (int u = 0; u < CHOL_UCH; ++u) {
                const bool ok = col[q] < n && u < kn && k0 + u <= col[q];
                rk[q][u] = ok ? HQR_AT(R, k0 + u, col[q], ldr) : 0.0;
            }
#pragma unroll
        for (int u = 0; u < CHOL_UCH; ++u) {
            if (u >= kn) break;
            const int64_t k = k0 + u;
            const int buf = (int)(k & 1);
            // the owner of column k forms rotation k
#pragma unroll
            for (int q = 0; q < CPT; ++q) {
                if (col[q] == k) {
                    const double a = rk[q][u], b = vj[q];
                    const double h = hypot(a, b);
                    const double r = (a >= 0.0) ? h : -h;
                    double c = 1.0, s = 0.0;
                    if (r != 0.0) {
                        c = a / r;
                        s = b / r;
                    }
                    rk[q][u] = r;
                    vj[q] = 0.0;
                    cs[buf][0] = c;
                    cs[buf][1] = s;
                }
            }
            __syncthreads();
            const double c = cs[buf][0], s = cs[buf][1];
#pragma unroll
            for (int q = 0; q < CPT; ++q) {
                if (col[q] > k && col[q] < n) {
                    const double a = rk[q][u], b = vj[q];
                    rk[q][u] = c * a + s * b;
                    vj[q] = -s * a + c * b;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < CPT; ++q)
#pragma unroll
            for (int u = 0; u < CHOL_UCH; ++u) {
                const bool ok = col[q] < n && u < kn && k0 + u <= col[q];
                if (ok) HQR_AT(R, k0 + u, col[q], ldr) = rk[q][u];
            }
    }
#pragma unroll
    for (int q = 0; q < CPT; ++q)
        if (col[q] < n) v[col[q]] = vj[q];
}

} // namespace hqr
