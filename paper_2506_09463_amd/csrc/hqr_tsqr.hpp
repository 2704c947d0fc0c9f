// hqr_tsqr.hpp -- the data movement of the TSQR panel (tall-skinny QR by a
// reduction tree of row-block factorizations, followed by Householder
// reconstruction of the panel's one-reflector-per-column form).
//
// A panel A_p (m_p x bw) is split into row blocks of at most
// TSQR_LEAF_ROWS rows; each block is factored by the one-workgroup kernel
// (A_i = Q_i R_i), the R_i are stacked and factored again, level by level,
// until one block remains (R).  The explicit orthonormal factor follows
// top-down: the top block's Q applied to [I; 0], then each level's blocks
// applied to their rows of the level above (padded with zeros).  The
// result Q (m_p x bw, orthonormal to working precision at any conditioning
// of A_p) and R with A_p = Q R replace the panel and the first CholeskyQR
// factor; the reconstruction of the CholeskyQR2 path then runs on Q
// (its Gram matrix is the identity up to rounding) and gives the stored
// reflectors, T and R_house = S R2 R.  Because every reflector of the
// per-column loop is unchanged by a nonzero scaling of the vector it is built
// from, Householder QR of Q has the reflectors of Householder QR of A_p as
// long as R's diagonal is positive; the last two kernels make it so by scaling
// rows of R and columns of Q by -1.
//
// The descriptor kernel reads the panel's flag on the device: a panel with
// an exactly zero column tail (flag 1) keeps its exact one-reflector path,
// so every TSQR launch of that panel is empty (descriptors with n = 0).
#pragma once

#include "hqr_args.hpp"

namespace hqr {

// Level l and block i of thread index t of the flattened block list.
HQR_DEV bool tsqr_locate(const TsqrArgs &a, int64_t t, int &l, int64_t &i)
{
    for (l = 0; l < a.nlev; ++l) {
        if (t < a.lev[l].nblk) {
            i = t;
            return true;
        }
        t -= a.lev[l].nblk;
    }
    return false;
}

// The factor and apply descriptors of every block of every level; the
// batched launches' queue heads to zero.  grid-stride, 256 threads.
__global__ void __launch_bounds__(256) tsqr_desc_kernel(TsqrArgs a)
{
    const int64_t t0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t0 < 2 * a.nlev) a.heads[t0] = 0;
    const bool skip = *((volatile int *)a.flag) == 1;
    const int64_t n = skip ? 0 : a.bw;
    int64_t total = 0;
    for (int l = 0; l < a.nlev; ++l) total += a.lev[l].nblk;
    for (int64_t t = t0; t < total; t += (int64_t)gridDim.x * 256) {
        int l;
        int64_t i;
        if (!tsqr_locate(a, t, l, i)) continue;
        const TsqrLevel &L = a.lev[l];
        const int64_t r0 = tsqr_block_start(L, i), rows = tsqr_block_rows(L, i);
        double *Ai = L.X + r0;
        double *upi = L.up + i * NB;
        L.fdesc[i] = WgDesc{rows, n, 0, L.ldx, 1, Ai, nullptr, upi, nullptr, 0, WG_FACTOR};
        const int64_t fl = WG_APPLY_Q | ((l == a.nlev - 1) ? WG_QSKIP : 0);
        L.adesc[i] = WgDesc{rows, n, (int64_t)a.bw, L.ldx, L.ldq, Ai, L.Q + r0, upi, nullptr, 0, fl};
    }
}

// Level l + 1's X = the stacked R factors of level l's (factored) blocks,
// zeros below each diagonal.  grid: level l's block count, 256 threads.
__global__ void __launch_bounds__(256) tsqr_gather_kernel(TsqrArgs a, int l)
{
    if (*((volatile int *)a.flag) == 1) return;
    const TsqrLevel &S = a.lev[l];
    const TsqrLevel &D = a.lev[l + 1];
    const int64_t i = blockIdx.x;
    const int bw = a.bw;
    const int64_t r0 = tsqr_block_start(S, i);
    for (int e = threadIdx.x; e < bw * bw; e += 256) {
        const int k = e % bw, j = e / bw;     // row k, column j of R_i
        const double v = (k <= j) ? S.X[(size_t)(r0 + k) + (size_t)j * S.ldx] : 0.0;
        D.X[(size_t)(i * bw + k) + (size_t)j * D.ldx] = v;
    }
}

// Level l's Q input: block i's rows take rows i*bw .. i*bw + bw - 1 of level
// l + 1's Q on top, zeros below.  grid: ceil(level l rows / 256), 256 threads.
__global__ void __launch_bounds__(256) tsqr_scatter_kernel(TsqrArgs a, int l)
{
    if (*((volatile int *)a.flag) == 1) return;
    const TsqrLevel &L = a.lev[l];
    const TsqrLevel &U = a.lev[l + 1];
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= L.rows) return;
    const int64_t big = L.rem * (L.base + 1);   // rows in the blocks of base + 1 rows
    int64_t i, off;
    if (r < big) {
        i = r / (L.base + 1);
        off = r - i * (L.base + 1);
    } else {
        i = L.rem + (r - big) / L.base;
        off = (r - big) - (i - L.rem) * L.base;
    }
    const int bw = a.bw;
    for (int j = 0; j < bw; ++j)
        L.Q[(size_t)r + (size_t)j * L.ldq] = (off < bw) ? U.Q[(size_t)(i * bw + off) + (size_t)j * U.ldq] : 0.0;
}

// The first CholeskyQR factor := D R (64 x 64, row-major, identity beyond
// bw), its inverse := the identity, and D = diag(sgn R_kk) (sgn(0) = +1)
// into sign[0..bw-1].  R is read from the top level, which is the panel
// itself for a one-level tree: the panel is only overwritten by the next
// kernel.  One workgroup of 256 threads.
__global__ void __launch_bounds__(256) tsqr_r_kernel(TsqrArgs a, double *r1, double *r1inv, double *sign)
{
    if (*((volatile int *)a.flag) == 1) return;
    const TsqrLevel &T = a.lev[a.nlev - 1];
    const int bw = a.bw;
    for (int e = threadIdx.x; e < NB * NB; e += 256) {
        const int i = e / NB, j = e % NB;
        double v = (i == j) ? 1.0 : 0.0;
        if (i < bw && j < bw) {
            const double di = (T.X[(size_t)i + (size_t)i * T.ldx] < 0.0) ? -1.0 : 1.0;
            v = (i <= j) ? di * T.X[(size_t)i + (size_t)j * T.ldx] : 0.0;
            if (i == j) sign[i] = di;
        }
        r1[e] = v;
        r1inv[e] = (i == j) ? 1.0 : 0.0;
    }
}

// The panel := Q D (level 0's explicit Q).  A panel flagged for the exact
// loop is left alone; the flag of an ill-conditioned panel (2) is cleared so
// the second pass runs (every workgroup reads it before any clears it, or
// reads 0: both mean "proceed").  grid: ceil(m_p / 256), 256 threads.
__global__ void __launch_bounds__(256) tsqr_final_kernel(TsqrArgs a, double *Ap, int64_t lda, const double *sign)
{
    if (*((volatile int *)a.flag) == 1) return;
    const TsqrLevel &L0 = a.lev[0];
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r < L0.rows) {
        for (int k = 0; k < a.bw; ++k) Ap[(size_t)r + (size_t)k * lda] = sign[k] * L0.Q[(size_t)r + (size_t)k * L0.ldq];
    }
    if (threadIdx.x == 0 && *((volatile int *)a.flag) == 2) *((volatile int *)a.flag) = 0;
}

} // namespace hqr
