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
// (exact_panel) instead:
//   - a column whose part below the pivot row is exactly zero (the loop then
//     keeps H_k = I; this includes an empty tail when m_p == bw);
//   - a Cholesky pivot whose squared ratio to the column's norm falls below
//     CQR_RATIO (conditioning beyond what two CholeskyQR passes repair, or
//     rank deficiency).
// The decision is taken on the device: `flag` then makes pass 2 run the exact
// loop instead.
//
// A panel takes two kernels, each a grid-wide step whose reduction and
// small-matrix stage run in the workgroup that finishes last:
//   cqr_pass1_kernel  (previous panel's update of these columns +) Gram
//                     partials -> G -> R1, R1^{-1}
//   cqr_pass2_kernel  Q1 and its Gram partials -> G2 -> R2 -> reconstruction
// and the bottom rows become V_bot = A_bot W^{-1} in narrow_vtx_kernel (which
// also forms W = T^T V^T C for the next panel's columns, with look-ahead) or
// cqr_finish_kernel.
#pragma once

#include "hqr_args.hpp"

namespace hqr {


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

// 16 x 16 LDS block in D layout (to accumulate an MFMA update onto it)
HQR_DEV f64x4 ld_blk(const double (*M)[LD65], int r0, int c0, int lane)
{
    f64x4 d;
#pragma unroll
    for (int r = 0; r < 4; ++r) d[r] = M[r0 + 4 * r + (lane >> 4)][c0 + (lane & 15)];
    return d;
}

// ------------------------------------------------- in-row broadcasts
// The value that lane 16r + I holds, in every lane of the 16-lane row r
// (DPP row_newbcast; one v_mov_b64_dpp for a double).
template <int I> HQR_DEV double bc16c(double v)
{
    const long b = __builtin_bit_cast(long, v);
    const long r = __builtin_amdgcn_mov_dpp(b, 0x150 + I, 0xf, 0xf, false);
    return __builtin_bit_cast(double, r);
}

// Pins v in a register at this point of the program: the compiler may not
// move its computation past it (used to keep long update chains in order).
HQR_DEV void pin(double &v) { asm volatile("" : "+v"(v)); }

// i must be a constant once the caller's loops are unrolled
HQR_DEV double bc16(double v, int i)
{
    switch (i) {
    case 0: return bc16c<0>(v);
    case 1: return bc16c<1>(v);
    case 2: return bc16c<2>(v);
    case 3: return bc16c<3>(v);
    case 4: return bc16c<4>(v);
    case 5: return bc16c<5>(v);
    case 6: return bc16c<6>(v);
    case 7: return bc16c<7>(v);
    case 8: return bc16c<8>(v);
    case 9: return bc16c<9>(v);
    case 10: return bc16c<10>(v);
    case 11: return bc16c<11>(v);
    case 12: return bc16c<12>(v);
    case 13: return bc16c<13>(v);
    case 14: return bc16c<14>(v);
    default: return bc16c<15>(v);
    }
}

// s = sqrt(d) and r = 1/sqrt(d): the hardware reciprocal square root refined
// by two coupled Newton steps (Goldschmidt's iteration for s and 1/(2s)) and
// a final residual correction of s.  d below 2^-900 is scaled by 2^1000
// first; d <= 0 (or NaN) gives s = r = 1, the caller flags such pivots.
HQR_DEV void pivot_sqrt(double d, double &s, double &r)
{
    const bool pos = d > 0.0;
    const bool sc = pos && d < 0x1p-900;
    const double x = pos ? (sc ? d * 0x1p+1000 : d) : 1.0;
    const double y = __builtin_amdgcn_rsq(x);
    double sv = x * y, h = 0.5 * y;
    double e = fma(-sv, h, 0.5);
    sv = fma(sv, e, sv);
    h = fma(h, e, h);
    e = fma(-sv, h, 0.5);
    sv = fma(sv, e, sv);
    h = fma(h, e, h);
    sv = fma(h, fma(-sv, sv, x), sv);
    s = sc ? sv * 0x1p-500 : sv;
    r = sc ? (2.0 * h) * 0x1p+500 : 2.0 * h;
}

// 1/u from the hardware reciprocal and two Newton steps (|u| >= 1 here).
HQR_DEV double recip_nr(double u)
{
    double y = __builtin_amdgcn_rcp(u);
    double e = fma(-u, y, 1.0);
    y = fma(y, e, y);
    e = fma(-u, y, 1.0);
    return fma(y, e, y);
}

// In-place upper Cholesky G = R^T R of the n x n leading block of G (R in the
// upper triangle, zeros below, identity beyond n; G's entries outside the
// block must be zero), right-looking by 16-column block steps.
//
// Block step kb: wave 0 factors block row kb in registers.  Lane t holds
// column 16kb + t of the block row, and every 16-lane row also holds a copy
// of the diagonal block (lane 16r + j: its column j), so the entries of the
// current row of R that a rank-1 update needs are taken from the lane's own
// row by DPP broadcast.  The same wave then inverts the diagonal block by back
// substitution into X's diagonal block.  All waves then subtract
// R_kb^T R_kb from the trailing upper blocks on MFMA.
//
// gdiag gets G's diagonal (1 beyond n), rdiag R's; *bad is set when a pivot
// is not above ratio * G_kk.  Starts and ends with a barrier.
HQR_DEV void chol64_dpp(double (*G)[LD65], double (*X)[LD65], int n, int lane, int w, double ratio,
                        double *gdiag, double *rdiag, int *bad)
{
    const int tid = 64 * w + lane;
    __syncthreads();
    if (tid < NB) {
        gdiag[tid] = (tid < n) ? G[tid][tid] : 1.0;
        if (tid >= n) G[tid][tid] = 1.0;
    }
    if (tid == 0) *bad = 0;
    __syncthreads();
#pragma unroll 1
    for (int kb = 0; kb < 4; ++kb) {
        const int b0 = 16 * kb;
        if (w == 0) {
            // opaque per block step: keeps the per-pivot lane masks from being
            // hoisted out of the kb loop (they would occupy ~100 SGPRs)
            int ln = lane;
            asm volatile("" : "+v"(ln));
            const int jj = ln & 15, c = b0 + ln;
            const bool act = c < NB;
            double g[16], p[16], acc[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                g[i] = G[b0 + i][b0 + jj];
                p[i] = act ? G[b0 + i][c] : 0.0;
                acc[i] = 0.0;
            }
            // lane i keeps pivot i and R_ii.  X = R_kk^{-1} is built along:
            // lane j holds row j of X; acc[l] = sum_{i<l} X[j][i] R[i][l], and
            // column i of X is -acc[i] / R_ii above the diagonal.
            double my_d = 1.0, my_s = 0.0;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int gi = b0 + i;
                const double d = bc16(g[i], i);
                double s, r;
                pivot_sqrt(d, s, r);
                const double vg = (jj > i) ? g[i] * r : ((jj == i) ? s : 0.0);
                const double vp = (c > gi) ? p[i] * r : ((c == gi) ? s : 0.0);
                const double xi = (jj < i) ? -acc[i] * r : ((jj == i) ? r : 0.0);   // X[j][i]
                g[i] = vg;
                p[i] = vp;
                my_d = (ln == i) ? d : my_d;
                my_s = (ln == i) ? s : my_s;
                X[b0 + jj][b0 + i] = xi;   // the four rows store the same value
#pragma unroll
                for (int i2 = i + 1; i2 < 16; ++i2) {
                    const double t = bc16(vg, i2);          // R[i][i2]
                    g[i2] = fma(-t, vg, g[i2]);
                    p[i2] = fma(-t, vp, p[i2]);
                    acc[i2] = fma(xi, t, acc[i2]);
                    pin(g[i2]);
                    pin(p[i2]);
                    pin(acc[i2]);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            if (act) {
#pragma unroll
                for (int i = 0; i < 16; ++i) G[b0 + i][c] = p[i];
            }
            const bool badl = lane < 16 && b0 + lane < n && !(my_d > ratio * gdiag[b0 + lane]);
            if (lane < 16) rdiag[b0 + lane] = my_s;
            if (badl) *bad = 1;
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
    __syncthreads();
}

// One block step of the LU below, in one wave: LPART = false computes U's
// block row (lane t: column 16kb + t) and U_kk^{-1}; LPART = true computes
// L's block column (lane t: row 16kb + t) and L_kk^{-1}.  Both keep the
// diagonal block (lane 16r + j: its column j in dc, its row j in dr, in
// every 16-lane row for the DPP broadcasts) and take the same pivots.
// ov: U[.][c] (block row) or L[c][.] (block column) of the block step
template <bool LPART>
HQR_DEV void lu64_load(const double (*M)[LD65], int b0, int lane, double (&ov)[16], double (&dc)[16],
                       double (&dr)[16])
{
    const int jj = lane & 15, c = b0 + lane;
    const bool act = c < NB;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        ov[i] = act ? (LPART ? M[c][b0 + i] : M[b0 + i][c]) : 0.0;
        dc[i] = M[b0 + i][b0 + jj];
        dr[i] = M[b0 + jj][b0 + i];
    }
}

// The block step on the loaded values (after a barrier: the other wave's
// writes to M cannot race with these reads).  ax: the running sums of
// U_kk^{-1} (row j: ax[l] = sum_{i<l} XU[j][i] U[i][l]) or of L_kk^{-1}
// (column j: ax[l] = sum_{i<l} L[l][i] XL[i][j]).
template <bool LPART>
HQR_DEV void lu64_block(double (*M)[LD65], double (*DX)[17], int b0, int lane, double *sgn, double *udiag,
                        double (&ov)[16], double (&dc)[16], double (&dr)[16])
{
    // opaque per block step: keeps the per-pivot lane masks from being
    // hoisted out of the caller's kb loop (they would occupy ~100 SGPRs)
    int ln = lane;
    asm volatile("" : "+v"(ln));
    const int jj = ln & 15, c = b0 + ln;
    const bool act = c < NB;
    double ax[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) ax[i] = 0.0;
    double my_sg = 0.0, my_uk = 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int gi = b0 + i;
        const double q = bc16(dc[i], i);
        const double sg = (q >= 0.0) ? -1.0 : 1.0;
        const double ukk = q - sg;
        const double uinv = recip_nr(ukk);
        const double ud = (jj > i) ? dc[i] : ((jj == i) ? ukk : 0.0);
        const double ld = (jj > i) ? dr[i] * uinv : 0.0;
        // U[gi][c] or L[c][gi]
        const double oc = LPART ? ((c > gi) ? ov[i] * uinv : 0.0) : ((c > gi) ? ov[i] : ((c == gi) ? ukk : 0.0));
        // XU[j][i] or XL[i][j]
        const double xv = LPART ? ((jj < i) ? -ax[i] : ((jj == i) ? 1.0 : 0.0))
                                : ((jj < i) ? -ax[i] * uinv : ((jj == i) ? uinv : 0.0));
        dc[i] = ud;
        dr[i] = ld;
        ov[i] = oc;
        if (!LPART) {
            my_sg = (ln == i) ? sg : my_sg;
            my_uk = (ln == i) ? ukk : my_uk;
            DX[b0 + jj][i] = xv;       // the four rows store the same value
        } else {
            DX[b0 + i][jj] = xv;
        }
#pragma unroll
        for (int i2 = i + 1; i2 < 16; ++i2) {
            const double lb = bc16(ld, i2), ub = bc16(ud, i2);   // L[i2][i], U[i][i2]
            dc[i2] = fma(-lb, ud, dc[i2]);
            dr[i2] = fma(-ld, ub, dr[i2]);
            if (!LPART) {
                ov[i2] = fma(-lb, oc, ov[i2]);
                ax[i2] = fma(xv, ub, ax[i2]);
            } else {
                ov[i2] = fma(-oc, ub, ov[i2]);
                ax[i2] = fma(lb, xv, ax[i2]);
            }
            pin(dc[i2]);
            pin(dr[i2]);
            pin(ov[i2]);
            pin(ax[i2]);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    if (act) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int gi = b0 + i;
            if (!LPART && c >= gi) M[gi][c] = ov[i];
            if (LPART && c > gi) M[c][gi] = ov[i];
        }
    }
    if (!LPART && ln < 16) {
        sgn[b0 + ln] = my_sg;
        udiag[b0 + ln] = my_uk;
    }
}

// In place: M (n x n leading block; entries outside it zero) becomes L
// (strict lower, unit diagonal implied) and U (upper, diagonal U_kk) of the
// LU factorization without pivoting of M - S, s_k = -sgn(pivot of step k)
// (sgn(0) = +1); beyond n the factors continue as the identity (s_k = -1,
// U_kk = 1).  Block step kb: wave 0 computes U's block row and the diagonal
// block of U^{-1} (into DU, rows 16kb..16kb+15), wave 1 L's block column and
// the diagonal block of L^{-1} (into DL), both by lu64_block; all waves then
// subtract L_kb U_kb from the trailing blocks on MFMA.  sgn and udiag get s_k
// and U_kk for all 64 steps.  Starts and ends with a barrier.
HQR_DEV void lu64_dpp(double (*M)[LD65], double (*DU)[17], double (*DL)[17], int lane, int w, double *sgn,
                      double *udiag)
{
    __syncthreads();
#pragma unroll 1
    for (int kb = 0; kb < 4; ++kb) {
        const int b0 = 16 * kb;
        double ov[16], dc[16], dr[16];
        if (w == 0) lu64_load<false>(M, b0, lane, ov, dc, dr);
        else if (w == 1) lu64_load<true>(M, b0, lane, ov, dc, dr);
        __syncthreads();
        if (w == 0) lu64_block<false>(M, DU, b0, lane, sgn, udiag, ov, dc, dr);
        else if (w == 1) lu64_block<true>(M, DL, b0, lane, sgn, udiag, ov, dc, dr);
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

// Off-diagonal blocks of triangular inverses whose diagonal blocks are
// already in place, by distance from the diagonal on MFMA:
//   upper U:      X_ij = -X_ii sum_{k=i+1..j} U_ik X_kj   (i < j)
//   unit lower L: X_ij = -X_ii sum_{k=j..i-1} L_ik X_kj   (i > j)
// One 16 x 16 block task: t = sum of the products, X_ij = -X_ii t.
HQR_DEV void inv_upper_task(double (*X)[LD65], const double (*U)[LD65], int i, int j, int lane)
{
    f64x4 t = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int k = i + 1; k <= j; ++k) t = mma_blk(t, U, 16 * i, 16 * k, X, 16 * k, 16 * j, lane);
    st_blk(X, 16 * i, 16 * j, mma_blk_reg(f64x4{0.0, 0.0, 0.0, 0.0}, X, 16 * i, 16 * i, t, lane), -1.0, lane);
}

HQR_DEV void inv_lower_task(double (*X)[LD65], const double (*L)[LD65], int i, int j, int lane)
{
    f64x4 t = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int k = j; k < i; ++k) t = mma_blk(t, L, 16 * i, 16 * k, X, 16 * k, 16 * j, lane);
    st_blk(X, 16 * i, 16 * j, mma_blk_reg(f64x4{0.0, 0.0, 0.0, 0.0}, X, 16 * i, 16 * i, t, lane), -1.0, lane);
}

// zero the blocks of X strictly below (lower = true: above) the diagonal
HQR_DEV void zero_off_blocks(double (*X)[LD65], bool above, int tid)
{
    for (int idx = tid; idx < NB * NB; idx += 256) {
        const int r = idx / NB, c = idx % NB;
        if (above ? ((c >> 4) > (r >> 4)) : ((r >> 4) > (c >> 4))) X[r][c] = 0.0;
    }
}

// X = U^{-1} (64 x 64 upper U) given X's diagonal blocks.  Starts and ends
// with a barrier.
HQR_DEV void inv_upper_levels(double (*X)[LD65], const double (*U)[LD65], int lane, int w)
{
    __syncthreads();
    zero_off_blocks(X, false, 64 * w + lane);
    if (w < 3) inv_upper_task(X, U, w, w + 1, lane);
    __syncthreads();
    if (w < 2) inv_upper_task(X, U, w, w + 2, lane);
    __syncthreads();
    if (w == 0) inv_upper_task(X, U, 0, 3, lane);
    __syncthreads();
}

// XU = U^{-1} and XL = L^{-1} for the U (upper) and L (strict lower, unit
// diagonal) that share M, given the diagonal blocks of XU and XL.  Starts and
// ends with a barrier.
HQR_DEV void inv_lu_levels(double (*XU)[LD65], double (*XL)[LD65], const double (*M)[LD65], int lane, int w)
{
    __syncthreads();
    zero_off_blocks(XU, false, 64 * w + lane);
    zero_off_blocks(XL, true, 64 * w + lane);
    for (int task = w; task < 6; task += 4) {
        if (task < 3) inv_upper_task(XU, M, task, task + 1, lane);
        else inv_lower_task(XL, M, task - 2, task - 3, lane);
    }
    __syncthreads();
    if (w < 2) inv_upper_task(XU, M, w, w + 2, lane);
    else inv_lower_task(XL, M, w, w - 2, lane);
    __syncthreads();
    if (w == 0) inv_upper_task(XU, M, 0, 3, lane);
    else if (w == 1) inv_lower_task(XL, M, 3, 0, lane);
    __syncthreads();
}

// Products of 64 x 64 operands given by element functions fa(r, c), fb(r, c),
// into D-layout accumulators (acc[s][q] = C[16 bi + 4q + lane/16][16 bj +
// lane%16] for the wave's block (bi, bj) of slot s).
//
// Upper x upper: the 10 blocks bi <= bj, each summed over k = bi..bj (20
// block products), spread 5 per wave; uu_slot gives slot s of wave w as
// 4 bi + bj, or -1.
HQR_DEV int uu_slot(int w, int s)
{
    // w0: (0,3) (3,3)  w1: (0,2) (1,2)  w2: (1,3) (0,1)  w3: (2,3) (0,0) (1,1) (2,2)
    const unsigned tab = (w == 0) ? 0xffff0f03u : (w == 1) ? 0xffff0602u : (w == 2) ? 0xffff0107u : 0x0a05000bu;
    const int e = (int)((tab >> (8 * s)) & 0xffu);
    return e == 0xff ? -1 : e;
}

template <class FA, class FB>
HQR_DEV void mm_upper_upper(f64x4 (&acc)[4], FA fa, FB fb, int lane, int w)
{
    const int i16 = lane & 15, kk = lane >> 4;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        acc[s] = f64x4{0.0, 0.0, 0.0, 0.0};
        const int e = uu_slot(w, s);
        if (e < 0) continue;
        const int bi = e >> 2, bj = e & 3;
        for (int kb = bi; kb <= bj; ++kb) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = 16 * kb + 4 * q + kk;
                acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa(16 * bi + i16, k), fb(k, 16 * bj + i16), acc[s], 0, 0, 0);
            }
        }
    }
}

// Full x upper: wave w computes block row w, block (w, bj) summed over
// k = 0..bj (slot s = bj).
template <class FA, class FB>
HQR_DEV void mm_full_upper(f64x4 (&acc)[4], FA fa, FB fb, int lane, int w)
{
    const int i16 = lane & 15, kk = lane >> 4;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        acc[s] = f64x4{0.0, 0.0, 0.0, 0.0};
        for (int kb = 0; kb <= s; ++kb) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = 16 * kb + 4 * q + kk;
                acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa(16 * w + i16, k), fb(k, 16 * s + i16), acc[s], 0, 0, 0);
            }
        }
    }
}

// Visit the elements of the wave's upper x upper accumulators:
// f(row, col, value).
template <class F>
HQR_DEV void for_uu(const f64x4 (&acc)[4], F f, int lane, int w)
{
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int e = uu_slot(w, s);
        if (e < 0) continue;
        const int bi = e >> 2, bj = e & 3;
#pragma unroll
        for (int q = 0; q < 4; ++q) f(16 * bi + 4 * q + (lane >> 4), 16 * bj + (lane & 15), acc[s][q]);
    }
}

// M[r][c] = A[r0 + r][c0 + c] (r < 64, c < NB), zero for rows >= m or
// columns >= ncol.  256 threads; the loads are unconditional (clamped into
// the matrix, zeroed afterwards), so all 16 of a thread are in flight
// together instead of each waiting behind its own branch.
HQR_DEV void tile_issue(double (&v)[16], const double *A, int64_t lda, int64_t m, int64_t r0, int c0, int ncol,
                        int tid)
{
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int idx = tid + 256 * q, c = idx / 64, r = idx % 64;
        const int64_t gi = r0 + r;
        v[q] = HQR_AT(A, (gi < m) ? gi : m - 1, c0 + ((c < ncol) ? c : 0), lda);
    }
}

HQR_DEV void tile_store(double (*M)[LD65], double (&v)[16], int64_t m, int64_t r0, int ncol, int tid)
{
#pragma unroll
    for (int q = 0; q < 16; ++q) pin_f64(v[q]);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int idx = tid + 256 * q, c = idx / 64, r = idx % 64;
        M[r][c] = (r0 + r < m && c < ncol) ? v[q] : 0.0;
    }
}

// M[r][c] = V[r0 + r][c] of the panel starting at cv (width NB; unit lower
// triangle with up on the diagonal in its top block), zero for rows >= m.
// The issue half loads A's entries and up; the store half applies the
// triangle.
HQR_DEV void vtile_issue(double (&v)[16], double (&u)[16], const double *A, int64_t lda, const double *up, int64_t m,
                         int64_t r0, int cv, int tid)
{
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int idx = tid + 256 * q, c = idx / 64, r = idx % 64;
        const int64_t gi = r0 + r;
        v[q] = HQR_AT(A, (gi < m) ? gi : m - 1, cv + c, lda);
        u[q] = up[cv + c];
    }
}

HQR_DEV void vtile_store(double (*M)[LD65], double (&v)[16], double (&u)[16], int64_t m, int64_t r0, int cv, int tid)
{
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        pin_f64(v[q]);
        pin_f64(u[q]);
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int idx = tid + 256 * q, c = idx / 64, r = idx % 64;
        const int64_t d = r0 + r - cv;   // row offset from the panel's first row
        const double e = (d < c) ? 0.0 : ((d == c) ? u[q] : v[q]);
        M[r][c] = (r0 + r < m) ? e : 0.0;
    }
}

// A 64 x 64 row-major matrix into LDS in two halves (transposed when TRANS),
// so that its loads can be issued together with a tile's.
HQR_DEV void mat64_issue(double (&v)[16], const double *src, int tid)
{
#pragma unroll
    for (int t = 0; t < 16; ++t) v[t] = src[tid + 256 * t];
}

template <bool TRANS>
HQR_DEV void mat64_store(double (*M)[LD65], double (&v)[16], int tid)
{
#pragma unroll
    for (int t = 0; t < 16; ++t) pin_f64(v[t]);
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const int idx = tid + 256 * t;
        if (TRANS)
            M[idx % NB][idx / NB] = v[t];
        else
            M[idx / NB][idx % NB] = v[t];
    }
}

// acc[t] (t = 0..3) += sign * A[16w:16w+16][:] * B[:][16t:16t+16] over k = 0..63
HQR_DEV void mm64_acc(f64x4 (&acc)[4], const double (*A)[LD65], const double (*B)[LD65], double sign, int lane, int w)
{
#pragma unroll 4
    for (int k0 = 0; k0 < NB; k0 += 4) {
        const int kr = k0 + (lane >> 4);
        const double a = sign * A[16 * w + (lane & 15)][kr];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, B[kr][16 * t + (lane & 15)], acc[t], 0, 0, 0);
    }
}

// acc[t] = Z^T Z (rows 16w.., column tile t) for a 64 x 64 LDS tile Z
HQR_DEV void gram64(f64x4 (&acc)[4], const double (*Z)[LD65], int lane, int w)
{
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int k0 = 0; k0 < NB; k0 += 4) {
        const int kr = k0 + (lane >> 4);
        const double a = Z[kr][16 * w + (lane & 15)];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Z[kr][16 * t + (lane & 15)], acc[t], 0, 0, 0);
    }
}

// D-layout accumulators of a full 64 x 64 product -> row-major global
HQR_DEV void st64_global(double *out, const f64x4 (&acc)[4], int lane, int w)
{
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) out[(16 * w + 4 * r + (lane >> 4)) * NB + 16 * t + (lane & 15)] = acc[t][r];
}

// ------------------------------------------------- exact one-workgroup panel
// The one-reflector-at-a-time loop on the panel (the arithmetic of the
// per-column launches, the dot products split over NG row groups), streamed
// from global memory by 64 NG threads, followed by T from V^T V.  Used when a
// panel is flagged (structurally exact reflectors, or conditioning beyond
// what two CholeskyQR passes repair).
struct ExactArgs {
    double *A;
    int64_t lda;
    int64_t m;
    int c0, bw;
    double *up;
    double *T;
};

template <int NG>
HQR_DEV void exact_panel(const ExactArgs &p, int tid, double (*red)[PW], double *wsh, double *sc, double (*G)[LD65],
                         double (*Ts)[LD65], double *tau, double *tmp)
{
    constexpr int NT = 64 * NG;
    const int j = tid & 63, g = tid >> 6;
    const int bw = p.bw, c0 = p.c0;
    const int64_t m = p.m;
    __syncthreads();
    for (int k = 0; k < bw; ++k) {
        const int64_t pr = (int64_t)c0 + k;
        // partial dots x . a_j over rows > pr, plus max|x| and #nonzero
        double acc = 0.0, mx = 0.0, nz = 0.0;
        for (int64_t i = pr + 1 + g; i < m; i += NG) {
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
                for (int q = 0; q < NG; ++q) v = fmax(v, red[q][NB]);
            } else {
                for (int q = 0; q < NG; ++q) v += red[q][tid];
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
                for (int64_t i = pr + g; i < m; i += NG) {
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
    for (int e = tid; e < NB * NB; e += NT) {
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
    for (int e = tid; e < NB * NB; e += NT) p.T[e] = Ts[e / NB][e % NB];
}


__global__ void __launch_bounds__(256) cqr_gram1_kernel(Gram1Args p)
{
    __shared__ double M0[NB][LD65];
    __shared__ double M1[NB][LD65];
    __shared__ double M2[NB][LD65];
    __shared__ unsigned long long msk;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int bw = p.bw, t = blockIdx.x;
    const int64_t rbase = p.upd ? (int64_t)p.cp : (int64_t)p.c0;
    const int64_t r0 = rbase + 64 * (int64_t)t;
    const bool flagged = *((volatile int *)p.flag) != 0;
    if (tid == 0) msk = 0ull;
    // M0 = C tile (panel columns); with the update M1 = V tile, M2 = W; all
    // loads are issued before the first wait
    {
        double cv[16], vv[16], uv[16], wv[16];
        tile_issue(cv, p.A, p.lda, p.m, r0, p.c0, bw, tid);
        if (p.upd) {
            vtile_issue(vv, uv, p.A, p.lda, p.up, p.m, r0, p.cp, tid);
            mat64_issue(wv, p.Wt, tid);
        }
        tile_store(M0, cv, p.m, r0, bw, tid);
        if (p.upd) {
            vtile_store(M1, vv, uv, p.m, r0, p.cp, tid);
            mat64_store<true>(M2, wv, tid);
        }
    }
    __syncthreads();
    if (p.upd) {
        f64x4 acc[4];
        // C -= V W: each wave reads and rewrites only its own 16 rows of M0
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = ld_blk(M0, 16 * w, 16 * q, lane);
        mm64_acc(acc, M1, M2, -1.0, lane, w);
#pragma unroll
        for (int q = 0; q < 4; ++q) st_blk(M0, 16 * w, 16 * q, acc[q], 1.0, lane);
        __syncthreads();
        for (int idx = tid; idx < 64 * NB; idx += 256) {
            const int c = idx / 64, r = idx % 64;
            const int64_t gi = r0 + r;
            if (gi < p.m && c < bw) HQR_AT(p.A, gi, p.c0 + c, p.lda) = M0[r][c];
        }
    }
    if (flagged) return;                 // the exact loop factors this panel
    if (p.upd && t == 0) return;         // rows above the panel
    const int gidx = p.upd ? t - 1 : t;
    unsigned long long mymask = 0ull;
    for (int idx = tid; idx < 64 * NB; idx += 256) {
        const int c = idx / 64, r = idx % 64;
        const int64_t gi = r0 + r;
        if (c < bw && gi > (int64_t)p.c0 + c && gi < p.m && M0[r][c] != 0.0) mymask |= (1ull << c);
    }
    if (mymask) atomicOr(&msk, mymask);
    f64x4 acc[4];
    gram64(acc, M0, lane, w);
    st64_global(p.gpart + (size_t)gidx * NB * NB, acc, lane, w);
    __syncthreads();
    if (tid == 0) p.mask[gidx] = msk;
}


__global__ void __launch_bounds__(256) cqr_gram2_kernel(Gram2Args p)
{
    __shared__ double X[NB][LD65];
    __shared__ double Y[NB][LD65];
    __shared__ double Ri[NB][LD65];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (*((volatile int *)p.flag)) return;
    const int t = blockIdx.x;
    const int64_t r0 = (int64_t)p.c0 + 64 * (int64_t)t;
    {
        double xv[16], rv[16];
        tile_issue(xv, p.A, p.lda, p.m, r0, p.c0, p.bw, tid);
        mat64_issue(rv, p.r1inv, tid);
        tile_store(X, xv, p.m, r0, p.bw, tid);
        mat64_store<false>(Ri, rv, tid);
    }
    __syncthreads();
    mm64(Y, X, Ri, lane, w);
    __syncthreads();
    if (t == 0)
        for (int idx = tid; idx < NB * NB; idx += 256) {
            const int r = idx / NB, c = idx % NB;
            p.q1top[idx] = (r < p.bw && c < p.bw) ? Y[r][c] : 0.0;
        }
    f64x4 acc[4];
    gram64(acc, Y, lane, w);
    st64_global(p.gpart + (size_t)t * NB * NB, acc, lane, w);
}


__global__ void __launch_bounds__(256) gram_reduce_kernel(GredArgs p)
{
    __shared__ double part[4][64];
    const int tid = threadIdx.x, e = blockIdx.x * 64 + (tid & 63), g4 = tid >> 6;
    if (p.flag && *((volatile int *)p.flag)) return;
    // thread (e, g4) sums partials q = g4, g4 + 4, ... in that order; 16
    // loads at a time are issued before any is used (clamped, zeroed after)
    double s = 0.0;
    for (int q0 = g4; q0 < p.ngroups; q0 += 64) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int q = q0 + 4 * u;
            v[u] = p.gpart[(size_t)((q < p.ngroups) ? q : g4) * NB * NB + e];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) pin_f64(v[u]);
#pragma unroll
        for (int u = 0; u < 16; ++u) s += (q0 + 4 * u < p.ngroups) ? v[u] : 0.0;
    }
    part[g4][tid & 63] = s;
    __syncthreads();
    if (tid < 64) p.G[e] = ((part[0][tid] + part[1][tid]) + part[2][tid]) + part[3][tid];
    if (p.with_mask && blockIdx.x == 0 && tid >= 64 && tid < 128) {
        // OR of the masks: 64 lanes, strided loads all in flight, then a
        // butterfly over the wave
        const int l = tid - 64;
        unsigned long long all = 0ull;
        for (int q = l; q < p.ngroups; q += 64) all |= p.mask[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const unsigned lo = (unsigned)all, hi = (unsigned)(all >> 32);
            all |= (unsigned long long)(unsigned)__shfl_xor((int)lo, off) |
                   ((unsigned long long)(unsigned)__shfl_xor((int)hi, off) << 32);
        }
        if (l == 0) *p.mask_all = all;
    }
}

// ------------------------------------ Cholesky of a near-identity Gram matrix
// For G = I + E with every |E_ij| <= CQR_SERIES_TAU, the upper factor is
// R = I + X with X + X^T + X^T X = E.  Writing Phi(M) for the strict upper
// part of a symmetric M plus half its diagonal, X0 = Phi(E) and
// X1 = Phi(E - X0^T X0) satisfy ||X1 - X||_F <= 2 eps^3 (eps = ||E||_F <=
// 64 tau), and R^{-1} = I - X1 + X1^2 up to eps^3: below 3e-22 for
// tau = 2^-30, far under FP64 rounding.  Three block products on MFMA replace
// the 64 sequential pivots.  The second CholeskyQR pass meets this bound
// unless the panel's condition number exceeds about 1e3 (its Gram matrix is
// then I + O(kappa^2 u)).
constexpr double CQR_SERIES_TAU = 0x1p-30;

// On entry (after a barrier) G holds I + E in full and X holds Phi(E).  On
// exit G = R and X = R^{-1} (upper, zeros below), rdiag = diag(R); ends with
// a barrier.
HQR_DEV void chol_near_identity(double (*G)[LD65], double (*X)[LD65], double *rdiag, int lane, int w)
{
    const int i16 = lane & 15, kk = lane >> 4;
    // P = X0^T X0 on the wave's upper blocks (w, s >= w): k-blocks 0..w
    f64x4 acc[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        acc[s] = f64x4{0.0, 0.0, 0.0, 0.0};
        if (s < w) continue;
        for (int kb = 0; kb <= w; ++kb) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = 16 * kb + 4 * q + kk;
                acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(X[k][16 * w + i16], X[k][16 * s + i16], acc[s], 0, 0, 0);
            }
        }
    }
    // X1 = Phi(E - P) on the wave's rows, kept in registers
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = 16 * w + 4 * q + kk, c = 16 * s + i16;
            const double e = (G[r][c] - ((r == c) ? 1.0 : 0.0)) - acc[s][q];
            acc[s][q] = (r > c) ? 0.0 : ((r == c) ? 0.5 * e : e);
        }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = 16 * w + 4 * q + kk, c = 16 * s + i16;
            X[r][c] = acc[s][q];
            G[r][c] = ((r == c) ? 1.0 : 0.0) + acc[s][q];
            if (r == c) rdiag[r] = 1.0 + acc[s][q];
        }
    __syncthreads();
    // X = I - X1 + X1^2 (X1^2 upper; the lower blocks keep X1's zeros)
    f64x4 sq[4];
    mm_upper_upper(sq, [&](int r, int c) { return X[r][c]; }, [&](int r, int c) { return X[r][c]; }, lane, w);
    __syncthreads();
    for_uu(sq, [&](int r, int c, double v) { X[r][c] = (((r == c) ? 1.0 : 0.0) - X[r][c]) + v; }, lane, w);
    __syncthreads();
}


// One workgroup, 256 threads.
//   pass 1: R1 = chol(G), R1^{-1}; flags the panel (structurally exact
//           reflectors, or a pivot below CQR_RATIO).
//   flagged panel, pass 2: the exact one-reflector loop instead.
//   pass 2: R2 = chol(G2), Q_top = Q1_top R2^{-1}, LU of Q_top - S, then
//           R_house = S R2 R1, up, the stored tails of the top block, T_V
//           and W^{-1} = R1^{-1} R2^{-1} U^{-1} diag(up).
__global__ void __launch_bounds__(256) cqr_chol_kernel(CholArgs p)
{
    __builtin_amdgcn_s_setprio(3);   // single workgroup on the critical path: issue ahead of co-resident bulk waves
    __shared__ double M0[NB][LD65];
    __shared__ double M1[NB][LD65];
    __shared__ double M2[NB][LD65];
    __shared__ double M3[NB][LD65];
    __shared__ double DU[NB][17], DL[NB][17];
    __shared__ double gdiag[NB], rdiag[NB], sgn[NB], udiag[NB], upv[NB], rupv[NB];
    __shared__ int bad, structural_sh, nonid_sh;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int bw = p.bw;
    if (tid == 0) {
        structural_sh = 0;
        nonid_sh = 0;
        bad = 0;
    }
    __shared__ double red[4][PW], wsh[NB], sc[4];
    const ExactArgs ex{p.A, p.lda, p.m, p.c0, bw, p.up, p.T};
    if (*((volatile int *)p.flag)) {
        // flagged up front or in pass 1: the exact loop factors the panel
        if (p.pass == 2) exact_panel<4>(ex, tid, red, wsh, sc, M0, M1, gdiag, rdiag);
        return;
    }
    int tsi = 0;
#define HQR_TS()                                                                 \
    do {                                                                         \
        if (p.tstamp && tid == 0) p.tstamp[tsi] = (long long)wall_clock64();     \
        ++tsi;                                                                   \
    } while (0)
    HQR_TS();
    // G -> M0, Q1_top -> M2 and R1 -> M3 (the last two idle until after the
    // Cholesky factorization; read in pass 1 too, where they are unused):
    // all 48 loads of a thread are issued before the first is waited for
    {
        double gl[16], ql[16], rl[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const int idx = tid + 256 * t;
            gl[t] = p.G[idx];
            ql[t] = p.q1top[idx];
            rl[t] = p.r1[idx];
        }
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            pin(gl[t]);
            pin(ql[t]);
            pin(rl[t]);
        }
        int far = 0;   // an entry of G - I beyond CQR_SERIES_TAU
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const int idx = tid + 256 * t, i = idx / NB, j = idx % NB;
            const double g = (i < bw && j < bw) ? gl[t] : 0.0;
            M0[i][j] = g;
            M2[i][j] = ql[t];
            M3[i][j] = rl[t];
            if (p.pass == 2) {
                const double e = g - ((i == j) ? 1.0 : 0.0);
                far |= !(fabs(e) <= CQR_SERIES_TAU);
                M1[i][j] = (i < j) ? e : ((i == j) ? 0.5 * e : 0.0);   // Phi(E)
            }
        }
        if (far) nonid_sh = 1;
    }
    int structural = 0;
    if (p.pass == 1 && tid == 0) {
        const unsigned long long all = *p.mask_all;
        const unsigned long long need = (bw == 64) ? ~0ull : ((1ull << bw) - 1ull);
        structural = ((all & need) != need);
        structural_sh = structural;
    }
    __syncthreads();
    // pass 2 of a full-width panel whose Gram matrix is within the series
    // bound of the identity: no sequential pivots
    const bool series = p.pass == 2 && bw == NB && !nonid_sh;
    HQR_TS();
    if (series)
        chol_near_identity(M0, M1, rdiag, lane, w);
    else
        chol64_dpp(M0, M1, bw, lane, w, CQR_RATIO, gdiag, rdiag, &bad);
    HQR_TS();
    // 1: an exactly zero column tail (only the exact loop keeps H_k = I);
    // 2: a pivot below the ratio (a TSQR panel can still take over)
    if (tid == 0 && (bad || structural)) *((volatile int *)p.flag) = structural ? 1 : 2;
    __syncthreads();
    if (bad && p.pass == 2) {
        exact_panel<4>(ex, tid, red, wsh, sc, M0, M1, gdiag, rdiag);
        return;
    }
    if (bad || structural_sh) return;
    if (!series) inv_upper_levels(M1, M0, lane, w);     // M1 = R^{-1} of this pass
    HQR_TS();

    if (p.pass == 1) {
        for (int idx = tid; idx < NB * NB; idx += 256) {
            p.r1[idx] = M0[idx / NB][idx % NB];
            p.r1inv[idx] = M1[idx / NB][idx % NB];
        }
        return;
    }

    // ---- pass 2: M0 = R2, M1 = R2^{-1}, M2 = Q1_top, M3 = R1
    {
        f64x4 qacc[4];
        mm_full_upper(qacc, [&](int r, int c) { return M2[r][c]; }, [&](int r, int c) { return M1[r][c]; }, lane, w);
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 4; ++s) st_blk(M2, 16 * w, 16 * s, qacc[s], 1.0, lane);  // M2 = Q_top
    }
    HQR_TS();
    // LU of Q_top - S in M2; diagonal blocks of U^{-1} -> DU, of L^{-1} -> DL
    lu64_dpp(M2, DU, DL, lane, w, sgn, udiag);
    HQR_TS();
    // R = R2 R1; R_house = S R into the upper triangle of the panel's top block
    {
        f64x4 racc[4];
        mm_upper_upper(racc, [&](int r, int c) { return M0[r][c]; }, [&](int r, int c) { return M3[r][c]; }, lane, w);
        for_uu(racc, [&](int r, int c, double v) {
            if (r <= c && c < bw) HQR_AT(p.A, (int64_t)p.c0 + r, p.c0 + c, p.lda) = sgn[r] * v;
        }, lane, w);
    }
    if (tid < bw) {
        const double rkk = sgn[tid] * rdiag[tid] * M3[tid][tid];  // diag of S R2 R1
        const double tau = -udiag[tid] * sgn[tid];                // = 1 + |pivot|
        upv[tid] = -tau * rkk;
        rupv[tid] = 1.0 / upv[tid];   // nonzero: tau >= 1 and R_kk != 0 on this path
    }
    __syncthreads();
    // diagonal blocks of U^{-1} -> M0, of L^{-1} -> M3; then the rest
    for (int idx = tid; idx < NB * 16; idx += 256) {
        const int r = idx >> 4, cc = idx & 15, c = 16 * (r >> 4) + cc;
        M0[r][c] = DU[r][cc];
        M3[r][c] = DL[r][cc];
    }
    inv_lu_levels(M0, M3, M2, lane, w);                 // M0 = U^{-1}, M3 = L^{-1}
    HQR_TS();
    // R1^{-1} is fetched now (into M1 once V1 no longer needs R2^{-1} there),
    // so its latency overlaps the two products below
    double r1i[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) r1i[t] = p.r1inv[tid + 256 * t];
    // T_Y = -(U S) L^{-T}, T_V = T_Y / (up_i up_j) -> global; V1 = R2^{-1} U^{-1}
    f64x4 vacc[4];
    {
        f64x4 tacc[4];
        mm_upper_upper(tacc, [&](int r, int c) { return (c >= r && c < bw) ? M2[r][c] * sgn[c] : 0.0; },
                       [&](int r, int c) { return M3[c][r]; }, lane, w);
        for (int idx = tid; idx < NB * NB; idx += 256) {
            const int i = idx / NB, j = idx % NB;
            if (!(i <= j && j < bw)) p.T[idx] = 0.0;
        }
        for_uu(tacc, [&](int r, int c, double v) {
            if (r <= c && c < bw) p.T[r * NB + c] = -v * (rupv[r] * rupv[c]);
        }, lane, w);
    }
    HQR_TS();
    mm_upper_upper(vacc, [&](int r, int c) { return M1[r][c]; }, [&](int r, int c) { return M0[r][c]; }, lane, w);
    __syncthreads();
    // M0 = V1 (its blocks below the diagonal are still U^{-1}'s zeros), M1 = R1^{-1}
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int e = uu_slot(w, s);
        if (e >= 0) st_blk(M0, 16 * (e >> 2), 16 * (e & 3), vacc[s], 1.0, lane);
    }
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const int idx = tid + 256 * t;
        M1[idx / NB][idx % NB] = r1i[t];
    }
    __syncthreads();
    HQR_TS();
    // W^{-1} = R1^{-1} V1 diag(up) -> global (zero beyond bw and below the diagonal)
    {
        f64x4 wacc[4];
        mm_upper_upper(wacc, [&](int r, int c) { return M1[r][c]; }, [&](int r, int c) { return M0[r][c]; }, lane, w);
        for (int idx = tid; idx < NB * NB; idx += 256) {
            const int i = idx / NB, j = idx % NB;
            if ((i >> 4) > (j >> 4) || j >= bw) p.winv[idx] = 0.0;
        }
        for_uu(wacc, [&](int r, int c, double v) {
            if (c < bw) p.winv[r * NB + c] = v * upv[c];
        }, lane, w);
    }
    HQR_TS();
    // stored tails of the top block: L[i][j] * up_j (strict lower)
    for (int idx = tid; idx < NB * NB; idx += 256) {
        const int c = idx / NB, r = idx % NB;
        if (r > c && r < bw) HQR_AT(p.A, (int64_t)p.c0 + r, p.c0 + c, p.lda) = M2[r][c] * upv[c];
    }
    if (tid < bw) p.up[p.c0 + tid] = upv[tid];
    HQR_TS();
#undef HQR_TS
}


__global__ void __launch_bounds__(256) cqr_finish_kernel(FinArgs p)
{
    __shared__ double X[NB][LD65];
    __shared__ double Wi[NB][LD65];
    __shared__ double Y[NB][LD65];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (*((volatile int *)p.flag)) return;
    const int64_t r0 = (int64_t)p.c0 + p.bw + (int64_t)blockIdx.x * 64;
    {
        double wv[16], xv[16];
        mat64_issue(wv, p.winv, tid);
        tile_issue(xv, p.A, p.lda, p.m, r0, p.c0, p.bw, tid);
        mat64_store<false>(Wi, wv, tid);
        tile_store(X, xv, p.m, r0, p.bw, tid);
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


__global__ void __launch_bounds__(256) narrow_vtx_kernel(NarrowArgs p)
{
    __shared__ double M0[NB][LD65];
    __shared__ double M1[NB][LD65];
    __shared__ double M2[NB][LD65];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int t = blockIdx.x;
    const int64_t r0 = (int64_t)p.c0 + 64 * (int64_t)t;
    const bool flagged = *((volatile int *)p.flag) != 0;
    const bool fin = (t > 0) && !flagged;
    // M0 = V rows (top block: unit lower with up on the diagonal), or A_bot;
    // M2 = C; M1 = W^{-1} when finishing
    {
        // the V/A_bot tile and up are loaded alike (the triangle is applied
        // when t == 0), W^{-1} always: every load is issued before the first wait
        double av[16], uv[16], cv[16], wv[16];
        vtile_issue(av, uv, p.A, p.lda, p.up, p.m, r0, p.c0, tid);
        tile_issue(cv, p.A, p.lda, p.m, r0, p.c0 + NB, p.nc, tid);
        mat64_issue(wv, p.winv, tid);
#pragma unroll
        for (int q = 0; q < 16; ++q) pin_f64(wv[q]);   // keeps its loads out of the conditional store
        if (t == 0)
            vtile_store(M0, av, uv, p.m, r0, p.c0, tid);
        else
            tile_store(M0, av, p.m, r0, NB, tid);
        tile_store(M2, cv, p.m, r0, p.nc, tid);
        if (fin) mat64_store<false>(M1, wv, tid);
    }
    __syncthreads();
    double (*V)[LD65] = M0;
    if (fin) {
        // V rows = A_bot W^{-1}: into M1's place after the product
        f64x4 acc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = f64x4{0.0, 0.0, 0.0, 0.0};
        mm64_acc(acc, M0, M1, 1.0, lane, w);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) st_blk(M1, 16 * w, 16 * q, acc[q], 1.0, lane);
        __syncthreads();
        V = M1;
        for (int idx = tid; idx < 64 * NB; idx += 256) {
            const int c = idx / 64, r = idx % 64;
            const int64_t gi = r0 + r;
            if (gi < p.m) HQR_AT(p.A, gi, p.c0 + c, p.lda) = M1[r][c];
        }
    }
    // partial V_t^T C_t
    {
        f64x4 acc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
        for (int k0 = 0; k0 < NB; k0 += 4) {
            const int kr = k0 + (lane >> 4);
            const double a = V[kr][16 * w + (lane & 15)];
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, M2[kr][16 * q + (lane & 15)], acc[q], 0, 0, 0);
        }
        // stored transposed, [column j][reflector i], for xw_reduce_kernel
        double *out = p.gpart + (size_t)t * NB * NB;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) out[(16 * q + (lane & 15)) * NB + 16 * w + 4 * r + (lane >> 4)] = acc[q][r];
    }
}


__global__ void __launch_bounds__(256) xw_reduce_kernel(XwArgs p)
{
    __shared__ double part[4][64];
    __shared__ double xc[64];
    const int tid = threadIdx.x, i = tid & 63, g4 = tid >> 6, j = blockIdx.x;
    const size_t e = (size_t)j * NB + i;
    double s = 0.0;
    for (int q0 = g4; q0 < p.parts; q0 += 64) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int q = q0 + 4 * u;
            v[u] = p.gpart[(size_t)((q < p.parts) ? q : g4) * NB * NB + e];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) pin_f64(v[u]);
#pragma unroll
        for (int u = 0; u < 16; ++u) s += (q0 + 4 * u < p.parts) ? v[u] : 0.0;
    }
    part[g4][i] = s;
    __syncthreads();
    if (tid < 64) xc[i] = ((part[0][i] + part[1][i]) + part[2][i]) + part[3][i];
    __syncthreads();
    double tl[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) tl[u] = p.T[(16 * g4 + u) * NB + i];
#pragma unroll
    for (int u = 0; u < 16; ++u) pin_f64(tl[u]);
    double wv = 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int l = 16 * g4 + u;
        wv = (l <= i) ? fma(tl[u], xc[l], wv) : wv;
    }
    part[g4][i] = wv;
    __syncthreads();
    if (tid < 64) p.Wt[e] = ((part[0][i] + part[1][i]) + part[2][i]) + part[3][i];
}

// T of a stored panel (compact WY, T upper, Q_panel^T = I + V T^T V^T with
// T[k][k] = tau_k = -1/b_k) from G = V^T V, the splits' partial sums of the
// V^T X pass.  T^{-1} = diag(1/tau) + the strict upper triangle of G, so T
// is the inverse of that upper triangular matrix: its four 16 x 16 diagonal
// blocks by the column recurrence T[i][k] = -tau_k sum_{l=i}^{k-1} T[i][l]
// G[l][k] (one wave each, lane i < 16 keeping row i and adding T[i][l]
// G[l][k] into every later column's sum once T[i][l] is final), then the
// blocks above them by distance from the diagonal on MFMA
// (inv_upper_levels).  Zero taus (identity reflectors, columns past bw) give
// zero rows and columns.  One workgroup of 256 threads.
__global__ void __launch_bounds__(256) tfactor_kernel(TArgs p)
{
    __shared__ double G[NB][LD65];
    __shared__ double Ts[NB][LD65];
    __shared__ double tau[NB];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // G = the splits' partial V^T V summed in split order; a thread's 16
    // elements are loaded together for each split
    constexpr int EPT = NB * NB / 256;
    double gs[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) gs[e] = 0.0;
#pragma unroll 4
    for (int q = 0; q < p.nsplit; ++q) {
        const double *src = p.wpart + (size_t)q * NB * p.nxpad;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int idx = tid + 256 * e, i = idx / NB, j = idx - i * NB;
            gs[e] += (i < p.bw && j < p.bw) ? src[(size_t)i * p.nxpad + j] : 0.0;
        }
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int idx = tid + 256 * e;
        G[idx / NB][idx % NB] = gs[e];
    }
    if (tid < NB) {
        double t = 0.0;
        if (tid < p.bw) {
            const double u = p.up[p.c0 + tid];
            const double rkk = HQR_AT(p.A, (int64_t)p.c0 + tid, p.c0 + tid, p.lda);
            t = (u == 0.0) ? 0.0 : -1.0 / (u * rkk);
        }
        tau[tid] = t;
    }
    __syncthreads();
    if (lane < 16) {
        const int b0 = 16 * w, i = lane;
        double acc[16], trow[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) acc[k] = 0.0;
#pragma unroll
        for (int l = 0; l < 16; ++l) {
            trow[l] = (i > l) ? 0.0 : ((i == l) ? tau[b0 + l] : -tau[b0 + l] * acc[l]);
#pragma unroll
            for (int k = l + 1; k < 16; ++k) acc[k] = fma(trow[l], G[b0 + l][b0 + k], acc[k]);
        }
#pragma unroll
        for (int l = 0; l < 16; ++l) Ts[b0 + i][b0 + l] = trow[l];
    }
    inv_upper_levels(Ts, G, lane, w);
    for (int idx = tid; idx < NB * NB; idx += 256) p.T[idx] = Ts[idx / NB][idx % NB];
}

} // namespace hqr
