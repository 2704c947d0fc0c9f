// hqr_blocked.hpp -- blocked in-place Householder QR for problems that do not
// fit one workgroup.
//
// The matrix is processed in panels of NB columns (the coarsened "Task 1"
// of the paper's Alg. 3: alpha pivots generated back to back) followed by a
// blocked trailing update (the coarsened "Task 2" of Alg. 4, all of a panel's
// reflectors applied to the trailing columns at once).  On the GPU the
// trailing update is a compact-WY contraction on FP64 MFMA:
//     W  = V^T X            (split over rows, partial sums per split)
//     W' = T^T W            (T upper triangular, Q_panel = I - V T V^T)
//     X <- X - V W'
// where X = [trailing columns of A | B].  V's columns are the stored
// reflectors: v_k = (0..0, up_k, A[k+1:m, k]) with up_k kept in `up`.
//
// Panel factorization, one launch per pivot (panel_col_kernel): launch k
// applies reflector k-1 (derived from the reduced partial dot products of
// launch k-1) to every row chunk, then writes this launch's partial dot
// products of pivot column k, so every reflector is derived from the same
// data, in the same order, by every workgroup.
#pragma once

#include "hqr_args.hpp"

#define HQR_HD __host__ __device__
#include "hqr_refine_rule.hpp"

namespace hqr {



__global__ void __launch_bounds__(256) panel_col_kernel(PanelArgs p)
{
    __shared__ double S[NB][PC_ROWS + 1];
    __shared__ double red[4][PW];
    __shared__ double wsh[NB];
    __shared__ double scal[4];

    const int tid = threadIdx.x, lane = tid & 63, g = tid >> 6;
    const int bw = p.bw, k = p.k, c0 = p.c0;
    const int64_t row_lo = (int64_t)c0 + (int64_t)blockIdx.x * PC_ROWS;
    const int64_t mp = p.m;
    const int nrow = (int)min<int64_t>((int64_t)PC_ROWS, mp - row_lo);

    // load my chunk (column-major in LDS)
    for (int idx = tid; idx < nrow * bw; idx += 256) {
        const int j = idx / nrow, r = idx - j * nrow;
        S[j][r] = HQR_AT(p.A, row_lo + r, c0 + j, p.lda);
    }
    __syncthreads();

    // ---- apply reflector k-1
    if (k > 0) {
        const int kp = k - 1;
        const int par = kp & 1;
        const double *X = p.xbuf + (size_t)par * p.nchunk * PW;
        const double *prow = p.pbuf + (size_t)par * NB;
        // reduced partials, same order in every workgroup: thread (value v,
        // quarter g4) sums chunks q = g4, g4+4, ...; quarters then summed 0..3
        for (int t = tid; t < 4 * PW; t += 256) {
            const int v = t % PW, g4 = t / PW;
            double acc4 = 0.0;
            if (v == NB) {
                for (int q = g4; q < p.nchunk; q += 4) acc4 = fmax(acc4, X[(size_t)q * PW + v]);
            } else {
#pragma unroll 4
                for (int q = g4; q < p.nchunk; q += 4) acc4 += X[(size_t)q * PW + v];
            }
            red[g4][v] = acc4;
        }
        __syncthreads();
        double d_j = 0.0;
        if (tid < bw) d_j = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
        if (tid == 0) {
            scal[0] = ((red[0][kp] + red[1][kp]) + red[2][kp]) + red[3][kp];
            scal[1] = fmax(fmax(red[0][NB], red[1][NB]), fmax(red[2][NB], red[3][NB]));
            scal[2] = ((red[0][NB + 1] + red[1][NB + 1]) + red[2][NB + 1]) + red[3][NB + 1];
        }
        __syncthreads();
        const double x0 = prow[kp];
        double up_k, s_k;
        if (scal[2] == 0.0) {
            up_k = 0.0;
            s_k = x0;
        } else {
            const double c = fmax(fabs(x0), scal[1]);
            double nu;
            if (norm_fast_path_ok(c)) {
                nu = sqrt(x0 * x0 + scal[0]);
            } else {
                // rare: the partials of this launch's pivot were not scaled;
                // recompute the scaled norm from the tail in global memory
                // (a deterministic single-thread loop, identical in every WG)
                double t = 0.0;
                const int64_t pr = (int64_t)c0 + kp;
                for (int64_t i = pr + 1; i < mp; ++i) {
                    const double y = HQR_AT(p.A, i, c0 + kp, p.lda) / c;
                    t += y * y;
                }
                const double x0c = x0 / c;
                nu = c * sqrt(x0c * x0c + t);
            }
            s_k = (x0 >= 0.0) ? -nu : nu;
            up_k = x0 - s_k;
        }
        const bool skip = (up_k == 0.0);
        const double b_k = up_k * s_k;
        if (tid < NB) wsh[tid] = (!skip && tid > kp && tid < bw) ? (up_k * prow[tid] + d_j) / b_k : 0.0;
        const int64_t prow_g = (int64_t)c0 + kp;
        if (blockIdx.x == 0 && tid == 0) p.up[c0 + kp] = up_k;
        __syncthreads();
        // rows of my chunk that are >= the pivot row
        if (!skip) {
            for (int idx = tid; idx < nrow * bw; idx += 256) {
                const int j = idx / nrow, r = idx - j * nrow;
                const int64_t gi = row_lo + r;
                if (j <= kp || gi < prow_g) continue;
                const double v = (gi == prow_g) ? up_k : S[kp][r];
                S[j][r] += wsh[j] * v;
            }
        }
        if (prow_g >= row_lo && prow_g < row_lo + nrow && tid == 0) S[kp][prow_g - row_lo] = s_k;
        __syncthreads();
    }

    // ---- partials of pivot column k (x = A[c0+k+1 : m, c0+k])
    if (k < bw) {
        const int par = k & 1;
        double *X = p.xbuf + (size_t)par * p.nchunk * PW;
        double *prow = p.pbuf + (size_t)par * NB;
        const int64_t pr = (int64_t)c0 + k;
        // thread (column j = lane, row group g)
        double acc = 0.0, mx = 0.0, nz = 0.0;
        for (int r = g; r < nrow; r += 4) {
            const int64_t gi = row_lo + r;
            if (gi <= pr) continue;
            const double xi = S[k][r];
            if (lane < bw) acc += xi * S[lane][r];
            mx = fmax(mx, fabs(xi));
            nz += (xi != 0.0) ? 1.0 : 0.0;
        }
        red[g][lane] = acc;
        if (lane == 0) {
            red[g][NB] = mx;
            red[g][NB + 1] = nz;
        }
        __syncthreads();
        if (tid < PW) {
            double v;
            if (tid == NB) v = fmax(fmax(red[0][NB], red[1][NB]), fmax(red[2][NB], red[3][NB]));
            else v = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
            X[(size_t)blockIdx.x * PW + tid] = v;
        }
        if (pr >= row_lo && pr < row_lo + nrow && tid < NB)
            prow[tid] = (tid < bw) ? S[tid][pr - row_lo] : 0.0;
    }
    __syncthreads();

    // store the chunk back
    for (int idx = tid; idx < nrow * bw; idx += 256) {
        const int j = idx / nrow, r = idx - j * nrow;
        HQR_AT(p.A, row_lo + r, c0 + j, p.lda) = S[j][r];
    }
}


// V element (global row gi >= c0, panel column c) with both candidate loads
// issued unconditionally (no branch around a load, so a tile's loads stay in
// flight together); gi and c must address the matrix.
HQR_DEV double v_elem_nb(const double *A, int64_t lda, const double *up, int c0, int64_t gi, int c)
{
    const double a = HQR_AT(A, gi, c0 + c, lda);
    const double u = up[c0 + c];
    const int64_t d = gi - c0;
    return (d < c) ? 0.0 : ((d == c) ? u : a);
}

// A 64 x 64 row-major matrix from global memory into LDS (transposed when
// TRANS), by 256 threads: a thread's 16 loads are all issued before the first
// is waited for (a plain copy loop waits on each load in turn).
template <bool TRANS, int LD>
HQR_DEV void ld64_lds(double (*M)[LD], const double *src, int tid)
{
    double v[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) v[t] = src[tid + 256 * t];
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


// F32: operands rounded to FP32, FP32 MFMA with FP32 accumulation (the
// partial sums are stored widened to FP64).  WITHV: the first bw X columns
// are the panel's own V columns (the per-column panel mode forms V^T V there).
//
// Register budget: the prefetch loads are unconditional, with rows and
// columns clamped into the matrix and column addresses formed at each fetch
// (no per-thread pointer tables); the rows past the split, the columns past
// nx and the triangle of V near the pivot rows are applied by selects when
// the chunk is stored.  This keeps two waves per SIMD.
template <bool F32, bool WITHV>
__global__ void __launch_bounds__(256, 2) vtx_kernel(VtxArgs p)
{
    __shared__ double Vs[KC][NB + 1];
    __shared__ double Xs[KC][VTX_COLS + 1];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int x0 = blockIdx.x * VTX_COLS;
    const int64_t r_begin = (int64_t)p.c0 + (int64_t)blockIdx.y * p.split_rows;
    const int64_t r_end = min<int64_t>(p.m, r_begin + p.split_rows);

    f64x4 acc[8];
    f32x4 acc32[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
        acc32[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    }

    // staging layout: thread t loads row t % KC of V columns t / KC + 8 q
    // and of X columns x0 + t / KC + 8 q
    constexpr int VPT = KC * NB / 256;       // V elements per thread
    constexpr int XPT = KC * VTX_COLS / 256; // X elements per thread
    const int sr = tid % KC, sc = tid / KC;  // sc in [0, 8)
    const int bwm = p.bw - 1;
    double upq[VPT];                         // up of this thread's V columns
#pragma unroll
    for (int q = 0; q < VPT; ++q) upq[q] = p.up[p.c0 + min(sc + 8 * q, bwm)];
    double vreg[VPT], xreg[XPT];
    auto fetch = [&](int64_t r0) {
        const int64_t gi0 = r0 + sr;
        const int64_t gi = (gi0 < r_end) ? gi0 : r_end - 1;
#pragma unroll
        for (int q = 0; q < VPT; ++q) vreg[q] = HQR_AT(p.A, gi, p.c0 + min(sc + 8 * q, bwm), p.lda);
#pragma unroll
        for (int q = 0; q < XPT; ++q) {
            const int x = min(x0 + sc + 8 * q, p.nx - 1);
            const double *col;
            if (WITHV && x < p.bw) {
                col = p.A + (size_t)(p.c0 + x) * p.lda;
            } else {
                const int xa = WITHV ? x - p.bw : x;
                col = (xa < p.ncA) ? p.A + (size_t)(p.c0 + p.bw + p.aoff + xa) * p.lda
                                   : p.B + (size_t)(xa - p.ncA) * p.ldb;
            }
            xreg[q] = __builtin_nontemporal_load(col + gi);
        }
    };
    // waits for the chunk's loads, then zeroes what lies outside and applies
    // the triangle of V (row offset d from the panel's first row)
    auto finish = [&](int64_t r0) {
#pragma unroll
        for (int q = 0; q < VPT; ++q) pin_f64(vreg[q]);
#pragma unroll
        for (int q = 0; q < XPT; ++q) pin_f64(xreg[q]);
        const int64_t gi0 = r0 + sr;
        const bool ok = gi0 < r_end;
        const int64_t d = gi0 - p.c0;
#pragma unroll
        for (int q = 0; q < VPT; ++q) {
            const int c = sc + 8 * q;
            const double v = (d < c) ? 0.0 : ((d == c) ? upq[q] : vreg[q]);
            vreg[q] = (ok && c < p.bw) ? v : 0.0;
        }
#pragma unroll
        for (int q = 0; q < XPT; ++q) {
            const int x = x0 + sc + 8 * q;
            // WITHV: X column x < bw is V column x, held by this thread as
            // vreg[q] (x < 64 only in tile 0, where x = sc + 8 q)
            double v = xreg[q];
            if (WITHV && q < VPT && x < p.bw) v = vreg[q < VPT ? q : 0];
            xreg[q] = (ok && x < p.nx) ? v : 0.0;
        }
    };
    if (r_begin < r_end) fetch(r_begin);
    for (int64_t r0 = r_begin; r0 < r_end; r0 += KC) {
        finish(r0);
#pragma unroll
        for (int q = 0; q < VPT; ++q) Vs[sr][sc + 8 * q] = vreg[q];
#pragma unroll
        for (int q = 0; q < XPT; ++q) Xs[sr][sc + 8 * q] = xreg[q];
        __syncthreads();
        if (r0 + KC < r_end) fetch(r0 + KC);
#pragma unroll 2
        for (int kk = 0; kk < KC; kk += 4) {
            const int kr = kk + (lane >> 4);
            const double a = Vs[kr][16 * w + (lane & 15)];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const double b = Xs[kr][16 * t + (lane & 15)];
                if (F32)
                    acc32[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(to_f32(a), to_f32(b), acc32[t], 0, 0, 0);
                else
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // FP64 MFMA: D[i][j] at lane j + 16*(i%4), register i/4;
    // FP32 MFMA: D[i][j] at lane j + 16*(i/4), register i%4
    double *out = p.wpart + (size_t)blockIdx.y * NB * p.nxpad;
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = F32 ? 16 * w + 4 * (lane >> 4) + r : 16 * w + 4 * r + (lane >> 4);
            const int x = x0 + 16 * t + (lane & 15);
            if (x < p.nxpad) out[(size_t)i * p.nxpad + x] = F32 ? (double)acc32[t][r] : acc[t][r];
        }
}





__global__ void __launch_bounds__(256) wsolve_kernel(WArgs p)
{
    __shared__ double Ws[NB][WS_COLS + 1];
    __shared__ double Ts[NB][NB + 1];
    const int tid = threadIdx.x;
    const int xb = p.xoff + blockIdx.x * WS_COLS;
    const int xe = p.xoff + p.ncols;
    ld64_lds<false>(Ts, p.T, tid);
    // 1024 partial sums: thread t reduces elements (i = t / 4 + 64 q?) -- four per thread
#pragma unroll
    for (int e4 = 0; e4 < 4; ++e4) {
        const int e = tid + 256 * e4;          // e in [0, 1024)
        const int i = e / WS_COLS, c = e % WS_COLS;
        const int x = xb + c;
        double s = 0.0;
        if (i < p.bw && x < xe) {
            const double *src = p.wpart + (size_t)i * p.nxpad + x;
            const size_t stride = (size_t)NB * p.nxpad;
#pragma unroll 8
            for (int q = 0; q < p.nsplit; ++q) s += src[q * stride];
        }
        Ws[i][c] = s;
    }
    __syncthreads();
#pragma unroll
    for (int e4 = 0; e4 < 4; ++e4) {
        const int e = tid + 256 * e4;
        const int i = e / WS_COLS, c = e % WS_COLS;
        const int x = xb + c;
        if (x >= xe) continue;
        double s = 0.0;
        if (p.tmode == 0) {
            for (int l = 0; l <= i && l < p.bw; ++l) s += Ts[l][i] * Ws[l][c];
        } else {
            for (int l = i; l < p.bw; ++l) s += Ts[i][l] * Ws[l][c];
        }
        p.wp[(size_t)i * p.nxpad + x] = (i < p.bw) ? s : 0.0;
    }
}

__global__ void __launch_bounds__(256) wsolve_narrow_kernel(WArgs p)
{
    __shared__ double Ws[NB][WSN_COLS + 1];
    __shared__ double Ts[NB][NB + 1];
    const int tid = threadIdx.x;
    const int i = tid / WSN_COLS, c = tid % WSN_COLS;
    const int x = p.xoff + blockIdx.x * WSN_COLS + c;
    const int xe = p.xoff + p.ncols;
    ld64_lds<false>(Ts, p.T, tid);
    double s = 0.0;
    if (i < p.bw && x < xe) {
        const double *src = p.wpart + (size_t)i * p.nxpad + x;
        const size_t stride = (size_t)NB * p.nxpad;
#pragma unroll 16
        for (int q = 0; q < p.nsplit; ++q) s += src[q * stride];
    }
    Ws[i][c] = s;
    __syncthreads();
    if (x < xe) {
        double t = 0.0;
        if (p.tmode == 0) {
            for (int l = 0; l <= i && l < p.bw; ++l) t += Ts[l][i] * Ws[l][c];
        } else {
            for (int l = i; l < p.bw; ++l) t += Ts[i][l] * Ws[l][c];
        }
        p.wp[(size_t)i * p.nxpad + x] = (i < p.bw) ? t : 0.0;
    }
}


HQR_DEV double *col_ptr(const UpdArgs &p, int c)
{
    if (c < p.ncA) return p.A + (size_t)(p.c0 + p.bw + p.aoff + c) * p.lda;
    return p.B + (size_t)(c - p.ncA) * p.ldb;
}


// F32: V and W' rounded to FP32, the product accumulated in FP32 by FP32
// MFMA from zero, then subtracted from the FP64 trailing matrix.
template <bool F32>
__global__ void __launch_bounds__(256, 2) update_kernel(UpdArgs p)
{
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = w & 1, wc = w >> 1;
    const int64_t rb = (int64_t)p.c0 + (int64_t)blockIdx.x * UPD_TILE + 64 * wr;
    const int cb = blockIdx.y * UPD_TILE + 64 * wc;
    const int ncols = p.ncA + p.nB;
    if (rb >= p.m || cb >= ncols) return;
    const int li = lane & 15, lk = lane >> 4;
    const bool masked = rb < (int64_t)p.c0 + p.bw; // rows that meet the triangle of V

    // Loads are unconditional: rows and columns are clamped into the matrix.
    // A lane outside it only ever feeds accumulator entries that are never
    // stored, except through k >= bw, which is zeroed after the loads.
    int64_t gr[4];
    bool rok[4];
#pragma unroll
    for (int ti = 0; ti < 4; ++ti) {
        const int64_t gi = rb + 16 * ti + li;
        rok[ti] = gi < p.m;
        gr[ti] = rok[ti] ? gi : p.m - 1;
    }
    f64x4 acc[4][4]; // [column tile][row tile]
    f32x4 acc32[4][4];
    double *cptr[4][4];
    bool cok[4][4];
    // accumulator register r of lane (li, lk) holds column cb + 16 tj + ccol(r), row li
#define HQR_CCOL(r) (F32 ? 4 * lk + (r) : 4 * (r) + lk)
#pragma unroll
    for (int tj = 0; tj < 4; ++tj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int c = cb + 16 * tj + HQR_CCOL(r);
            cok[tj][r] = c < ncols;
            cptr[tj][r] = col_ptr(p, cok[tj][r] ? c : 0);
        }
#pragma unroll
    for (int tj = 0; tj < 4; ++tj)
#pragma unroll
        for (int ti = 0; ti < 4; ++ti) {
            acc32[tj][ti] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int r = 0; r < 4; ++r)
                acc[tj][ti][r] = F32 ? 0.0 : __builtin_nontemporal_load(&cptr[tj][r][gr[ti]]);
        }

    const double *wrow = p.wp + p.xoff + cb + li;
    int wofs[4];
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) wofs[tj] = (cb + 16 * tj + li < ncols) ? 16 * tj : 0;
    // raw operands of a k-step: W' row k, V column k and up_k (plain loads,
    // no branch); the triangle of V and k >= bw are applied after the pins
    double an[4], bn[4], un;
    auto issue = [&](int k0) {
        const int k = k0 + lk;
        const int kc = (k < p.bw) ? k : 0;
#pragma unroll
        for (int tj = 0; tj < 4; ++tj) an[tj] = wrow[(size_t)kc * p.nxpad + wofs[tj]];
#pragma unroll
        for (int ti = 0; ti < 4; ++ti) bn[ti] = HQR_AT(p.A, gr[ti], p.c0 + kc, p.lda);
        un = p.up[p.c0 + kc];
    };
    issue(0);
#pragma unroll 1
    for (int k0 = 0; k0 < NB; k0 += 4) {
        const int k = k0 + lk;
        const bool kok = k < p.bw;
        double a[4], b[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            pin_f64(an[q]);
            pin_f64(bn[q]);
        }
        pin_f64(un);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t d = rb + 16 * q + li - p.c0;   // row offset from the panel's first row
            const double v = (masked && d <= k) ? ((d == k) ? un : 0.0) : bn[q];
            a[q] = kok ? -an[q] : 0.0;
            b[q] = kok ? v : 0.0;
        }
        if (k0 + 4 < NB) issue(k0 + 4);
#pragma unroll
        for (int tj = 0; tj < 4; ++tj)
#pragma unroll
            for (int ti = 0; ti < 4; ++ti) {
                if (F32)
                    acc32[tj][ti] = __builtin_amdgcn_mfma_f32_16x16x4f32(to_f32(a[tj]), to_f32(b[ti]), acc32[tj][ti], 0, 0, 0);
                else
                    acc[tj][ti] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[tj], b[ti], acc[tj][ti], 0, 0, 0);
            }
    }
    if (F32) {
        // C += the FP32 product: the old values are loaded together first
#pragma unroll
        for (int tj = 0; tj < 4; ++tj)
#pragma unroll
            for (int ti = 0; ti < 4; ++ti)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[tj][ti][r] = __builtin_nontemporal_load(&cptr[tj][r][gr[ti]]);
    }
#pragma unroll
    for (int tj = 0; tj < 4; ++tj)
#pragma unroll
        for (int ti = 0; ti < 4; ++ti)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = rb + 16 * ti + li;
                if (cok[tj][r] && rok[ti]) {
                    if (F32) __builtin_nontemporal_store(acc[tj][ti][r] + (double)acc32[tj][ti][r], &cptr[tj][r][gi]);
                    else __builtin_nontemporal_store(acc[tj][ti][r], &cptr[tj][r][gi]);
                }
            }
#undef HQR_CCOL
}

// X <- X - V W' for at most 64 columns (the next panel's columns on the
// critical path): grid ceil(rows / 64); wave w owns rows [64 bx + 16 w, +16)
// and all columns (four 16-column MFMA tiles), so the 64-deep contraction is
// spread over many waves instead of a few 64 x 64 tiles.  Same operand
// layout as update_kernel (D' = -W'^T V^T).
template <bool F32>
__global__ void __launch_bounds__(256) update_narrow_kernel(UpdArgs p)
{
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t rb = (int64_t)p.c0 + (int64_t)blockIdx.x * 64 + 16 * w;
    const int ncols = p.ncA + p.nB;
    if (rb >= p.m) return; // no barriers below
    const int li = lane & 15, lk = lane >> 4;
    const int64_t gi = rb + li;
    const bool rok = gi < p.m;
    const int64_t gr = rok ? gi : p.m - 1;   // loads are unconditional (clamped, zeroed after)
    const bool masked = rb < (int64_t)p.c0 + p.bw;
#define HQR_NCOL(r) (F32 ? 4 * lk + (r) : 4 * (r) + lk)
    f64x4 acc[4];
    f32x4 acc32[4];
    double *cptr[4][4];
    bool cok[4][4];
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) {
        acc32[tj] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int c = 16 * tj + HQR_NCOL(r);
            cok[tj][r] = c < ncols;
            cptr[tj][r] = col_ptr(p, cok[tj][r] ? c : 0);
            const double v = cptr[tj][r][gr];
            acc[tj][r] = (cok[tj][r] && rok) ? v : 0.0;
        }
    }
    // every operand is loaded before the first MFMA (80 values per lane, plus
    // up_k): plain loads first, all pinned, then the selects
    const double *wrow = p.wp + p.xoff + li;
    double a[NB / 4][4], bv[NB / 4], uv[NB / 4];
#pragma unroll
    for (int k4 = 0; k4 < NB / 4; ++k4) {
        const int k = 4 * k4 + lk;
        const int kc = (k < p.bw) ? k : 0;
#pragma unroll
        for (int tj = 0; tj < 4; ++tj) a[k4][tj] = wrow[(size_t)kc * p.nxpad + ((16 * tj + li < ncols) ? 16 * tj : 0)];
        bv[k4] = HQR_AT(p.A, gr, p.c0 + kc, p.lda);
        uv[k4] = p.up[p.c0 + kc];
    }
#pragma unroll
    for (int k4 = 0; k4 < NB / 4; ++k4) {
#pragma unroll
        for (int tj = 0; tj < 4; ++tj) pin_f64(a[k4][tj]);
        pin_f64(bv[k4]);
        pin_f64(uv[k4]);
    }
    const int64_t d = gi - p.c0;   // row offset from the panel's first row
#pragma unroll
    for (int k4 = 0; k4 < NB / 4; ++k4) {
        const int k = 4 * k4 + lk;
        const bool kok = k < p.bw;
#pragma unroll
        for (int tj = 0; tj < 4; ++tj) a[k4][tj] = (kok && 16 * tj + li < ncols) ? -a[k4][tj] : 0.0;
        const double b = (masked && d <= k) ? ((d == k) ? uv[k4] : 0.0) : bv[k4];
        bv[k4] = (kok && rok) ? b : 0.0;
    }
#pragma unroll
    for (int k4 = 0; k4 < NB / 4; ++k4) {
        const double b = bv[k4];
#pragma unroll
        for (int tj = 0; tj < 4; ++tj) {
            if (F32)
                acc32[tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(to_f32(a[k4][tj]), to_f32(b), acc32[tj], 0, 0, 0);
            else
                acc[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[k4][tj], b, acc[tj], 0, 0, 0);
        }
    }
#pragma unroll
    for (int tj = 0; tj < 4; ++tj)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (cok[tj][r] && rok) {
                if (F32) cptr[tj][r][gi] = acc[tj][r] + (double)acc32[tj][r];
                else cptr[tj][r][gi] = acc[tj][r];
            }
#undef HQR_NCOL
}

// ------------------------------------------------------------ triangular
// info = smallest k+1 with R[k][k] == 0 (0 if none).  One workgroup.
__global__ void __launch_bounds__(256) diag_check_kernel(const double *A, int64_t lda, int64_t n, int *info)
{
    __shared__ int first;
    if (threadIdx.x == 0) first = 0x7fffffff;
    __syncthreads();
    for (int64_t k = threadIdx.x; k < n; k += 256)
        if (HQR_AT(A, k, k, lda) == 0.0) atomicMin(&first, (int)(k + 1));
    __syncthreads();
    if (threadIdx.x == 0) *info = (first == 0x7fffffff) ? 0 : first;
}



// Workgroup b owns row block b (64 rows; for TRANS, R^T x = b by forward
// substitution and the blocks above it).  Everything that does not depend on
// other blocks is loaded before the first wait: the diagonal block (with the
// reciprocals of its diagonal), the block's right-hand sides, and each
// off-diagonal block of R one iteration ahead, in registers.  The remaining
// critical path per block is: poll the predecessor's x values until none
// holds TRSV_EMPTY (one read of memory shared by all XCDs, no separate flag
// and no cache invalidation), one 64 x 64 block product, a 64-step
// substitution with multiplies by the precomputed reciprocals, and the
// stores that publish the result (no release fence: no other data rides on
// them).  NR: right-hand sides handled per pass (1, or TRSV_MAXRHS for
// 2..8); the four waves take the right-hand sides' substitutions in turn.
template <bool TRANS, int NR>
__global__ void __launch_bounds__(256) trsv_kernel(TrsvArgs p)
{
    __shared__ double xs[64][NR];
    __shared__ double accs[64][NR];
    __shared__ double part[4][64][NR];
    __shared__ double Rd[64][65];
    __shared__ double rinv[64];
    __shared__ int bad;
    const int tid = threadIdx.x, lane = tid & 63, g = tid >> 6;
    if (*((volatile int *)p.info) != 0) return;
    if (p.active && *((volatile int *)p.active) == 0) return;
    const int nblk = (int)((p.n + 63) / 64);
    const int ib = TRANS ? (int)blockIdx.x : nblk - 1 - (int)blockIdx.x;
    const int64_t r0 = (int64_t)ib * 64;
    const int nr = (int)min<int64_t>(64, p.n - r0);
    const int nrhs = p.nrhs;
    if (tid == 0) bad = 0;
    // independent of the other blocks: diagonal block, own right-hand sides
    for (int idx = tid; idx < nr * nr; idx += 256) {
        const int cc = idx / nr, r = idx - cc * nr;
        Rd[r][cc] = HQR_AT(p.A, r0 + r, r0 + cc, p.lda);
    }
    for (int idx = tid; idx < nr * NR; idx += 256) {
        const int c = idx / nr, r = idx - c * nr;
        accs[r][c] = (c < nrhs) ? HQR_AT(p.B, r0 + r, c, p.ldb) : 0.0;
    }
    double acc[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) acc[c] = 0.0;
    const int npred = TRANS ? ib : nblk - 1 - ib;
    // off-diagonal block of iteration jj: thread (row lane, group g) takes
    // columns g, g + 4, .., of the predecessor block
    auto fetch = [&](int jj, double (&rv)[16]) {
        const int jb = TRANS ? jj : nblk - 1 - jj;
        const int64_t c0 = (int64_t)jb * 64;
        const int nc = (int)min<int64_t>(64, p.n - c0);
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int l = g + 4 * q;
            rv[q] = (lane < nr && l < nc) ? (TRANS ? HQR_AT(p.A, c0 + l, r0 + lane, p.lda) : HQR_AT(p.A, r0 + lane, c0 + l, p.lda))
                                          : 0.0;
        }
    };
    double rv[16], rn[16];
    if (npred > 0) fetch(0, rv);
    __syncthreads();
    if (tid < nr) rinv[tid] = 1.0 / Rd[tid][tid];
    for (int jj = 0; jj < npred; ++jj) {
        const int jb = TRANS ? jj : nblk - 1 - jj;
        if (jj + 1 < npred) fetch(jj + 1, rn);
        const int64_t c0 = (int64_t)jb * 64;
        const int nc = (int)min<int64_t>(64, p.n - c0);
        for (int idx = tid; idx < 64 * NR; idx += 256) {
            const int r = idx / NR, c = idx - r * NR;
            unsigned long long u = 0;   // the bits of +0.0
            if (r < nc && c < nrhs) {
                unsigned long long *slot = (unsigned long long *)(p.xpub + (size_t)c * p.n + (size_t)(c0 + r));
                long spins = 0;
                while ((u = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == TRSV_EMPTY) {
                    if (++spins > p.spin_limit) {
                        bad = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            xs[r][c] = __longlong_as_double((long long)u);
        }
        __syncthreads();
        if (bad) break;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int l = g + 4 * q;
#pragma unroll
            for (int c = 0; c < NR; ++c) acc[c] = fma(rv[q], xs[l][c], acc[c]);
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) rv[q] = rn[q];
        __syncthreads();
    }
    if (bad) {
        if (tid == 0) atomicExch(p.info, HQR_INFO_TIMEOUT);
        return;
    }
#pragma unroll
    for (int c = 0; c < NR; ++c) part[g][lane][c] = acc[c];
    __syncthreads();
    if (g < nrhs && g < NR) {
        // the substitution runs fully unrolled on registers: lane l holds its
        // row (column when TRANS) of the diagonal block and 1/R_ll, so a step
        // is two lane reads, a multiply and an FMA (no LDS access on the
        // dependency chain).  Wave g solves right-hand sides g, g + 4.
        double rowv[64];
#pragma unroll
        for (int i = 0; i < 64; ++i) rowv[i] = TRANS ? Rd[i][lane] : Rd[lane][i];
        const double rl = (lane < nr) ? rinv[lane] : 0.0;
        for (int c = g; c < nrhs && c < NR; c += 4) {
            // fresh copies per right-hand side, so that the 64 steps' lane
            // masks and lane reads are not hoisted out of this loop into
            // hundreds of SGPRs (which spill to VGPR lanes and are read back
            // at every step)
            double rlc = rl;
            pin_f64(rlc);
            int lc = lane, nrc = nr;
            asm volatile("" : "+v"(lc));
            asm volatile("" : "+s"(nrc));
            double t = 0.0;
            if (lane < nr)
                t = accs[lane][c] - (((part[0][lane][c] + part[1][lane][c]) + part[2][lane][c]) + part[3][lane][c]);
            if (TRANS) {
#pragma unroll
                for (int i = 0; i < 64; ++i) {
                    if (i < nrc) {
                        const double xi = readlane_f64(t, i) * readlane_f64(rlc, i);
                        if (lc > i && lc < nrc) t = fma(-rowv[i], xi, t);
                    }
                }
            } else {
#pragma unroll
                for (int i = 63; i >= 0; --i) {
                    if (i < nrc) {
                        const double xi = readlane_f64(t, i) * readlane_f64(rlc, i);
                        if (lc < i) t = fma(-rowv[i], xi, t);
                    }
                }
            }
            // lane l's value is final once step l has read it, so x_l is the
            // same product t_l / R_ll (as t_l * rinv) that step l used; taking
            // it here keeps a select off each step's dependency chain
            t *= rl;
            if (lane < nr) {
                // publish first (the successors wait on it), then the result
                unsigned long long u = (unsigned long long)__double_as_longlong(t);
                if (u == TRSV_EMPTY) u = 0x7FF8000000000000ull;
                __hip_atomic_store((unsigned long long *)(p.xpub + (size_t)c * p.n + (size_t)(r0 + lane)), u,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                p.B[(size_t)(r0 + lane) + (size_t)c * p.ldb] = t;
            }
        }
    }
}

// resnorm[c] = ||B[n:m, c]||, one workgroup per column.
__global__ void __launch_bounds__(256) resnorm_kernel(const double *B, int64_t ldb, int64_t n, int64_t m, double *out)
{
    __shared__ double ss[4], mxs[4];
    const int tid = threadIdx.x, lane = tid & 63, g = tid >> 6;
    const double *col = B + (size_t)blockIdx.x * ldb;
    double s = 0.0, mx = 0.0;
    for (int64_t i = n + tid; i < m; i += 256) {
        s += col[i] * col[i];
        mx = fmax(mx, fabs(col[i]));
    }
    for (int o = 32; o > 0; o >>= 1) {
        s += __shfl_xor(s, o);
        mx = fmax(mx, __shfl_xor(mx, o));
    }
    if (lane == 0) {
        ss[g] = s;
        mxs[g] = mx;
    }
    __syncthreads();
    const double tot = ((ss[0] + ss[1]) + ss[2]) + ss[3];
    const double gmx = fmax(fmax(mxs[0], mxs[1]), fmax(mxs[2], mxs[3]));
    if (gmx == 0.0 || norm_fast_path_ok(gmx)) {
        if (tid == 0) out[blockIdx.x] = sqrt(tot);
        return;
    }
    double t = 0.0;
    for (int64_t i = n + tid; i < m; i += 256) {
        const double y = col[i] / gmx;
        t += y * y;
    }
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
    __syncthreads();
    if (lane == 0) ss[g] = t;
    __syncthreads();
    if (tid == 0) out[blockIdx.x] = gmx * sqrt(((ss[0] + ss[1]) + ss[2]) + ss[3]);
}

// ------------------------------------------------------------ refinement
// r = b - A0 x (FP64) for RESID_ROWS rows (blockIdx.x) and up to RESID_NR
// right-hand sides (blockIdx.y), so A0 is streamed once per RESID_NR columns
// of x.  Lane l of wave w takes row l % 32 and lane group k = 2w + l / 32,
// which owns columns [64k, 64k + 64) of each 512-column chunk of x (staged in
// LDS): a load instruction reads two 256-byte column segments, and every lane
// keeps 16 loads in flight with two partial sums per right-hand side.  The
// eight groups' sums are combined in a fixed order (deterministic).  Columns
// that are frozen are skipped unless `all`.
constexpr int RESID_ROWS = 32, RESID_NR = 4, RESID_CHUNK = 512, RESID_UNROLL = 16;
__global__ void __launch_bounds__(256) resid_kernel(RefineArgs a, int all)
{
    __shared__ double xs[RESID_CHUNK][RESID_NR];
    __shared__ double red[8][RESID_ROWS][RESID_NR];
    const int tid = threadIdx.x, lane = tid & 63, row = lane & 31, grp = 2 * (tid >> 6) + (lane >> 5);
    if (!all && *((volatile int *)a.active) == 0) return;
    const int c0 = (int)blockIdx.y * RESID_NR;
    int act = 0;   // bit c: right-hand side c0 + c is computed
#pragma unroll
    for (int c = 0; c < RESID_NR; ++c)
        if (c0 + c < a.nrhs && (all || a.stat[4 * (c0 + c) + 3] == 0)) act |= 1 << c;
    if (act == 0) return;
    const int64_t i = (int64_t)blockIdx.x * RESID_ROWS + row;
    const bool rok = i < a.m;
    const double *arow = a.A0 + (rok ? i : 0);   // rows past m read row 0; discarded
    double s0[RESID_NR], s1[RESID_NR];
#pragma unroll
    for (int c = 0; c < RESID_NR; ++c) s0[c] = s1[c] = 0.0;
    for (int64_t j0 = 0; j0 < a.n; j0 += RESID_CHUNK) {
        const int nj = (int)min<int64_t>(RESID_CHUNK, a.n - j0);
        __syncthreads();
        {
            // all loads first (unconditional, at a clamped address: X[0] when
            // not needed), then the selects: no wait between the loads
            constexpr int PER = RESID_CHUNK * RESID_NR / 256;
            double v[PER];
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const int idx = tid + 256 * q, j = idx / RESID_NR, c = idx - j * RESID_NR;
                const bool ok = j < nj && ((act >> c) & 1);
                v[q] = a.X[ok ? (size_t)(c0 + c) * a.ldx + (size_t)(j0 + j) : 0];
            }
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const int idx = tid + 256 * q, j = idx / RESID_NR, c = idx - j * RESID_NR;
                const bool ok = j < nj && ((act >> c) & 1);
                xs[j][c] = ok ? v[q] : 0.0;
            }
        }
        __syncthreads();
        const int jb = 64 * grp;
        const int cnt = max(0, min(64, nj - jb));   // uniform over the 32-lane group
        const double *ap = arow + (size_t)(j0 + jb) * a.lda0;
        int jj = 0;
        for (; jj + RESID_UNROLL <= cnt; jj += RESID_UNROLL) {
            double av[RESID_UNROLL];
#pragma unroll
            for (int u = 0; u < RESID_UNROLL; ++u) av[u] = ap[(size_t)(jj + u) * a.lda0];
#pragma unroll
            for (int u = 0; u < RESID_UNROLL; u += 2) {
#pragma unroll
                for (int c = 0; c < RESID_NR; ++c) {
                    s0[c] = fma(av[u], xs[jb + jj + u][c], s0[c]);
                    s1[c] = fma(av[u + 1], xs[jb + jj + u + 1][c], s1[c]);
                }
            }
        }
        for (; jj < cnt; ++jj) {
            const double av = ap[(size_t)jj * a.lda0];
#pragma unroll
            for (int c = 0; c < RESID_NR; ++c) s0[c] = fma(av, xs[jb + jj][c], s0[c]);
        }
    }
#pragma unroll
    for (int c = 0; c < RESID_NR; ++c) red[grp][row][c] = s0[c] + s1[c];
    __syncthreads();
    if (tid < RESID_ROWS * RESID_NR) {
        const int r = tid % RESID_ROWS, c = tid / RESID_ROWS;
        const int64_t ir = (int64_t)blockIdx.x * RESID_ROWS + r;
        if (ir < a.m && ((act >> c) & 1)) {
            const double t = ((red[0][r][c] + red[1][r][c]) + (red[2][r][c] + red[3][r][c])) +
                             ((red[4][r][c] + red[5][r][c]) + (red[6][r][c] + red[7][r][c]));
            a.rvec[(size_t)(c0 + c) * a.m + ir] = a.borig[(size_t)(c0 + c) * a.m + ir] - t;
        }
    }
}

// g = A0^T r for column blockIdx.y (FP64): one wave per column of A0, lanes
// down the rows.
__global__ void __launch_bounds__(256) gemvt_kernel(RefineArgs a)
{
    const int c = blockIdx.y;
    if (*((volatile int *)a.active) == 0 || a.stat[4 * c + 3]) return;
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= a.n) return;
    const double *aj = a.A0 + (size_t)j * a.lda0;
    const double *r = a.rvec + (size_t)c * a.m;
    double s = 0.0;
    for (int64_t i = lane; i < a.m; i += 64) s += aj[i] * r[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) a.gvec[(size_t)c * a.n + j] = s;
}

// One correction step for column blockIdx.x: x += dx, then the stopping rule
// of hqr_refine_rule.hpp on ||dx|| and ||x||.  A column that converges or
// fails is frozen (its x stays as it is) and leaves the active count.
__global__ void __launch_bounds__(1024) csne_update_kernel(RefineArgs a, int step)
{
    __shared__ double s1[16], s2[16];
    const int c = blockIdx.x;
    int *st = a.stat + 4 * c;
    if (*((volatile int *)a.active) == 0 || st[3]) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    double *x = a.X + (size_t)c * a.ldx;
    const double *dx = a.gvec + (size_t)c * a.n;
    double sa = 0.0, sb = 0.0;
    for (int64_t j = tid; j < a.n; j += 1024) {
        const double xn = x[j] + dx[j];
        x[j] = xn;
        sa += dx[j] * dx[j];
        sb += xn * xn;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        sa += __shfl_xor(sa, o);
        sb += __shfl_xor(sb, o);
    }
    if (lane == 0) {
        s1[w] = sa;
        s2[w] = sb;
    }
    __syncthreads();
    if (tid == 0) {
        double da = 0.0, xb = 0.0;
        for (int q = 0; q < 16; ++q) {
            da += s1[q];
            xb += s2[q];
        }
        RefineState rs{st[0], st[1], st[2], st[3], a.dxprev[c]};
        refine_rule_step(rs, step, sqrt(da), sqrt(xb), a.tol, REFINE_STALL_FLOOR);
        st[0] = rs.first;
        st[1] = rs.failed;
        st[2] = rs.stalls;
        st[3] = rs.frozen;
        a.dxprev[c] = rs.prev;
        if (rs.frozen) atomicSub(a.active, 1);
    }
}

// Initial state of a refinement run: every column active.
__global__ void refine_init_kernel(RefineArgs a)
{
    for (int i = threadIdx.x; i < 4 * a.nrhs; i += blockDim.x) a.stat[i] = 0;
    for (int i = threadIdx.x; i < a.nrhs; i += blockDim.x) a.dxprev[i] = 0.0;
    if (threadIdx.x == 0) *a.active = a.nrhs;
}

// Outcome of a refinement run: verdict[0] = 1 when every column converged;
// iters = the largest first-converged step (max_iter when some column did
// not converge); with or_info, HQR_INFO_NOCONV is ORed into *info when not
// every column converged.  One thread.
__global__ void refine_verdict_kernel(RefineArgs a, int *verdict, int *info, int *iters, int or_info)
{
    if (threadIdx.x != 0) return;
    int conv = 1, it = 0;
    for (int c = 0; c < a.nrhs; ++c) {
        const int *st = a.stat + 4 * c;
        if (st[0] == 0 || st[1]) conv = 0;
        it = max(it, st[0]);
    }
    if (!conv) it = a.max_iter;
    if (verdict) *verdict = conv;
    if (iters) *iters = it;
    if (or_info && !conv && info) *info |= HQR_INFO_NOCONV;
}

// Q (m x k, leading dimension ldq) <- the leading k columns of the m x m
// identity; grid-stride over the k columns.
__global__ void __launch_bounds__(256) eye_kernel(double *Q, int64_t ldq, int64_t m, int64_t k)
{
    for (int64_t j = blockIdx.x; j < k; j += gridDim.x) {
        double *col = Q + (size_t)j * ldq;
        for (int64_t i = threadIdx.x; i < m; i += 256) col[i] = (i == j) ? 1.0 : 0.0;
    }
}

// *p |= v (one thread).
__global__ void or_int_kernel(int *p, int v)
{
    if (threadIdx.x == 0) *p |= v;
}

__global__ void fill_int_kernel(int *p, int v, int64_t count)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

} // namespace hqr
