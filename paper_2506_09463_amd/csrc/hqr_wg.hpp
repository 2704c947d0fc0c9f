// hqr_wg.hpp -- one workgroup solves one least-squares problem, blocked.
//
// The factorization is the paper's one-reflector-per-column loop (Section 3,
// Alg. 2, with the (up, b) storage of Alg. 3), grouped in panels of WG_P = 16
// columns:
//   * panel: the panel's rows are spread over the threads (thread t owns
//     rows c0 + t + NT*q) and kept in registers.  For column k one block
//     reduction gives, from each thread's own rows below the pivot,
//     s_j = sum_r A[r][j] A[r][k] for the panel columns j >= k: j = k is the
//     tail's squared norm, j > k the dots the reflector's application needs.
//     Every thread then forms the same s = -sgn(x0)||x||, up = x0 - s,
//     b = up s and updates its own rows, so one barrier per column suffices;
//     the compact-WY T of the panel follows from V^T V once it is factored;
//   * trailing update (and Q^T B, B's columns riding as trailing columns):
//     Q_panel^T C = C - V T^T (V^T C) on FP64 MFMA, V and T staged in LDS,
//     every wave owning whole 16-column tiles (no cross-wave reduction).
// Then residual norms ||(Q^T B)[n:m]|| and a blocked back-substitution
// (16-row diagonal blocks solved inside one wave, updates of the rows above
// spread over the workgroup).
//
// A stored factorization (flags without WG_FACTOR) is applied instead: V is
// read back from A and up, T rebuilt from V^T V.
#pragma once

#include <utility>

#include "hqr_args.hpp"

namespace hqr {

// Rows a variant holds (NT threads x QM rows) bound m; n * nrhs must fit the
// V area for the back-substitution.
template <int NT, int QM>
struct WgShared {
    double v[NT * QM * WG_LD];
    double t[WG_P * WG_LD];
    double red[2][NT / 64][WG_P + 1];
    double prow[2][WG_P];
    double aux[NT / 64];
    int isc[4];
};

template <int NT, int QM>
constexpr int64_t wg_max_rows() { return (int64_t)NT * QM; }
template <int NT, int QM>
constexpr int64_t wg_max_x() { return (int64_t)NT * QM * WG_LD; }

// Cross-lane moves of a double without LDS: gfx950's permlane swaps between
// the wave's halves (32) and between row pairs (16), and DPP within rows.
HQR_DEV unsigned lo32(double v) { return (unsigned)__double2loint(v); }
HQR_DEV unsigned hi32(double v) { return (unsigned)__double2hiint(v); }
HQR_DEV double mk64(unsigned hi, unsigned lo) { return __hiloint2double((int)hi, (int)lo); }

// S = 32 or 16: one step of the halving sum over the lanes that differ in
// bit log2(S).  The swap exchanges a's half of the lanes with that bit set
// and b's half with it clear (one instruction per 32-bit half), so afterwards
// every lane holds, in the two registers, its own and its partner's copy of
// the value it keeps: a in the lanes with the bit clear, b in the others.
// Their sum is that value's partial total (own + partner, or partner + own:
// the same double).
template <int S>
HQR_DEV double swap_add(double a, double b)
{
    if (S == 32) {
        const auto rl = __builtin_amdgcn_permlane32_swap(lo32(a), lo32(b), false, false);
        const auto rh = __builtin_amdgcn_permlane32_swap(hi32(a), hi32(b), false, false);
        return mk64(rh[0], rl[0]) + mk64(rh[1], rl[1]);
    } else {
        const auto rl = __builtin_amdgcn_permlane16_swap(lo32(a), lo32(b), false, false);
        const auto rh = __builtin_amdgcn_permlane16_swap(hi32(a), hi32(b), false, false);
        return mk64(rh[0], rl[0]) + mk64(rh[1], rl[1]);
    }
}

// DPP move of a double within 16-lane rows (CTRL: a DPP16 control code
// whose source lane is valid for every lane, so no old value is needed).
template <int CTRL>
HQR_DEV double dpp64(double v)
{
    const long r = __builtin_amdgcn_mov_dpp(__builtin_bit_cast(long, v), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, r);
}

constexpr int DPP_ROW_ROR8 = 0x128;      // lane i <- i ^ 8 within the row
constexpr int DPP_ROW_HALF_MIRROR = 0x141; // lane i <- 7 - i within 8 lanes
constexpr int DPP_QUAD_XOR2 = 0x4E;      // quad_perm [2, 3, 0, 1]
constexpr int DPP_QUAD_XOR1 = 0xB1;      // quad_perm [1, 0, 3, 2]

// Sum over the wave of N = 16, 8, 4 or 2 values v[0..N-1] by recursive
// halving: lane L ends with the total of index wave_sum_index<N>(L), from
// bits 5, 4, 3, 2 of L (the top log2(N) of them).  At each halving step a
// lane keeps the half of its values selected by one bit of its id and adds
// the other half of a partner lane across that bit; any pairing that crosses
// the bit inside the lanes that share the higher bits adds up the same sums
// (the bit-2 step pairs i with 7 - i, the others with i ^ 2^b).  The lanes
// then add across bits 1 and 0 and, for N < 16, across the bits above the
// index, so every lane holding an index holds the same total.  No LDS.
template <int N>
HQR_DEV double wave_sum(const double (&v)[N], int lane)
{
    static_assert(N == 16 || N == 8 || N == 4 || N == 2, "N");
    double x8[8], x4[4], x2[2];
    const bool h3 = (lane & 8) != 0, h2 = (lane & 4) != 0;
    if constexpr (N == 16) {
#pragma unroll
        for (int t = 0; t < 8; ++t) x8[t] = swap_add<32>(v[t], v[8 + t]);
    } else if constexpr (N == 8) {
#pragma unroll
        for (int t = 0; t < 8; ++t) x8[t] = v[t];
    }
    if constexpr (N >= 8) {
#pragma unroll
        for (int t = 0; t < 4; ++t) x4[t] = swap_add<16>(x8[t], x8[4 + t]);
    } else if constexpr (N == 4) {
#pragma unroll
        for (int t = 0; t < 4; ++t) x4[t] = v[t];
    }
    if constexpr (N >= 4) {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const double keep = h3 ? x4[2 + t] : x4[t];
            const double give = h3 ? x4[t] : x4[2 + t];
            x2[t] = keep + dpp64<DPP_ROW_ROR8>(give);
        }
    } else {
        x2[0] = v[0];
        x2[1] = v[1];
    }
    double a1 = (h2 ? x2[1] : x2[0]) + dpp64<DPP_ROW_HALF_MIRROR>(h2 ? x2[0] : x2[1]);
    a1 += dpp64<DPP_QUAD_XOR2>(a1);
    a1 += dpp64<DPP_QUAD_XOR1>(a1);
    if constexpr (N <= 2) a1 += dpp64<DPP_ROW_ROR8>(a1);
    if constexpr (N <= 4) a1 = swap_add<16>(a1, a1);
    if constexpr (N <= 8) a1 = swap_add<32>(a1, a1);
    return a1;
}

template <int N>
HQR_DEV int wave_sum_index(int lane)
{
    const int i = ((lane >> 5) & 1) * 8 + ((lane >> 4) & 1) * 4 + ((lane >> 3) & 1) * 2 + ((lane >> 2) & 1);
    return i & (N - 1);
}

// lanes that write a wave_sum<N> total: one per index
template <int N>
HQR_DEV bool wave_sum_writer(int lane)
{
    constexpr int dup = (N == 16) ? 3 : (N == 8) ? 32 + 3 : (N == 4) ? 48 + 3 : 56 + 3;
    return (lane & dup) == 0;
}

// The value lane 16r + i holds, in every lane of row r (DPP row_newbcast;
// i must be a constant once the caller's loop is unrolled).
template <int I> HQR_DEV double row_bcast16_c(double v)
{
    const long r = __builtin_amdgcn_mov_dpp(__builtin_bit_cast(long, v), 0x150 + I, 0xf, 0xf, false);
    return __builtin_bit_cast(double, r);
}

HQR_DEV double row_bcast16(double v, int i)
{
    switch (i) {
    case 0: return row_bcast16_c<0>(v);
    case 1: return row_bcast16_c<1>(v);
    case 2: return row_bcast16_c<2>(v);
    case 3: return row_bcast16_c<3>(v);
    case 4: return row_bcast16_c<4>(v);
    case 5: return row_bcast16_c<5>(v);
    case 6: return row_bcast16_c<6>(v);
    case 7: return row_bcast16_c<7>(v);
    case 8: return row_bcast16_c<8>(v);
    case 9: return row_bcast16_c<9>(v);
    case 10: return row_bcast16_c<10>(v);
    case 11: return row_bcast16_c<11>(v);
    case 12: return row_bcast16_c<12>(v);
    case 13: return row_bcast16_c<13>(v);
    case 14: return row_bcast16_c<14>(v);
    default: return row_bcast16_c<15>(v);
    }
}

// Block-wide sum (op 0) or max (op 1) of one value per thread; uniform result.
template <int NT, int QM>
HQR_DEV double wg_block_reduce(double x, int op, WgShared<NT, QM> &sh)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double y = __shfl_xor(x, o);
        x = op ? fmax(x, y) : x + y;
    }
    __syncthreads();
    if (lane == 0) sh.aux[w] = x;
    __syncthreads();
    double r = sh.aux[0];
#pragma unroll
    for (int i = 1; i < NT / 64; ++i) r = op ? fmax(r, sh.aux[i]) : r + sh.aux[i];
    return r;
}

// ||(x0, x)|| for a column whose sum of squares under- or overflows: the
// entries scaled by c = max |x_i| first (each thread passes its QM <= 4 rows
// below the pivot, zeros elsewhere; every thread of the workgroup calls it).
template <int NT, int QM>
__device__ __noinline__ double wg_scaled_norm(double x0, double x1, double x2, double x3, double x4,
                                              WgShared<NT, QM> &sh)
{
    const double xs[4] = {x1, x2, x3, x4};
    double mx = 0.0;
#pragma unroll
    for (int q = 0; q < QM; ++q) mx = fmax(mx, fabs(xs[q]));
    const double c = fmax(fabs(x0), wg_block_reduce<NT, QM>(mx, 1, sh));
    double ss = 0.0;
#pragma unroll
    for (int q = 0; q < QM; ++q) {
        const double y = xs[q] / c;
        ss = fma(y, y, ss);
    }
    const double t2 = wg_block_reduce<NT, QM>(ss, 0, sh);
    const double x0c = x0 / c;
    return c * sqrt(x0c * x0c + t2);
}

// s = sqrt(d) and r = 1/sqrt(d) for 2^-920 <= d <= 2^920: the hardware
// reciprocal square root refined by two coupled Newton steps for s and
// 1/(2s) (Goldschmidt's iteration), then one residual correction of s.
HQR_DEV void wg_sqrt_rsqrt(double d, double &s, double &r)
{
    const double y = __builtin_amdgcn_rsq(d);
    double sv = d * y, h = 0.5 * y;
    double e = fma(-sv, h, 0.5);
    sv = fma(sv, e, sv);
    h = fma(h, e, h);
    e = fma(-sv, h, 0.5);
    sv = fma(sv, e, sv);
    h = fma(h, e, h);
    s = fma(h, fma(-sv, sv, d), sv);
    r = 2.0 * h;
}

// 1/u for a normal u whose reciprocal is normal: the hardware reciprocal
// and two Newton steps.
HQR_DEV double wg_recip(double u)
{
    double y = __builtin_amdgcn_rcp(u);
    double e = fma(-u, y, 1.0);
    y = fma(y, e, y);
    e = fma(-u, y, 1.0);
    return fma(y, e, y);
}

// ---------------------------------------------------------------- panel
// One column step of the panel: k is a compile-time constant so every
// register index is static (a runtime k would turn the register arrays into
// selects or scratch memory).
template <int NT, int QM, int k>
HQR_DEV void wg_panel_step(const WgDesc &d, int c0, int pw, int m, double (&a)[QM][WG_P], double &myup,
                           WgShared<NT, QM> &sh)
{
    constexpr int NWV = NT / 64;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (k >= pw) return;
    const int pr = c0 + k;
    const int buf = k & 1;
    // the step needs the dots with columns k .. 15 only (the norm and the
    // weights; T comes from V^T V after the panel): they are reduced over
    // the last N = 16, 8, 4 or 2 columns, starting at column j0
    constexpr int j0 = (k < 8) ? 0 : (k < 12) ? 8 : (k < 14) ? 12 : 14;
    constexpr int NRED = WG_P - j0;
    // partial dots of the column below the pivot with the panel columns
    double xk[QM];
    bool nz = false;
    {
        double s[NRED];
#pragma unroll
        for (int j = 0; j < NRED; ++j) s[j] = 0.0;
        // no branches on the row (a divergent branch around the register
        // arrays makes the compiler copy them at every join): rows outside
        // the column below the pivot contribute x = 0
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            const int r = c0 + tid + NT * q;
            xk[q] = a[q][k];
            const bool below = r > pr && r < m;
            const double xm = below ? xk[q] : 0.0;
            nz = nz || (xm != 0.0);
#pragma unroll
            for (int j = k; j < WG_P; ++j) s[j - j0] = fma(a[q][j], xm, s[j - j0]);
        }
        if (tid == k) {
#pragma unroll
            for (int j = k; j < WG_P; ++j) sh.prow[buf][j] = a[0][j];
        }
        const double part = wave_sum<NRED>(s, lane);
        if (wave_sum_writer<NRED>(lane)) sh.red[buf][w][j0 + wave_sum_index<NRED>(lane)] = part;
    }
    const bool wnz = __ballot(nz) != 0ull;
    if (lane == 0) sh.red[buf][w][WG_P] = wnz ? 1.0 : 0.0;
    __syncthreads();
    // every thread forms the same scalars from the reduction.  Lane 16r + j
    // sums the waves' partial dots of column j (the same total in each of the
    // four 16-lane rows) and holds A[pr][j]; the values a thread needs of
    // other columns come by DPP row broadcasts instead of LDS reads of their
    // own (columns below j0 hold stale sums that no lane takes)
    const int jl = lane & 15;
    bool anynz = false;
    double dsum = sh.red[buf][0][jl];
#pragma unroll
    for (int i = 1; i < NWV; ++i) dsum += sh.red[buf][i][jl];
    const double prow_l = sh.prow[buf][jl];
#pragma unroll
    for (int i = 0; i < NWV; ++i) anynz = anynz || (sh.red[buf][i][WG_P] != 0.0);
    const double sxx = row_bcast16_c<k>(dsum);
    const double x0 = row_bcast16_c<k>(prow_l);
    double upk = 0.0, sk = x0, inv_b = 0.0;
    if (anynz) {
        const double tot = x0 * x0 + sxx;
        double nu;
        if (tot >= 0x1p-920 && tot <= 0x1p920) {
            // nu and 1/nu together, then 1/b = 1/(up s) = (1/up)(1/s): no
            // division and no correctly rounded square root on the step's
            // dependency chain (|up| >= nu >= 2^-460, so nothing over- or
            // underflows)
            double rnu;
            wg_sqrt_rsqrt(tot, nu, rnu);
            sk = (x0 >= 0.0) ? -nu : nu;
            upk = x0 - sk;
            inv_b = wg_recip(upk) * ((x0 >= 0.0) ? -rnu : rnu);
        } else {
            // rare: the squares under- or overflow (one copy of this code,
            // outside the unrolled steps)
            double xs[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int q = 0; q < QM; ++q) {
                const int r = c0 + tid + NT * q;
                xs[q] = (r > pr && r < m) ? xk[q] : 0.0;
            }
            nu = wg_scaled_norm<NT, QM>(x0, xs[0], xs[1], xs[2], xs[3], sh);
            sk = (x0 >= 0.0) ? -nu : nu;
            upk = x0 - sk;
            inv_b = 1.0 / (upk * sk);
        }
    }
    if (tid == k) myup = upk;
    // w_j = (up A[pr][j] + sum_{r>pr} A[r][j] A[r][k]) / b for the later
    // panel columns
    const double wl = fma(upk, prow_l, dsum) * inv_b;   // w of column jl
    double wv[WG_P];
#pragma unroll
    for (int j = k + 1; j < WG_P; ++j) wv[j] = row_bcast16(wl, j);
    // T's diagonal: tau_k = -1/b_k (the rest of T follows the panel)
    if (tid == k) sh.t[k * WG_LD + k] = -inv_b;
    // apply H_k to the panel's columns k+1 .. pw-1 (own rows), by selects:
    // rows above the pivot and beyond m keep their values exactly
#pragma unroll
    for (int q = 0; q < QM; ++q) {
        const int r = c0 + tid + NT * q;
        const bool below = r > pr && r < m, piv = r == pr;
        const double vr = piv ? upk : xk[q];
#pragma unroll
        for (int j = k + 1; j < WG_P; ++j) {
            const double t = fma(wv[j], vr, a[q][j]);
            a[q][j] = (below || piv) ? t : a[q][j];
        }
        a[q][k] = piv ? sk : a[q][k];
    }
    // up_k is stored once per panel (thread k holds it in myup): a global
    // store here would make every later step reload the descriptor and wait
    // for the store to complete
}

template <int NT, int QM, int... Ks>
HQR_DEV void wg_panel_steps(const WgDesc &d, int c0, int pw, int m, double (&a)[QM][WG_P], double &myup,
                            WgShared<NT, QM> &sh, std::integer_sequence<int, Ks...>)
{
    (wg_panel_step<NT, QM, Ks>(d, c0, pw, m, a, myup, sh), ...);
}

// T of a factored panel: the Gram matrix G = V^T V of the panel's vectors
// (in sh.v, rows 0 .. nrows-1; columns beyond pw zero) on MFMA, then T row i
// by thread i from T[i][k] = -tau_k sum_{l=i}^{k-1} T[i][l] G[l][k], with
// tau_k = T[k][k] as the column steps left it.  Starts after a barrier, ends
// with one.
template <int NT, int QM>
HQR_DEV void wg_panel_t(int nrows, int pw, WgShared<NT, QM> &sh)
{
    constexpr int NWV = NT / 64;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    double tau[WG_P];
    if (tid < WG_P) {
#pragma unroll
        for (int k = 0; k < WG_P; ++k) tau[k] = sh.t[k * WG_LD + k];
    }
    f64x4 g = {0.0, 0.0, 0.0, 0.0};
    const int i16 = lane & 15, kq = lane >> 4;
    const int nb16 = (nrows + 15) / 16;
    for (int rb = w; rb < nb16; rb += NWV) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int rr = rb * 16 + 4 * kq + s;
            const double vv = (rr < nrows) ? sh.v[rr * WG_LD + i16] : 0.0;
            g = __builtin_amdgcn_mfma_f64_16x16x4f64(vv, vv, g, 0, 0, 0);
        }
    }
    __syncthreads();   // the taus are in registers before G overwrites the T area
    // G[i][j] at lane j + 16 (i % 4), reg i / 4; waves add into sh.t in turn
    for (int wv = 0; wv < NWV; ++wv) {
        if (w == wv) {
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
                double *dst = &sh.t[(4 * r4 + kq) * WG_LD + i16];
                *dst = (wv == 0) ? g[r4] : *dst + g[r4];
            }
        }
        __syncthreads();
    }
    // right-looking: once T[i][l] is final it is added into the sums of all
    // later columns (the same terms in the same order as summing each column
    // over l = i .. k-1 in turn, with the sums no longer one long chain)
    double trow[WG_P];
#pragma unroll
    for (int j = 0; j < WG_P; ++j) trow[j] = 0.0;
    if (tid < WG_P) {
        double acc[WG_P];
#pragma unroll
        for (int k = 0; k < WG_P; ++k) acc[k] = 0.0;
#pragma unroll
        for (int l = 0; l < WG_P; ++l) {
            trow[l] = (l >= pw || tid > l) ? 0.0 : ((tid == l) ? tau[l] : -tau[l] * acc[l]);
#pragma unroll
            for (int k = l + 1; k < WG_P; ++k) acc[k] = fma(trow[l], sh.t[l * WG_LD + k], acc[k]);
        }
    }
    __syncthreads();
    if (tid < WG_P) {
#pragma unroll
        for (int j = 0; j < WG_P; ++j) sh.t[tid * WG_LD + j] = trow[j];
    }
    __syncthreads();
}

// Factor columns c0 .. c0+pw-1 (rows c0 .. m-1) in registers; write them
// back, leave V (rows relative to c0, up on the diagonal, zeros above) and T
// in LDS.  Ends with a barrier.
template <int NT, int QM>
HQR_DEV void wg_panel_factor(const WgDesc &d, int c0, int pw, WgShared<NT, QM> &sh)
{
    const int tid = threadIdx.x;
    const int m = (int)d.m, nrows = m - c0;
    const size_t lda = (size_t)d.lda;
    double *const Ap = d.A + (size_t)c0 * lda + c0;   // A[c0][c0]
    double a[QM][WG_P];
    if (pw == WG_P) {
        // full panel: each thread loads its rows of the 16 columns straight
        // into registers; a row's 16 loads (and those of its other rows) are
        // all in flight before the first is used, instead of one round trip
        // per column through LDS
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            const int rr = tid + NT * q;
            if (rr < nrows) {
#pragma unroll
                for (int j = 0; j < WG_P; ++j) a[q][j] = Ap[(size_t)j * lda + rr];
            } else {
#pragma unroll
                for (int j = 0; j < WG_P; ++j) a[q][j] = 0.0;
            }
        }
        if (tid < WG_P) {
#pragma unroll
            for (int j = 0; j < WG_P; ++j) sh.t[tid * WG_LD + j] = 0.0;
        }
        __syncthreads();
    } else {
        // ragged last panel: staged in LDS (columns beyond pw as zeros), then
        // each thread takes its rows into registers
#pragma unroll 1
        for (int j = 0; j < WG_P; ++j) {
            if (j < pw) {
                const double *col = Ap + (size_t)j * lda;
                for (int rr = tid; rr < nrows; rr += NT) sh.v[rr * WG_LD + j] = col[rr];
            } else {
                for (int rr = tid; rr < nrows; rr += NT) sh.v[rr * WG_LD + j] = 0.0;
            }
        }
        if (tid < WG_P) {
#pragma unroll
            for (int j = 0; j < WG_P; ++j) sh.t[tid * WG_LD + j] = 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            const int rr = tid + NT * q;
#pragma unroll
            for (int j = 0; j < WG_P; ++j) a[q][j] = (rr < nrows) ? sh.v[rr * WG_LD + j] : 0.0;
        }
    }
    // up of the reflector whose pivot row this thread owns (V's diagonal);
    // the steps leave tau_k on T's diagonal
    double myup = 0.0;
    wg_panel_steps<NT, QM>(d, c0, pw, m, a, myup, sh, std::make_integer_sequence<int, WG_P>{});
    if (tid < pw) d.up[c0 + tid] = myup;
    if (pw == WG_P) {
        // the factored panel from registers to A; V (up on the diagonal, zeros
        // above it) into LDS for the trailing update.  The diagonal of row
        // rr < 16 belongs to thread rr (q = 0), whose myup it is.
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            const int rr = tid + NT * q;
            if (rr < nrows) {
#pragma unroll
                for (int j = 0; j < WG_P; ++j) {
                    Ap[(size_t)j * lda + rr] = a[q][j];
                    sh.v[rr * WG_LD + j] = (rr < j) ? 0.0 : ((rr == j) ? myup : a[q][j]);
                }
            }
        }
        __syncthreads();
        wg_panel_t<NT, QM>(nrows, pw, sh);
        return;
    }
    // back through LDS: the factored panel to A, then V (up on the diagonal,
    // zeros above it and beyond pw) stays in LDS for the trailing update
#pragma unroll
    for (int q = 0; q < QM; ++q) {
        const int rr = tid + NT * q;
        if (rr < nrows) {
#pragma unroll
            for (int j = 0; j < WG_P; ++j) sh.v[rr * WG_LD + j] = a[q][j];
        }
    }
    __syncthreads();
#pragma unroll 1
    for (int j = 0; j < pw; ++j) {
        double *col = Ap + (size_t)j * lda;
        for (int rr = tid; rr < nrows; rr += NT) col[rr] = sh.v[rr * WG_LD + j];
    }
    __syncthreads();
    if (tid < WG_P && tid < nrows) {
#pragma unroll
        for (int j = 0; j < WG_P; ++j) {
            if (j >= tid) sh.v[tid * WG_LD + j] = (j == tid) ? myup : 0.0;
        }
    }
#pragma unroll 1
    for (int j = pw; j < WG_P; ++j)
        for (int rr = tid; rr < nrows; rr += NT) sh.v[rr * WG_LD + j] = 0.0;
    __syncthreads();
    wg_panel_t<NT, QM>(nrows, pw, sh);
}

// Stored factorization: V from A's tails and up, T from V^T V.  Ends with a
// barrier.
template <int NT, int QM>
__device__ __noinline__ void wg_panel_load(const WgDesc &d, int64_t c0, int pw, WgShared<NT, QM> &sh)
{
    constexpr int NWV = NT / 64;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t m = d.m;
    const int64_t nrows = m - c0;
#pragma unroll
    for (int q = 0; q < QM; ++q) {
        const int64_t rr = tid + (int64_t)NT * q;
#pragma unroll
        for (int j = 0; j < WG_P; ++j) {
            double v = 0.0;
            if (rr < nrows && j < pw) {
                if (rr > j) v = d.A[(size_t)(c0 + j) * d.lda + c0 + rr];
                else if (rr == j) v = d.up[c0 + j];
            }
            sh.v[rr * WG_LD + j] = v;
        }
    }
    __syncthreads();
    // G = V^T V: each wave sums the 16-row blocks w, w + NWV, .. on MFMA,
    // then the waves add their partials into the T area in turn.
    f64x4 g = {0.0, 0.0, 0.0, 0.0};
    const int i16 = lane & 15, kq = lane >> 4;
    const int64_t nb16 = (nrows + 15) / 16;
    for (int64_t rb = w; rb < nb16; rb += NWV) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int64_t rr = rb * 16 + 4 * kq + s;
            const double vv = sh.v[rr * WG_LD + i16];
            g = __builtin_amdgcn_mfma_f64_16x16x4f64(vv, vv, g, 0, 0, 0);
        }
    }
    // G[i][j] at lane j + 16 (i % 4), reg i / 4; waves add into sh.t in turn
    for (int wv = 0; wv < NWV; ++wv) {
        if (w == wv) {
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
                const int i = 4 * r4 + kq;
                double *dst = &sh.t[i * WG_LD + i16];
                *dst = (wv == 0) ? g[r4] : *dst + g[r4];
            }
        }
        __syncthreads();
    }
    // T row i by thread i (T upper): T[i][k] = -tau_k sum_{l=i}^{k-1} T[i][l] G[l][k]
    double trow[WG_P];
#pragma unroll
    for (int j = 0; j < WG_P; ++j) trow[j] = 0.0;
    if (tid < WG_P) {
#pragma unroll
        for (int k = 0; k < WG_P; ++k) {
            if (k < pw) {
                const double upk = d.up[c0 + k];
                const double bk = upk * d.A[(size_t)(c0 + k) * d.lda + c0 + k];
                const double inv_b = (upk != 0.0) ? 1.0 / bk : 0.0;
                double acc = 0.0;
#pragma unroll
                for (int l = 0; l < k; ++l) acc = fma(trow[l], sh.t[l * WG_LD + k], acc);
                if (tid < k) trow[k] = inv_b * acc;
                if (tid == k) trow[k] = -inv_b;
            }
        }
    }
    __syncthreads();
    if (tid < WG_P) {
#pragma unroll
        for (int j = 0; j < WG_P; ++j) sh.t[tid * WG_LD + j] = trow[j];
    }
    __syncthreads();
}

// ------------------------------------------------------- trailing update
// C <- C - V T^T V^T C for the combined column list: A columns
// colA .. colA+ncA-1 then all B columns; rows c0 .. m-1.
HQR_DEV double *wg_colptr(const WgDesc &d, int64_t ci, int64_t colA, int64_t ncA, int64_t ntot)
{
    if (ci >= ntot) return nullptr;
    return (ci < ncA) ? d.A + (size_t)(colA + ci) * d.lda : d.B + (size_t)(ci - ncA) * d.ldb;
}

// QMODE: C <- C - V T V^T C instead (applying Q_panel rather than its
// transpose).  PIPE: 16-row blocks whose loads are issued together (load
// scheduling only: the arithmetic and its order do not depend on it).
template <int NT, int QM, int PIPE, bool QMODE = false>
HQR_DEV void wg_trailing(const WgDesc &d, int64_t c0, int64_t colA, int64_t ncA, WgShared<NT, QM> &sh)
{
    constexpr int NWV = NT / 64;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int i16 = lane & 15, kq = lane >> 4;
    const int64_t nrows = d.m - c0;
    const int64_t ntot = ncA + d.nrhs;
    const int64_t ntile = (ntot + 15) / 16;
    const int64_t nb16 = (nrows + 15) / 16;
    for (int64_t tile = w; tile < ntile; tile += NWV) {
        // W = V^T C: A operand V^T[i][k] = V[rho(k)][i], B operand C[rho(k)][j]
        const double *cp = wg_colptr(d, tile * 16 + i16, colA, ncA, ntot);
        f64x4 acc[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) acc[s] = f64x4{0.0, 0.0, 0.0, 0.0};
        // PIPE 16-row blocks per round: all their loads are issued first
        for (int64_t rb0 = 0; rb0 < nb16; rb0 += PIPE) {
            double cv[PIPE][4];
#pragma unroll
            for (int u = 0; u < PIPE; ++u) {
                const int64_t rr0 = (rb0 + u) * 16 + 4 * kq;
#pragma unroll
                for (int s = 0; s < 4; ++s) cv[u][s] = (cp && rr0 + s < nrows) ? cp[c0 + rr0 + s] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < PIPE; ++u) {
                const int64_t rr0 = (rb0 + u) * 16 + 4 * kq;
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const double av = (rr0 + s < nrows) ? sh.v[(rr0 + s) * WG_LD + i16] : 0.0;
                    acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, cv[u][s], acc[s], 0, 0, 0);
                }
            }
        }
        f64x4 wm;
#pragma unroll
        for (int r = 0; r < 4; ++r) wm[r] = (acc[0][r] + acc[1][r]) + (acc[2][r] + acc[3][r]);
        // W' = T^T W: A operand T^T[i][4q+k] = T[4q+k][i]; B operand = W's
        // register q (QMODE: W' = T W, A operand T[i][4q+k])
        f64x4 wp = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double tv = QMODE ? sh.t[i16 * WG_LD + 4 * q + kq] : sh.t[(4 * q + kq) * WG_LD + i16];
            wp = __builtin_amdgcn_mfma_f64_16x16x4f64(tv, wm[q], wp, 0, 0, 0);
        }
        // C^T <- C^T - W'^T V^T per 16-row block: D[c][row] at lane row + 16 (c % 4), reg c / 4
        double *cq[4];
#pragma unroll
        for (int g = 0; g < 4; ++g) cq[g] = wg_colptr(d, tile * 16 + 4 * g + kq, colA, ncA, ntot);
        for (int64_t rb0 = 0; rb0 < nb16; rb0 += PIPE) {
            f64x4 cacc[PIPE];
#pragma unroll
            for (int u = 0; u < PIPE; ++u) {
                const int64_t rr = (rb0 + u) * 16 + i16;
#pragma unroll
                for (int g = 0; g < 4; ++g) cacc[u][g] = (cq[g] && rr < nrows) ? cq[g][c0 + rr] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < PIPE; ++u) {
                const int64_t rr = (rb0 + u) * 16 + i16;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const double bv = (rr < nrows) ? sh.v[rr * WG_LD + 4 * q + kq] : 0.0;
                    cacc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(-wp[q], bv, cacc[u], 0, 0, 0);
                }
#pragma unroll
                for (int g = 0; g < 4; ++g)
                    if (cq[g] && rr < nrows) cq[g][c0 + rr] = cacc[u][g];
            }
        }
    }
}

// ------------------------------------------------ residual norms, solve
template <int NT, int QM>
__device__ __noinline__ void wg_resnorm(const WgDesc &d)
{
    constexpr int NWV = NT / 64;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int64_t c = w; c < d.nrhs; c += NWV) {
        const double *bc = d.B + (size_t)c * d.ldb;
        double s = 0.0, mx = 0.0;
        for (int64_t i = d.n + lane; i < d.m; i += 64) {
            s = fma(bc[i], bc[i], s);
            mx = fmax(mx, fabs(bc[i]));
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            s += __shfl_xor(s, o);
            mx = fmax(mx, __shfl_xor(mx, o));
        }
        if (mx != 0.0 && !norm_fast_path_ok(mx)) {
            double t = 0.0;
            for (int64_t i = d.n + lane; i < d.m; i += 64) {
                const double y = bc[i] / mx;
                t = fma(y, y, t);
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
            if (lane == 0) d.resnorm[c] = mx * sqrt(t);
        } else if (lane == 0) {
            d.resnorm[c] = sqrt(s);
        }
    }
}

// R X = B[0:n]: info = smallest k+1 with R[k][k] == 0 (B untouched), else X
// in B[0:n].  X staged column-major in the V area.  Block rows of 16 from the
// bottom: wave 0 solves the diagonal block (lane 16 cg + i: row i, right-hand
// side cg of each group of four; x_l broadcast by DPP, with 1/R_ll formed
// before the sequential steps), then every thread updates its rows above
// (all of a row's reads issued together, no branch per entry).
template <int NT, int QM>
HQR_DEV void wg_backsolve(const WgDesc &d, int *info, WgShared<NT, QM> &sh)
{
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t n = d.n, nrhs = d.nrhs;
    if (tid == 0) sh.isc[0] = 0x7fffffff;
    __syncthreads();
    for (int64_t k = tid; k < n; k += NT)
        if (d.A[(size_t)k * d.lda + k] == 0.0) atomicMin(&sh.isc[0], (int)(k + 1));
    __syncthreads();
    const int bad = sh.isc[0];
    if (tid == 0) info[d.index] = (bad == 0x7fffffff) ? 0 : bad;
    if (bad != 0x7fffffff || nrhs == 0 || n == 0) {
        __syncthreads();
        return;
    }
    double *xs = sh.v;
    for (int64_t idx = tid; idx < n * nrhs; idx += NT) {
        const int64_t c = idx / n, i = idx % n;
        xs[idx] = d.B[(size_t)c * d.ldb + i];
    }
    __syncthreads();
    const int64_t nblk = (n + 15) / 16;
    for (int64_t jb = nblk - 1; jb >= 0; --jb) {
        const int64_t b0 = jb * 16;
        const int bw = (int)((n - b0 < 16) ? n - b0 : 16);
        if (w == 0) {
            const int i = lane & 15, cg = lane >> 4;
            double rrow[WG_P];
#pragma unroll
            for (int l = 0; l < WG_P; ++l) rrow[l] = (i < bw && l < bw) ? d.A[(size_t)(b0 + l) * d.lda + b0 + i] : 1.0;
            double dii = 1.0;
#pragma unroll
            for (int l = 0; l < WG_P; ++l) dii = (l == i) ? rrow[l] : dii;
            const double rinv = 1.0 / dii;   // lane i's 1/R_ii (nonzero: checked above)
            for (int64_t cs = 0; cs < nrhs; cs += 4) {
                const int64_t c = cs + cg;
                const bool ok = (i < bw) && (c < nrhs);
                double xi = ok ? xs[c * n + b0 + i] : 0.0;
#pragma unroll
                for (int l = WG_P - 1; l >= 0; --l) {
                    if (l < bw) {
                        const double cand = xi * rinv;
                        const double xl = row_bcast16(cand, l);     // lane l of this 16-lane row
                        xi = (i == l) ? xl : ((i < l) ? fma(-rrow[l], xl, xi) : xi);
                    }
                }
                if (ok) xs[c * n + b0 + i] = xi;
            }
        }
        __syncthreads();
        for (int64_t i = tid; i < b0; i += NT) {
            double rv[WG_P];
#pragma unroll
            for (int l = 0; l < WG_P; ++l) rv[l] = (l < bw) ? d.A[(size_t)(b0 + l) * d.lda + i] : 0.0;
            for (int64_t c = 0; c < nrhs; ++c) {
                double acc = xs[c * n + i];
                // only the block's bw solved rows: past them the staging area
                // holds other columns' values or stale LDS, and 0 * NaN = NaN
                // (row b0 is read there instead and its value replaced by 0)
                double xv[WG_P];
#pragma unroll
                for (int l = 0; l < WG_P; ++l) xv[l] = xs[c * n + b0 + ((l < bw) ? l : 0)];
#pragma unroll
                for (int l = 0; l < WG_P; ++l) acc = fma(-rv[l], (l < bw) ? xv[l] : 0.0, acc);
                xs[c * n + i] = acc;
            }
        }
        __syncthreads();
    }
    for (int64_t idx = tid; idx < n * nrhs; idx += NT) {
        const int64_t c = idx / n, i = idx % n;
        d.B[(size_t)c * d.ldb + i] = xs[idx];
    }
    __syncthreads();
}

template <int NT, int QM, int PIPE>
HQR_DEV void wg_instance(const WgDesc &d, int *info, WgShared<NT, QM> &sh)
{
    if (d.flags & WG_APPLY_Q) {
        // Q B = H_0 .. H_{n-1} B: stored panels applied last to first
        const int64_t npan = (d.n + WG_P - 1) / WG_P;
        for (int64_t p = npan - 1; p >= 0; --p) {
            const int64_t c0 = p * WG_P;
            const int pw = (int)((d.n - c0 < WG_P) ? d.n - c0 : WG_P);
            const int64_t j0 = (d.flags & WG_QSKIP) ? c0 : 0;
            if (d.nrhs <= j0) continue;
            wg_panel_load<NT, QM>(d, c0, pw, sh);
            WgDesc dq = d;
            dq.B = d.B + (size_t)j0 * d.ldb;
            dq.nrhs = d.nrhs - j0;
            wg_trailing<NT, QM, PIPE, true>(dq, c0, c0 + pw, 0, sh);
            __syncthreads();
        }
        return;
    }
    const bool factor = (d.flags & WG_FACTOR) != 0;
    for (int64_t c0 = 0; c0 < d.n; c0 += WG_P) {
        const int pw = (int)((d.n - c0 < WG_P) ? d.n - c0 : WG_P);
        if (factor) wg_panel_factor<NT, QM>(d, (int)c0, pw, sh);
        else wg_panel_load<NT, QM>(d, c0, pw, sh);
        const int64_t ncA = factor ? d.n - c0 - pw : 0;
        wg_trailing<NT, QM, PIPE>(d, c0, c0 + pw, ncA, sh);
        __syncthreads();
    }
    if (d.resnorm && d.nrhs > 0) wg_resnorm<NT, QM>(d);
    if (d.flags & WG_SOLVE) wg_backsolve<NT, QM>(d, info, sh);
    __syncthreads();
}

// Persistent: workgroups take instances from an atomic queue head until it
// passes `count`.
template <int NT, int QM, int PIPE>
__global__ void __launch_bounds__(NT) wg_batched_kernel(const WgDesc *desc, int count, int *head, int *info)
{
    __shared__ WgShared<NT, QM> sh;
    for (;;) {
        if (threadIdx.x == 0) sh.isc[1] = atomicAdd(head, 1);
        __syncthreads();
        const int id = sh.isc[1];
        __syncthreads();
        if (id >= count) break;
        wg_instance<NT, QM, PIPE>(desc[id], info, sh);
    }
}

// One problem, descriptor by value (info slot d.index of `info`).
template <int NT, int QM, int PIPE>
__global__ void __launch_bounds__(NT) wg_single_kernel(WgDesc d, int *info)
{
    __shared__ WgShared<NT, QM> sh;
    wg_instance<NT, QM, PIPE>(d, info, sh);
}

} // namespace hqr
