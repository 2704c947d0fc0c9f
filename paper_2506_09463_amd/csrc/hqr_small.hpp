// hqr_small.hpp -- single-workgroup in-place Householder QR least squares.
//
// One workgroup owns a whole m x (n + nrhs) problem [A | B] in registers:
// lane c of every wave holds columns c, c+64, ..; wave w holds rows
// [w*RW, (w+1)*RW).  Per reflector k (paper Section 3, Alg. 2: the pivot
// update followed by the trailing non-pivot updates) the workgroup
//   1. reduces, over its waves, the partial dot products of the pivot tail
//      x = A[k+1:m, k] with every column it still updates (one barrier);
//   2. every thread derives the reflector (s, up, b = up*s) and the
//      coefficients w_j = (up*A[k][j] + x.a_j) / b itself, identically;
//   3. applies the reflector to its rows, and in the same pass accumulates
//      the next pivot's partial dot products.
// Q^T B is fused: the nrhs columns of B ride along as trailing columns.
// After the factorization, the back-substitution and the residual norms run
// out of LDS.  Modes:
//   SMALL_FACTOR  generate reflectors from A (writes A, up);
//   otherwise     apply the stored reflectors (A, up read-only) to B;
//   SMALL_SOLVE   back-substitute R x = (Q^T B)[0:n];
//   SMALL_RESNORM resnorm[c] = ||(Q^T B)[n:m, c]||.
#pragma once

#include "hqr_device.hpp"

namespace hqr {

enum : int { SMALL_FACTOR = 1, SMALL_SOLVE = 2, SMALL_RESNORM = 4 };

struct SmallArgs {
    int m, n, nrhs, mode;
    int64_t lda, ldb;
    double *A;
    double *B;
    double *up;
    double *resnorm;
    int *info;
    int ldl; // leading dimension of the LDS staging copy (>= m)
    long long *tstamp; // optional phase timestamps (thread 0), may be null
};

// Leading dimension of the LDS staging copy: odd, so that lanes reading one
// row across columns spread over the banks.
static inline int small_ldl(int m) { return (m & 1) ? m : m + 1; }

// LDS bytes beyond the static arrays: the staging copy of [A | B].
static inline size_t small_dyn_lds(int m, int n, int nrhs)
{
    return sizeof(double) * (size_t)small_ldl(m) * (size_t)(n + nrhs);
}

// a[q] for a runtime q < Q (select chain; the array stays in registers)
template <int Q>
HQR_DEV double pickq(const double (&a)[Q], int q)
{
    double r = a[0];
#pragma unroll
    for (int t = 1; t < Q; ++t) r = (t == q) ? a[t] : r;
    return r;
}

template <int NW, int RW, int Q>
__global__ void __launch_bounds__(NW * 64) small_lsq_kernel(SmallArgs p)
{
    constexpr int NT = NW * 64;
    constexpr int NC = Q * 64;
    constexpr int PW = NC + 2; // partial dots, then max|x|, then #nonzero
    __shared__ double part[2][NW][PW];
    __shared__ double prow[2][NC];
    __shared__ double scal[NW];
    __shared__ double sup[NC];   // reflector leading components (global up[] at the end)
    __shared__ double vcol[NW][RW], xcol[NW][RW];
    __shared__ int sinfo;
    extern __shared__ double lds[];

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int m = p.m, n = p.n, nrhs = p.nrhs, ntot = n + nrhs, L = p.ldl;
    const bool factor = (p.mode & SMALL_FACTOR) != 0;
    const int row0 = w * RW;
    int tsi = 0;
#define HQR_STS()                                                                \
    do {                                                                         \
        if (p.tstamp && tid == 0) p.tstamp[tsi] = (long long)wall_clock64();     \
        ++tsi;                                                                   \
    } while (0)
    HQR_STS();

    // ---- stage [A | B] into LDS (coalesced), then into registers
    for (int idx = tid; idx < m * ntot; idx += NT) {
        const int c = idx / m, i = idx - c * m;
        lds[c * L + i] = (c < n) ? HQR_AT(p.A, i, c, p.lda) : HQR_AT(p.B, i, c - n, p.ldb);
    }
    if (tid == 0) sinfo = 0;
    // apply mode reads the stored up[] once; no global memory in the step loop
    if (!factor)
        for (int k = tid; k < n; k += NT) sup[k] = p.up[k];
    __syncthreads();

    double a[RW][Q];
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int i = row0 + r, j = lane + 64 * q;
            a[r][q] = (i < m && j < ntot) ? lds[j * L + i] : 0.0;
        }

    // Columns updated by reflector k: (k, ntot) when factoring, [n, ntot) else.
    // ---- partials of step 0: x = column 0, rows > 0
    {
        double pn[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) pn[q] = 0.0;
        double mx = 0.0, nz = 0.0;
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const int i = row0 + r;
            if (i >= m) break;
            if (i == 0) {
#pragma unroll
                for (int q = 0; q < Q; ++q) prow[0][lane + 64 * q] = a[r][q];
                continue;
            }
            const double xi = readlane_f64(a[r][0], 0);
#pragma unroll
            for (int q = 0; q < Q; ++q) pn[q] += xi * a[r][q];
            mx = fmax(mx, fabs(xi));
            nz += (xi != 0.0) ? 1.0 : 0.0;
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) part[0][w][lane + 64 * q] = pn[q];
        if (lane == 0) {
            part[0][w][NC] = mx;
            part[0][w][NC + 1] = nz;
        }
    }
    __syncthreads();

    HQR_STS();
    for (int k = 0; k < n; ++k) {
        const int par = k & 1, nxt = par ^ 1;
        // ---- reflector k, derived identically by every thread
        double up_k, s_k;
        const double x0 = prow[par][k];
        if (factor) {
            double ssq = 0.0, mx = 0.0, nz = 0.0;
#pragma unroll
            for (int q = 0; q < NW; ++q) {
                ssq += part[par][q][k];
                mx = fmax(mx, part[par][q][NC]);
                nz += part[par][q][NC + 1];
            }
            if (nz == 0.0) {
                up_k = 0.0;
                s_k = x0;
            } else {
                const double c = fmax(fabs(x0), mx);
                double nu;
                if (norm_fast_path_ok(c)) {
                    nu = sqrt(x0 * x0 + ssq);
                } else {
                    // rare: scaled re-reduction of the tail (uniform branch)
                    double t = 0.0;
                    const int kq = k >> 6, kl = k & 63;
#pragma unroll
                    for (int r = 0; r < RW; ++r) {
                        const int i = row0 + r;
                        if (i > k && i < m) {
                            double xv = 0.0;
#pragma unroll
                            for (int q = 0; q < Q; ++q)
                                if (q == kq) xv = a[r][q];
                            const double xi = readlane_f64(xv, kl) / c;
                            t += xi * xi;
                        }
                    }
                    if (lane == 0) scal[w] = t;
                    __syncthreads();
                    double tot = 0.0;
#pragma unroll
                    for (int q = 0; q < NW; ++q) tot += scal[q];
                    const double x0c = x0 / c;
                    nu = c * sqrt(x0c * x0c + tot);
                    __syncthreads();
                }
                s_k = (x0 >= 0.0) ? -nu : nu;
                up_k = x0 - s_k;
            }
            if (tid == 0) sup[k] = up_k;
        } else {
            up_k = sup[k];
            s_k = x0; // R[k][k] as stored
        }
        const bool skip = (up_k == 0.0);
        const double b_k = up_k * s_k;

        double wj[Q];
        bool act[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int j = lane + 64 * q;
            act[q] = !skip && j < ntot && (factor ? j > k : j >= n);
            double d = 0.0;
            if (act[q]) {
#pragma unroll
                for (int v = 0; v < NW; ++v) d += part[par][v][j];
            }
            wj[q] = act[q] ? (up_k * prow[par][j] + d) / b_k : 0.0;
        }
        const int k1 = k + 1;
        const bool have_next = k1 < n;

        // ---- apply H_k to my rows; accumulate the partials of step k+1.
        // Columns k and k+1 of this wave's rows are broadcast through LDS by
        // their owner lanes (same wave: program order orders the accesses);
        // every lane recomputes the updated column k+1 (x') itself with the
        // same fused multiply-add its owner uses.
        const int kq = k >> 6, kl = k & 63, k1q = k1 >> 6, k1l = k1 & 63;
        double wk1 = 0.0;
        if (factor && have_next && !skip) {
            double d = 0.0;
#pragma unroll
            for (int v = 0; v < NW; ++v) d += part[par][v][k1];
            wk1 = (up_k * prow[par][k1] + d) / b_k;
        }
        if (lane == kl) {
#pragma unroll
            for (int r = 0; r < RW; ++r) vcol[w][r] = pickq<Q>(a[r], kq);
        }
        if (lane == k1l && have_next) {
#pragma unroll
            for (int r = 0; r < RW; ++r) xcol[w][r] = pickq<Q>(a[r], k1q);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        double vv[RW], xv[RW];
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            vv[r] = vcol[w][r];
            xv[r] = xcol[w][r];
        }
        const int rb = __builtin_amdgcn_readfirstlane(row0);
        const bool upd1 = factor && !skip;
        double pn[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) pn[q] = 0.0;
        double mx = 0.0, nz = 0.0;
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const int i = rb + r; // wave-uniform
            if (i < k || i >= m) continue;
            const double vi = (i == k) ? up_k : vv[r];
            // select, not multiply by zero: finished columns must not pick
            // up NaN/Inf from the reflector
#pragma unroll
            for (int q = 0; q < Q; ++q) a[r][q] = act[q] ? a[r][q] + wj[q] * vi : a[r][q];
            if (factor && i == k) {
#pragma unroll
                for (int q = 0; q < Q; ++q) a[r][q] = (lane == kl && q == kq) ? s_k : a[r][q];
            }
            if (!have_next) continue;
            if (i == k1) {
#pragma unroll
                for (int q = 0; q < Q; ++q) prow[nxt][lane + 64 * q] = a[r][q];
            } else if (i > k1) {
                const double xi = upd1 ? xv[r] + wk1 * vi : xv[r];
#pragma unroll
                for (int q = 0; q < Q; ++q) pn[q] += xi * a[r][q];
                mx = fmax(mx, fabs(xi));
                nz += (xi != 0.0) ? 1.0 : 0.0;
            }
        }
        if (have_next) {
#pragma unroll
            for (int q = 0; q < Q; ++q) part[nxt][w][lane + 64 * q] = pn[q];
            if (lane == 0) {
                part[nxt][w][NC] = mx;
                part[nxt][w][NC + 1] = nz;
            }
        }
        __syncthreads();
    }

    HQR_STS();
    // ---- registers -> LDS
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int i = row0 + r, j = lane + 64 * q;
            if (i < m && j < ntot) lds[j * L + i] = a[r][q];
        }
    __syncthreads();

    // ---- residual norms of (Q^T B)[n:m, c]
    if ((p.mode & SMALL_RESNORM) && p.resnorm) {
        for (int c = w; c < nrhs; c += NW) {
            const double *col = lds + (n + c) * L;
            double ss = 0.0, mx = 0.0;
            for (int i = n + lane; i < m; i += 64) {
                ss += col[i] * col[i];
                mx = fmax(mx, fabs(col[i]));
            }
            for (int o = 32; o > 0; o >>= 1) {
                ss += __shfl_xor(ss, o);
                mx = fmax(mx, __shfl_xor(mx, o));
            }
            if (!norm_fast_path_ok(mx) && mx != 0.0) {
                double t = 0.0;
                for (int i = n + lane; i < m; i += 64) {
                    const double y = col[i] / mx;
                    t += y * y;
                }
                for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
                if (lane == 0) p.resnorm[c] = mx * sqrt(t);
            } else if (lane == 0) {
                p.resnorm[c] = sqrt(ss);
            }
        }
    }

    HQR_STS();
    // ---- back-substitution: smallest k with R[k][k] == 0 blocks the solve
    if (p.mode & SMALL_SOLVE) {
        if (tid == 0) {
            int f = 0;
            for (int k = 0; k < n; ++k)
                if (lds[k * L + k] == 0.0) {
                    f = k + 1;
                    break;
                }
            sinfo = f;
        }
        __syncthreads();
        if (sinfo == 0) {
            for (int c = w; c < nrhs; c += NW) {
                double *x = lds + (n + c) * L;
                for (int i = n - 1; i >= 0; --i) {
                    const double xi = x[i] / lds[i * L + i];
                    __builtin_amdgcn_wave_barrier();
                    for (int r = lane; r < i; r += 64) x[r] -= lds[i * L + r] * xi;
                    if (lane == 0) x[i] = xi;
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                }
            }
        }
        __syncthreads();
        if (tid == 0 && p.info) *p.info = sinfo;
    } else if (tid == 0 && p.info) {
        *p.info = 0;
    }
    __syncthreads();

    HQR_STS();
    // ---- LDS -> global
    if (factor)
        for (int k = tid; k < n; k += NT) p.up[k] = sup[k];
    const int c0 = factor ? 0 : n;
    for (int idx = tid + c0 * m; idx < m * ntot; idx += NT) {
        const int c = idx / m, i = idx - c * m;
        if (c < n) HQR_AT(p.A, i, c, p.lda) = lds[c * L + i];
        else HQR_AT(p.B, i, c - n, p.ldb) = lds[c * L + i];
    }
    HQR_STS();
#undef HQR_STS
}

} // namespace hqr
