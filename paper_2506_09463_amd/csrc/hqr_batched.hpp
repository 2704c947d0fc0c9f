// hqr_batched.hpp -- many independent least-squares problems of uneven size
// in one persistent launch.
//
// Each workgroup (1024 threads) repeatedly takes the next instance from an
// atomic queue head (instances sorted longest-first on the host, so the
// largest start first and the tail is short) and solves it alone:
// the one-reflector-at-a-time loop of the paper's Alg. 2 with the (up, b)
// storage of Alg. 3, B riding along as trailing columns (Q^T B fused), then
// the residual norms and the back-substitution.  The data stay in global
// memory (L2); wave w owns columns j = k + w, k + w + 16, .. and its lanes
// walk down the rows, so every column access is a coalesced 512-byte read.
// Only the queue head is an atomic; every workgroup leaves the loop once the
// head passes the instance count.
#pragma once

#include "hqr_args.hpp"

namespace hqr {




HQR_DEV double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

HQR_DEV double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

HQR_DEV double *bcol(const BatchDesc &d, int64_t j)
{
    return (j < d.n) ? d.A + (size_t)j * d.lda : d.B + (size_t)(j - d.n) * d.ldb;
}

// One instance by one workgroup.  Scratch: xs (pivot tail, BATCH_MAX_ROWS),
// dots/ws (per column), sc (scalars).
HQR_DEV void batch_instance(const BatchDesc &d, int *info, double *xs, double *dots, double *sc, int *isc)
{
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t m = d.m, n = d.n, ntot = d.n + d.nrhs;
    const bool factor = d.factor != 0;
    const int64_t jlo = factor ? 0 : n;        // first column a reflector updates (beyond k)
    for (int64_t k = 0; k < n; ++k) {
        const double *ak = d.A + (size_t)k * d.lda;
        // stage the pivot column (rows k..m-1)
        for (int64_t i = k + tid; i < m; i += 1024) xs[i] = ak[i];
        if (!factor && tid == 0) {
            sc[0] = d.up[k];
            sc[3] = ak[k];                     // R[k][k] as stored
        }
        __syncthreads();
        if (!factor && sc[0] == 0.0) {         // identity reflector
            __syncthreads();
            continue;
        }
        // dots of the tail with every column j updated (and with itself when
        // factoring: ||tail||^2, max|x|, #nonzero)
        const int64_t jfirst = factor ? k : n;
        for (int64_t j = jfirst + w; j < ntot; j += BATCH_NW) {
            const double *cj = bcol(d, j);
            double s = 0.0, mx = 0.0, nz = 0.0;
            for (int64_t i = k + 1 + lane; i < m; i += 64) {
                const double xi = xs[i];
                s += xi * cj[i];
                if (j == k) {
                    mx = fmax(mx, fabs(xi));
                    nz += (xi != 0.0) ? 1.0 : 0.0;
                }
            }
            s = wave_sum(s);
            if (j == k) {
                mx = wave_max(mx);
                nz = wave_sum(nz);
                if (lane == 0) {
                    sc[1] = mx;
                    sc[2] = nz;
                }
            }
            if (lane == 0) dots[j] = s;
        }
        __syncthreads();
        if (factor && tid == 0) {
            const double x0 = xs[k];
            double upk, sk;
            if (sc[2] == 0.0) {
                upk = 0.0;
                sk = x0;
            } else {
                const double c = fmax(fabs(x0), sc[1]);
                double nu;
                if (norm_fast_path_ok(c)) {
                    nu = sqrt(x0 * x0 + dots[k]);
                } else {
                    double t = 0.0;
                    for (int64_t i = k + 1; i < m; ++i) {
                        const double y = xs[i] / c;
                        t += y * y;
                    }
                    const double x0c = x0 / c;
                    nu = c * sqrt(x0c * x0c + t);
                }
                sk = (x0 >= 0.0) ? -nu : nu;
                upk = x0 - sk;
            }
            sc[0] = upk;
            sc[3] = sk;
            d.up[k] = upk;
        }
        __syncthreads();
        const double upk = sc[0], sk = sc[3];
        if (upk != 0.0) {
            const double bk = upk * sk;
            const int64_t jup = factor ? k + 1 : jlo;
            for (int64_t j = jup + w; j < ntot; j += BATCH_NW) {
                double *cj = bcol(d, j);
                const double wj = (upk * cj[k] + dots[j]) / bk;
                for (int64_t i = k + lane; i < m; i += 64) {
                    const double v = (i == k) ? upk : xs[i];
                    cj[i] += wj * v;
                }
            }
        }
        if (factor && tid == 0) d.A[(size_t)k * d.lda + k] = sk;
        __syncthreads();
    }
    // residual norms
    if (d.resnorm) {
        for (int64_t c = w; c < d.nrhs; c += BATCH_NW) {
            const double *bc = d.B + (size_t)c * d.ldb;
            double s = 0.0, mx = 0.0;
            for (int64_t i = n + lane; i < m; i += 64) {
                s += bc[i] * bc[i];
                mx = fmax(mx, fabs(bc[i]));
            }
            s = wave_sum(s);
            mx = wave_max(mx);
            if (mx != 0.0 && !norm_fast_path_ok(mx)) {
                double t = 0.0;
                for (int64_t i = n + lane; i < m; i += 64) {
                    const double y = bc[i] / mx;
                    t += y * y;
                }
                t = wave_sum(t);
                if (lane == 0) d.resnorm[c] = mx * sqrt(t);
            } else if (lane == 0) {
                d.resnorm[c] = sqrt(s);
            }
        }
    }
    // back-substitution; smallest k with R[k][k] == 0 blocks it
    if (tid == 0) {
        int f = 0;
        for (int64_t k = 0; k < n; ++k)
            if (d.A[(size_t)k * d.lda + k] == 0.0) {
                f = (int)(k + 1);
                break;
            }
        isc[0] = f;
        info[d.index] = f;
    }
    __syncthreads();
    if (isc[0] == 0) {
        for (int64_t i = n - 1; i >= 0; --i) {
            const double *ri = d.A + (size_t)i * d.lda;
            const double rii = ri[i];
            for (int64_t c = 0; c < d.nrhs; ++c) {
                double *bc = d.B + (size_t)c * d.ldb;
                const double xi = bc[i] / rii;
                for (int64_t r = tid; r < i; r += 1024) bc[r] -= ri[r] * xi;
                __syncthreads();
                if (tid == 0) bc[i] = xi;
            }
            __syncthreads();
        }
    }
    __syncthreads();
}

__global__ void __launch_bounds__(1024) batched_lsq_kernel(BatchArgs p)
{
    __shared__ double xs[BATCH_MAX_ROWS];
    __shared__ double dots[BATCH_MAX_COLS];
    __shared__ double sc[4];
    __shared__ int isc[2];
    for (;;) {
        if (threadIdx.x == 0) isc[1] = atomicAdd(p.head, 1);
        __syncthreads();
        const int id = isc[1];
        __syncthreads();
        if (id >= p.count) break;
        batch_instance(p.desc[id], p.info, xs, dots, sc, isc);
    }
}

} // namespace hqr
