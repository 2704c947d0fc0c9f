// hqr_lse.hpp -- the small data-movement kernels of the equality-constrained
// least-squares solve (null-space method): a tiled transpose, the update
// b -= M y of the right-hand side by the constrained part, and the
// combination of the two solves' info codes.
#pragma once

#include "hqr_args.hpp"

namespace hqr {

// out (cols x rows, leading dimension ldo) <- in^T (in: rows x cols, ldi).
// 64 x 64 tiles through LDS: reads and writes are both coalesced.  grid:
// (ceil(rows/64), ceil(cols/64)), 256 threads.
__global__ void __launch_bounds__(256) transpose_kernel(const double *in, int64_t ldi, double *out, int64_t ldo,
                                                        int64_t rows, int64_t cols)
{
    __shared__ double t[64][65];
    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * 64, c0 = (int64_t)blockIdx.y * 64;
    for (int e = tid; e < 64 * 64; e += 256) {
        const int r = e & 63, c = e >> 6;
        if (r0 + r < rows && c0 + c < cols) t[c][r] = in[(size_t)(r0 + r) + (size_t)(c0 + c) * ldi];
    }
    __syncthreads();
    for (int e = tid; e < 64 * 64; e += 256) {
        const int c = e & 63, r = e >> 6;     // out row c0 + c, out column r0 + r
        if (r0 + r < rows && c0 + c < cols) out[(size_t)(c0 + c) + (size_t)(r0 + r) * ldo] = t[c][r];
    }
}

// b[i] -= sum_{j < p} M[i][j] y[j] for i < m; y staged in LDS in chunks.
// One thread per row.
__global__ void __launch_bounds__(256) gemv_sub_kernel(const double *M, int64_t ldm, const double *y, double *b,
                                                       int64_t m, int64_t p)
{
    __shared__ double ys[1024];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double s = 0.0;
    for (int64_t j0 = 0; j0 < p; j0 += 1024) {
        const int64_t nj = min<int64_t>(1024, p - j0);
        __syncthreads();
        for (int64_t j = threadIdx.x; j < nj; j += 256) ys[j] = y[j0 + j];
        __syncthreads();
        if (i < m)
            for (int64_t j = 0; j < nj; ++j) s += M[(size_t)i + (size_t)(j0 + j) * ldm] * ys[j];
    }
    if (i < m) b[i] -= s;
}

// dst[0:n] <- src[0:n]
__global__ void __launch_bounds__(256) copy_vec_kernel(const double *src, double *dst, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) dst[i] = src[i];
}

// info = info_c (a zero pivot of C's factor, k+1), else p + info_r (a zero
// pivot of the reduced problem), else 0.  One thread.
__global__ void lse_info_kernel(int *info, const int *info_c, const int *info_r, int64_t p)
{
    if (threadIdx.x != 0) return;
    const int ic = info_c ? *info_c : 0, ir = info_r ? *info_r : 0;
    *info = ic ? ic : (ir ? (int)p + ir : 0);
}

} // namespace hqr
