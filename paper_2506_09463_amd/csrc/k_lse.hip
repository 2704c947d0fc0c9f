// k_lse.hip -- launch functions of the equality-constrained least-squares
// kernels (hqr_lse.hpp).
#include "hqr_lse.hpp"

#include <algorithm>

namespace hqr {

hipError_t k_transpose(hipStream_t s, const double *in, int64_t ldi, double *out, int64_t ldo, int64_t rows,
                       int64_t cols)
{
    if (rows <= 0 || cols <= 0) return hipSuccess;
    const dim3 g((unsigned)((rows + 63) / 64), (unsigned)((cols + 63) / 64));
    HQR_LAUNCH(K_FILL, transpose_kernel, g, dim3(256), 0, s, in, ldi, out, ldo, rows, cols);
    return hipGetLastError();
}

hipError_t k_gemv_sub(hipStream_t s, const double *M, int64_t ldm, const double *y, double *b, int64_t m,
                      int64_t p)
{
    if (m <= 0 || p <= 0) return hipSuccess;
    HQR_LAUNCH(K_REFINE, gemv_sub_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, M, ldm, y, b, m, p);
    return hipGetLastError();
}

hipError_t k_copy_vec(hipStream_t s, const double *src, double *dst, int64_t n)
{
    if (n <= 0) return hipSuccess;
    const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    HQR_LAUNCH(K_FILL, copy_vec_kernel, dim3(g), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

hipError_t k_lse_info(hipStream_t s, int *info, const int *info_c, const int *info_r, int64_t p)
{
    HQR_LAUNCH(K_FILL, lse_info_kernel, dim3(1), dim3(64), 0, s, info, info_c, info_r, p);
    return hipGetLastError();
}

} // namespace hqr
