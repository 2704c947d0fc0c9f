// k_chol.hip -- launch functions of the Cholesky factorization and the
// rank-one factor update (hqr_chol.hpp).
#include "hqr_chol.hpp"

namespace hqr {

hipError_t k_chol_block(hipStream_t s, double *S, int64_t lds, int64_t n, int64_t k0, int bw, double *rinv,
                        int *info)
{
    CholArgsS a{S, lds, n, k0, bw, rinv, info};
    HQR_LAUNCH(K_CQR_CHOL, chol_diag_kernel, dim3(1), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t rest = n - k0 - bw;
    if (rest <= 0) return hipSuccess;
    const unsigned T = (unsigned)((rest + 63) / 64);
    HQR_LAUNCH(K_PANEL, chol_panel_kernel, dim3(T), dim3(256), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    HQR_LAUNCH(K_UPDATE, chol_syrk_kernel, dim3(T, T), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t k_chol_update(hipStream_t s, double *R, int64_t ldr, double *v, int64_t n)
{
    if (n <= 1024) HQR_LAUNCH(K_REFINE, chol_update_kernel<1>, dim3(1), dim3(1024), 0, s, R, ldr, v, n);
    else if (n <= 2048) HQR_LAUNCH(K_REFINE, chol_update_kernel<2>, dim3(1), dim3(1024), 0, s, R, ldr, v, n);
    else HQR_LAUNCH(K_REFINE, chol_update_kernel<4>, dim3(1), dim3(1024), 0, s, R, ldr, v, n);
    return hipGetLastError();
}

} // namespace hqr
