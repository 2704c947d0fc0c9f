// k_cqr.hip -- launch functions of the CholeskyQR2 + reconstruction panel
// kernels, the look-ahead chain and the T factor of stored panels
// (hqr_cqr.hpp).
#include "hqr_cqr.hpp"

namespace hqr {

hipError_t k_cqr_gram1(dim3 grid, hipStream_t s, const Gram1Args &a)
{
    HQR_LAUNCH(K_GRAM1, cqr_gram1_kernel, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t k_cqr_gram2(dim3 grid, hipStream_t s, const Gram2Args &a)
{
    HQR_LAUNCH(K_GRAM2, cqr_gram2_kernel, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t k_gram_reduce(hipStream_t s, const GredArgs &a)
{
    HQR_LAUNCH(K_GRED, gram_reduce_kernel, dim3(NB * NB / 64), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t k_cqr_chol(hipStream_t s, const CholArgs &a)
{
    HQR_LAUNCH(K_CQR_CHOL, cqr_chol_kernel, dim3(1), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t k_cqr_finish(dim3 grid, hipStream_t s, const FinArgs &a)
{
    HQR_LAUNCH(K_CQR_FINISH, cqr_finish_kernel, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t k_narrow_vtx(dim3 grid, hipStream_t s, const NarrowArgs &a)
{
    HQR_LAUNCH(K_NVTX, narrow_vtx_kernel, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t k_tfactor(hipStream_t s, const TArgs &a)
{
    HQR_LAUNCH(K_TFACTOR, tfactor_kernel, dim3(1), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t k_xw_reduce(hipStream_t s, const XwArgs &a)
{
    HQR_LAUNCH(K_GRED, xw_reduce_kernel, dim3(NB), dim3(256), 0, s, a);
    return hipGetLastError();
}

} // namespace hqr
