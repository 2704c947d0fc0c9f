// k_tsqr.hip -- launch functions of the TSQR panel's data-movement kernels
// (hqr_tsqr.hpp); the block factorizations and applications are batched
// launches of the one-workgroup kernel.
#include "hqr_tsqr.hpp"

#include <algorithm>

namespace hqr {

hipError_t k_tsqr_desc(hipStream_t s, const TsqrArgs &a)
{
    int64_t total = 0;
    for (int l = 0; l < a.nlev; ++l) total += a.lev[l].nblk;
    const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 1024));
    HQR_LAUNCH(K_TSQR, tsqr_desc_kernel, dim3(g), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t k_tsqr_gather(hipStream_t s, const TsqrArgs &a, int l)
{
    HQR_LAUNCH(K_TSQR, tsqr_gather_kernel, dim3((unsigned)a.lev[l].nblk), dim3(256), 0, s, a, l);
    return hipGetLastError();
}

hipError_t k_tsqr_scatter(hipStream_t s, const TsqrArgs &a, int l)
{
    HQR_LAUNCH(K_TSQR, tsqr_scatter_kernel, dim3((unsigned)((a.lev[l].rows + 255) / 256)), dim3(256), 0, s, a, l);
    return hipGetLastError();
}

hipError_t k_tsqr_final(hipStream_t s, const TsqrArgs &a, double *Ap, int64_t lda, double *r1, double *r1inv,
                        double *sign)
{
    HQR_LAUNCH(K_TSQR, tsqr_r_kernel, dim3(1), dim3(256), 0, s, a, r1, r1inv, sign);
    if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
    HQR_LAUNCH(K_TSQR, tsqr_final_kernel, dim3((unsigned)((a.lev[0].rows + 255) / 256)), dim3(256), 0, s, a, Ap,
               lda, (const double *)sign);
    return hipGetLastError();
}

} // namespace hqr
