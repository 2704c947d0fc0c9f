// k_blocked.hip -- launch functions of the blocked-path kernels
// (hqr_blocked.hpp): panel columns, V^T X, W', the trailing update, the
// triangular solve, residual norms and the refinement kernels.
#include "hqr_blocked.hpp"

#include <algorithm>

namespace hqr {

hipError_t k_panel_col(dim3 grid, hipStream_t s, const PanelArgs &a)
{
    HQR_LAUNCH(K_PANEL, panel_col_kernel, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t k_vtx(bool f32, bool with_v, dim3 grid, hipStream_t s, const VtxArgs &a)
{
    if (with_v) {
        if (f32) HQR_LAUNCH(K_VTX, (vtx_kernel<true, true>), grid, dim3(256), 0, s, a);
        else HQR_LAUNCH(K_VTX, (vtx_kernel<false, true>), grid, dim3(256), 0, s, a);
    } else {
        if (f32) HQR_LAUNCH(K_VTX, (vtx_kernel<true, false>), grid, dim3(256), 0, s, a);
        else HQR_LAUNCH(K_VTX, (vtx_kernel<false, false>), grid, dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t k_wsolve(bool narrow, dim3 grid, hipStream_t s, const WArgs &a)
{
    if (narrow) HQR_LAUNCH(K_WSOLVE, wsolve_narrow_kernel, grid, dim3(256), 0, s, a);
    else HQR_LAUNCH(K_WSOLVE, wsolve_kernel, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t k_update(bool narrow, bool f32, dim3 grid, hipStream_t s, const UpdArgs &a)
{
    if (narrow) {
        if (f32) HQR_LAUNCH(K_UPDATE, update_narrow_kernel<true>, grid, dim3(256), 0, s, a);
        else HQR_LAUNCH(K_UPDATE, update_narrow_kernel<false>, grid, dim3(256), 0, s, a);
    } else {
        if (f32) HQR_LAUNCH(K_UPDATE, update_kernel<true>, grid, dim3(256), 0, s, a);
        else HQR_LAUNCH(K_UPDATE, update_kernel<false>, grid, dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t k_diag_check(hipStream_t s, const double *A, int64_t lda, int64_t n, int *info)
{
    HQR_LAUNCH(K_DIAG, diag_check_kernel, dim3(1), dim3(256), 0, s, A, lda, n, info);
    return hipGetLastError();
}

hipError_t k_trsv(bool trans, int nrhs, dim3 grid, hipStream_t s, const TrsvArgs &a)
{
    if (nrhs == 1) {
        if (trans) HQR_LAUNCH(K_TRSV, (trsv_kernel<true, 1>), grid, dim3(256), 0, s, a);
        else HQR_LAUNCH(K_TRSV, (trsv_kernel<false, 1>), grid, dim3(256), 0, s, a);
    } else {
        if (trans) HQR_LAUNCH(K_TRSV, (trsv_kernel<true, TRSV_MAXRHS>), grid, dim3(256), 0, s, a);
        else HQR_LAUNCH(K_TRSV, (trsv_kernel<false, TRSV_MAXRHS>), grid, dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t k_resnorm(dim3 grid, hipStream_t s, const double *B, int64_t ldb, int64_t n, int64_t m, double *out)
{
    HQR_LAUNCH(K_RESNORM, resnorm_kernel, grid, dim3(256), 0, s, B, ldb, n, m, out);
    return hipGetLastError();
}

hipError_t k_fill_int(hipStream_t s, int *p, int v, int64_t count)
{
    // one workgroup for the small fills, up to 64 for the back-substitution's
    // published-value buffer (up to 8 x n doubles)
    const int grid = (int)std::min<int64_t>(64, std::max<int64_t>(1, (count + 4095) / 4096));
    HQR_LAUNCH(K_FILL, fill_int_kernel, dim3(grid), dim3(256), 0, s, p, v, count);
    return hipGetLastError();
}

hipError_t k_or_int(hipStream_t s, int *p, int v)
{
    HQR_LAUNCH(K_FILL, or_int_kernel, dim3(1), dim3(64), 0, s, p, v);
    return hipGetLastError();
}

hipError_t k_eye(hipStream_t s, double *Q, int64_t ldq, int64_t m, int64_t k)
{
    const unsigned g = (unsigned)std::min<int64_t>(std::max<int64_t>(k, 1), 4096);
    HQR_LAUNCH(K_FILL, eye_kernel, dim3(g), dim3(256), 0, s, Q, ldq, m, k);
    return hipGetLastError();
}

hipError_t k_refine_init(hipStream_t s, const RefineArgs &a)
{
    HQR_LAUNCH(K_REFINE, refine_init_kernel, dim3(1), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t k_resid(bool all, hipStream_t s, const RefineArgs &a)
{
    const dim3 g((unsigned)((a.m + RESID_ROWS - 1) / RESID_ROWS), (unsigned)((a.nrhs + RESID_NR - 1) / RESID_NR));
    HQR_LAUNCH(K_REFINE, resid_kernel, g, dim3(256), 0, s, a, all ? 1 : 0);
    return hipGetLastError();
}

hipError_t k_gemvt(hipStream_t s, const RefineArgs &a)
{
    const dim3 g((unsigned)((a.n + 3) / 4), (unsigned)a.nrhs);
    HQR_LAUNCH(K_REFINE, gemvt_kernel, g, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t k_csne_update(hipStream_t s, const RefineArgs &a, int step)
{
    HQR_LAUNCH(K_REFINE, csne_update_kernel, dim3((unsigned)a.nrhs), dim3(1024), 0, s, a, step);
    return hipGetLastError();
}

hipError_t k_refine_verdict(hipStream_t s, const RefineArgs &a, int *verdict, int *info, int *iters, bool or_info)
{
    HQR_LAUNCH(K_REFINE, refine_verdict_kernel, dim3(1), dim3(64), 0, s, a, verdict, info, iters, or_info ? 1 : 0);
    return hipGetLastError();
}

} // namespace hqr
