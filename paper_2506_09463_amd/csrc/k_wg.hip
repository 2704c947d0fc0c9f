// k_wg.hip -- the one-workgroup kernel variants (hqr_wg.hpp) and their
// launch functions.
#include "hqr_wg.hpp"

#include <algorithm>

namespace hqr {

namespace {

typedef void (*wg_batched_fn)(const WgDesc *, int, int *, int *);
typedef void (*wg_single_fn)(WgDesc, int *);

struct WgKernels {
    wg_batched_fn batched;
    wg_single_fn single;
};

template <int NT, int QM>
WgVariant describe(const char *name, int index)
{
    // workgroups per CU the LDS allows (at most 2 are launched per CU)
    const int per_cu = (int)std::max<size_t>(1, (160 * 1024) / sizeof(WgShared<NT, QM>));
    return WgVariant{name, NT, QM, std::min(per_cu, 2), wg_max_rows<NT, QM>(), wg_max_x<NT, QM>(), index};
}

#define HQR_WG_VARIANTS(X)                                                                                        \
    X(0, 64, 2)   /* m <= 128, one wave */                                                                        \
    X(1, 64, 4)   /* m <= 256, one wave */                                                                        \
    X(2, 128, 1)  /* m <= 128 */                                                                                  \
    X(3, 256, 1)  /* m <= 256 */                                                                                  \
    X(4, 128, 4)  /* m <= 512 */                                                                                  \
    X(5, 256, 2)  /* m <= 512 */                                                                                  \
    X(6, 256, 4)  /* m <= 1024 */

const WgKernels kernels[] = {
#define HQR_K(I, NT, QM) {wg_batched_kernel<NT, QM>, wg_single_kernel<NT, QM>},
    HQR_WG_VARIANTS(HQR_K)
#undef HQR_K
};

} // namespace

const WgVariant *wg_variants(int *count)
{
    static const WgVariant v[] = {
#define HQR_D(I, NT, QM) describe<NT, QM>("wg" #NT "x" #QM, I),
        HQR_WG_VARIANTS(HQR_D)
#undef HQR_D
    };
    *count = (int)(sizeof(v) / sizeof(v[0]));
    return v;
}

hipError_t k_wg_single(const WgVariant *v, hipStream_t s, const WgDesc &d, int *info)
{
    HQR_LAUNCH(K_SMALL, kernels[v->index].single, dim3(1), dim3(v->nt), 0, s, d, info);
    return hipGetLastError();
}

hipError_t k_wg_batched(const WgVariant *v, int grid, hipStream_t s, const WgDesc *desc, int count, int *head,
                        int *info)
{
    HQR_LAUNCH(K_BATCHED, kernels[v->index].batched, dim3(grid), dim3(v->nt), 0, s, desc, count, head, info);
    return hipGetLastError();
}

} // namespace hqr
