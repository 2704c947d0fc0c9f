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

template <int NT, int QM, int PIPE>
WgVariant describe(const char *name, int index)
{
    const int per_cu = (int)std::max<size_t>(1, (160 * 1024) / sizeof(WgShared<NT, QM>));
    return WgVariant{name, NT, QM, PIPE, std::min(per_cu, 8), wg_max_rows<NT, QM>(), wg_max_x<NT, QM>(), index};
}

// (index, threads, rows per thread, 16-row blocks loaded together).  The
// 256-thread variants differ only in rows per thread and load scheduling,
// never in arithmetic, so the batched launch may use any of them.
#define HQR_WG_VARIANTS(X)                                                                                        \
    X(0, 64, 2, 4)    /* m <= 128, one wave */                                                                    \
    X(1, 64, 4, 4)    /* m <= 256, one wave */                                                                    \
    X(2, 128, 1, 4)   /* m <= 128 */                                                                              \
    X(3, 256, 1, 4)   /* m <= 256 */                                                                              \
    X(4, 128, 4, 4)   /* m <= 512 */                                                                              \
    X(5, 256, 2, 4)   /* m <= 512 */                                                                              \
    X(6, 256, 4, 4)   /* m <= 1024 */                                                                             \
    X(7, 256, 1, 2)                                                                                               \
    X(8, 256, 1, 8)                                                                                               \
    X(9, 256, 2, 2)                                                                                               \
    X(10, 256, 2, 8)                                                                                              \
    X(11, 256, 4, 2)                                                                                              \
    X(12, 256, 4, 8)

const WgKernels kernels[] = {
#define HQR_K(I, NT, QM, P) {wg_batched_kernel<NT, QM, P>, wg_single_kernel<NT, QM, P>},
    HQR_WG_VARIANTS(HQR_K)
#undef HQR_K
};

} // namespace

const WgVariant *wg_variants(int *count)
{
    static const WgVariant v[] = {
#define HQR_D(I, NT, QM, P) describe<NT, QM, P>((P) == 4 ? "wg" #NT "x" #QM : "wg" #NT "x" #QM "p" #P, I),
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
