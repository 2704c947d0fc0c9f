// k_batched.hip -- launch function of the streaming batched kernel
// (hqr_batched.hpp).
#include "hqr_batched.hpp"

namespace hqr {

hipError_t k_batched_lsq(dim3 grid, hipStream_t s, const BatchArgs &a)
{
    HQR_LAUNCH(K_BATCHED, batched_lsq_kernel, grid, dim3(1024), 0, s, a);
    return hipGetLastError();
}

} // namespace hqr
