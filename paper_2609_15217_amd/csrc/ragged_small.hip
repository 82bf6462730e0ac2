/* Persistent kernel of the ragged path for sizes 1..16 (see kernels_ragged.h). */
#include "kernels_ragged.h"

namespace lupp {

/* Sizes 1..16 (items large_items .. total_items-1), held to 4 waves per SIMD
 * (the register budget of its largest size). */
__global__ void __launch_bounds__(kRaggedThreads) __attribute__((amdgpu_waves_per_eu(4)))
    k_ragged_small(RaggedArgs a)
{
    ragged_persistent_loop<1, kRaggedSmallMax>(a, &a.plan->next_small, a.plan->total_items);
}

hipError_t ragged_small_launch(const RaggedArgs &a, unsigned grid, hipStream_t st)
{
    hipLaunchKernelGGL(k_ragged_small, dim3(grid), dim3(kRaggedThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace lupp
