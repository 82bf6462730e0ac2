/* Persistent kernel of the ragged path for sizes 17..32 (see kernels_ragged.h). */
#include "kernels_ragged.h"

namespace lupp {

/* Sizes 17..32 (items 0 .. large_items-1): 16-lane segments need up to ~240
 * VGPRs, so this kernel runs 2 waves per SIMD. */
__global__ void __launch_bounds__(kRaggedThreads) __attribute__((amdgpu_waves_per_eu(2)))
    k_ragged_large(RaggedArgs a)
{
    ragged_persistent_loop<kRaggedSmallMax + 1, 32>(a, &a.plan->next_item, a.plan->large_items);
}

hipError_t ragged_large_launch(const RaggedArgs &a, unsigned grid, hipStream_t st)
{
    hipLaunchKernelGGL(k_ragged_large, dim3(grid), dim3(kRaggedThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace lupp
