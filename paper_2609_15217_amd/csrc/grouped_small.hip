/* Grouped-batch kernel for sizes 1..16 (see kernels_ragged.h), held to 4
 * waves per SIMD like the ragged kernel for the same sizes. */
#include "kernels_ragged.h"

namespace lupp {

__global__ void __launch_bounds__(kRaggedThreads) __attribute__((amdgpu_waves_per_eu(4)))
    k_grouped_small(GroupedArgs a)
{
    grouped_run<1, kRaggedSmallMax>(a, (int)xcd_block(blockIdx.x, gridDim.x));
}

hipError_t grouped_small_launch(const GroupedArgs &a, unsigned items, hipStream_t st)
{
    hipLaunchKernelGGL(k_grouped_small, dim3(items), dim3(kRaggedThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace lupp
