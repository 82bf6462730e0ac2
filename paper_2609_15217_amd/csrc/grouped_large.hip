/* Grouped-batch kernel for sizes 17..32 (see kernels_ragged.h): the register
 * budget of the ragged kernel for the same sizes (2 waves per SIMD). */
#include "kernels_ragged.h"

namespace lupp {

__global__ void __launch_bounds__(kRaggedThreads) __attribute__((amdgpu_waves_per_eu(2)))
    k_grouped_large(GroupedArgs a)
{
    grouped_run<kRaggedSmallMax + 1, 32>(a, (int)xcd_block(blockIdx.x, gridDim.x));
}

hipError_t grouped_large_launch(const GroupedArgs &a, unsigned items, hipStream_t st)
{
    hipLaunchKernelGGL(k_grouped_large, dim3(items), dim3(kRaggedThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace lupp
