/* Grouped-batch kernel of size class 1, sizes 17..23 (see kernels_ragged.h):
 * one workgroup per work item, 3 waves per SIMD. */
#include "kernels_ragged.h"

namespace lupp {

__global__ void __launch_bounds__(kRaggedThreads) __attribute__((amdgpu_waves_per_eu(3)))
    k_grouped_c1(GroupedArgs a)
{
    grouped_run<ragged_class_lo(1), ragged_class_hi(1)>(a, (int)xcd_block(blockIdx.x, gridDim.x));
}

hipError_t grouped_c1_launch(const GroupedArgs &a, unsigned items, hipStream_t st)
{
    hipLaunchKernelGGL(k_grouped_c1, dim3(items), dim3(kRaggedThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace lupp
