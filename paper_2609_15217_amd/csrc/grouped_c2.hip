/* Grouped-batch kernel of size class 2, sizes 1..16 (see kernels_ragged.h):
 * one workgroup per work item, 4 waves per SIMD. */
#include "kernels_ragged.h"

namespace lupp {

__global__ void __launch_bounds__(kRaggedThreads) __attribute__((amdgpu_waves_per_eu(4)))
    k_grouped_c2(GroupedArgs a)
{
    grouped_run<ragged_class_lo(2), ragged_class_hi(2)>(a, (int)xcd_block(blockIdx.x, gridDim.x));
}

hipError_t grouped_c2_launch(const GroupedArgs &a, unsigned items, hipStream_t st)
{
    hipLaunchKernelGGL(k_grouped_c2, dim3(items), dim3(kRaggedThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace lupp
