/* Grouped-batch kernel of size class 0, sizes 24..32 (see kernels_ragged.h):
 * one workgroup per work item, 2 waves per SIMD. */
#include "kernels_ragged.h"

namespace lupp {

__global__ void __launch_bounds__(kRaggedThreads) __attribute__((amdgpu_waves_per_eu(2)))
    k_grouped_c0(GroupedArgs a)
{
    grouped_run<ragged_class_lo(0), ragged_class_hi(0)>(a, (int)xcd_block(blockIdx.x, gridDim.x));
}

hipError_t grouped_c0_launch(const GroupedArgs &a, unsigned items, hipStream_t st)
{
    hipLaunchKernelGGL(k_grouped_c0, dim3(items), dim3(kRaggedThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace lupp
