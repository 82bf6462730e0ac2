/* Ragged kernel of size class 1, sizes 17..23 (see kernels_ragged.h): 16-lane
 * segments need at most 164 VGPRs, so it runs 3 waves per SIMD. */
#include "kernels_ragged.h"

namespace lupp {

__global__ void __launch_bounds__(kRaggedThreads)
    __attribute__((amdgpu_waves_per_eu(ragged_class_waves(1)))) k_ragged_c1(RaggedArgs a)
{
    ragged_class_loop<1>(a);
}

hipError_t ragged_c1_launch(const RaggedArgs &a, unsigned grid, hipStream_t st)
{
    hipLaunchKernelGGL(k_ragged_c1, dim3(grid), dim3(kRaggedThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace lupp
