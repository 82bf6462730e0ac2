/* Ragged kernel of size class 0, sizes 24..32 (see kernels_ragged.h): 16-lane
 * segments need up to 217 VGPRs, so it runs 2 waves per SIMD. */
#include "kernels_ragged.h"

namespace lupp {

__global__ void __launch_bounds__(kRaggedThreads)
    __attribute__((amdgpu_waves_per_eu(ragged_class_waves(0)))) k_ragged_c0(RaggedArgs a)
{
    ragged_class_loop<0>(a);
}

hipError_t ragged_c0_launch(const RaggedArgs &a, unsigned grid, hipStream_t st)
{
    hipLaunchKernelGGL(k_ragged_c0, dim3(grid), dim3(kRaggedThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace lupp
