/* Persistent kernel of the ragged path for sizes 1..16 (see kernels_ragged.h). */
#include "kernels_ragged.h"

namespace lupp {

/* Sizes 1..16 (items large_items .. total_items-1), held to 3 waves per SIMD
 * (140 VGPRs, no scratch). At 4 waves per SIMD the compiler spilled 144
 * bytes per lane (80 once the lane table became word-sized), and on MI355X
 * that build returned wrong, run-to-run different solutions for some size-16
 * systems (7 to 42 of 200 sampled per run) while the per-size kernels built
 * from the same solver code, without scratch, were exact; this kernel is
 * kept free of scratch memory. */
__global__ void __launch_bounds__(kRaggedThreads) __attribute__((amdgpu_waves_per_eu(3)))
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
