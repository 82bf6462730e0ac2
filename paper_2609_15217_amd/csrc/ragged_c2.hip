/* Ragged kernel of size class 2, sizes 1..16 (see kernels_ragged.h), held to
 * 3 waves per SIMD. A persistent form of it at 4 waves per SIMD spilled 144
 * bytes per lane (80 once the lane table became word-sized), and on MI355X
 * that build returned wrong, run-to-run different solutions for some size-16
 * systems (7 to 42 of 200 sampled per run) while the per-size kernels built
 * from the same solver code, without scratch, were exact; this kernel is
 * kept free of scratch memory. */
#include "kernels_ragged.h"

namespace lupp {

__global__ void __launch_bounds__(kRaggedThreads)
    __attribute__((amdgpu_waves_per_eu(ragged_class_waves(2)))) k_ragged_c2(RaggedArgs a)
{
    ragged_class_loop<2>(a);
}

hipError_t ragged_c2_launch(const RaggedArgs &a, unsigned grid, hipStream_t st)
{
    hipLaunchKernelGGL(k_ragged_c2, dim3(grid), dim3(kRaggedThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace lupp
