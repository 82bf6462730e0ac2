/* Ragged (mixed-size) batches: device-side grouping by size and two
 * persistent launches, one per size class (see kernels_ragged.h). */
#include <cstring>

#include "kernels_ragged.h"

namespace lupp {

/* clear the per-call counters (a kernel rather than a memset, so the whole
 * sequence can be captured in a graph) */
__global__ void k_ragged_zero(RaggedPlan *plan)
{
    const int i = threadIdx.x;
    if (i < 33) plan->count[i] = 0;
    if (i == 0) plan->bad = 0;
}

/* size histogram, privatised in LDS */
__global__ void __launch_bounds__(256) k_ragged_hist(RaggedArgs a)
{
    __shared__ int h[34];
    if (threadIdx.x < 34) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < a.batch) {
        const int n = a.n[s];
        atomicAdd(&h[(n >= 1 && n <= 32) ? n : 0], 1);
    }
    __syncthreads();
    if (threadIdx.x >= 1 && threadIdx.x <= 32 && h[threadIdx.x] != 0)
        atomicAdd(&a.plan->count[threadIdx.x], h[threadIdx.x]);
    if (threadIdx.x == 0 && h[0] != 0) atomicAdd(&a.plan->bad, h[0]);
}

/* bins in descending size, work items per bin */
__global__ void k_ragged_plan(RaggedPlan *plan)
{
    if (threadIdx.x != 0) return;
    int start = 0, items = 0;
    for (int n = 32; n >= 1; --n) {
        plan->bin_start[n] = start;
        plan->item_start[n] = items;
        plan->cursor[n] = 0;
        const int c = plan->count[n];
        start += c;
        items += (c + ragged_per_item(n) - 1) / ragged_per_item(n);
        if (n == kRaggedSmallMax + 1) plan->large_items = items;
    }
    plan->total_items = items;
    plan->next_item = 0;
    plan->next_small = plan->large_items;
}

/* scatter system indices into their bins: each workgroup reserves one range
 * per size with a single global atomic */
__global__ void __launch_bounds__(256) k_ragged_scatter(RaggedArgs a)
{
    __shared__ int cnt[33], base[33], fill[33];
    if (threadIdx.x < 33) {
        cnt[threadIdx.x] = 0;
        fill[threadIdx.x] = 0;
    }
    __syncthreads();
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int n = 0;
    if (s < a.batch) {
        n = a.n[s];
        if (n < 1 || n > 32) {
            a.info[s] = -1;
            n = 0;
        } else {
            atomicAdd(&cnt[n], 1);
        }
    }
    __syncthreads();
    if (threadIdx.x >= 1 && threadIdx.x <= 32)
        base[threadIdx.x] =
            cnt[threadIdx.x] ? atomicAdd(&a.plan->cursor[threadIdx.x], cnt[threadIdx.x]) : 0;
    __syncthreads();
    if (n != 0) {
        const int p = atomicAdd(&fill[n], 1);
        a.sorted[a.plan->bin_start[n] + base[n] + p] = (int32_t)s;
    }
}

template <int N>
__device__ __forceinline__ bool ragged_try(const RaggedArgs &a, int n, int it)
{
    if (n != N) return false;
    ragged_run_item<N>(a, it);
    return true;
}

template <int LO, int... Ns>
__device__ __forceinline__ void ragged_dispatch(const RaggedArgs &a, int n, int it,
                                                std::integer_sequence<int, Ns...>)
{
    (void)(ragged_try<LO + Ns>(a, n, it) || ...);
}

/* Persistent loop over the work items [first, end) of sizes LO..HI:
 * workgroups take items (largest sizes first) from the atomic `counter`
 * until every item is taken; every wave leaves the loop on the same
 * broadcast item index. */
template <int LO, int HI>
__device__ __forceinline__ void ragged_persistent_loop(const RaggedArgs &a, int32_t *counter, int end)
{
    __shared__ int sh_item;
    const RaggedPlan *plan = a.plan;
    for (;;) {
        if (threadIdx.x == 0) sh_item = atomicAdd(counter, 1);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(sh_item);
        __syncthreads();
        if (it >= end) break;
        int n = LO;
        for (int m = LO; m <= HI; ++m) {
            const int c = plan->count[m];
            const int nitems = (c + ragged_per_item(m) - 1) / ragged_per_item(m);
            const int st = plan->item_start[m];
            if (it >= st && it < st + nitems) n = m;
        }
        n = __builtin_amdgcn_readfirstlane(n);
        ragged_dispatch<LO>(a, n, it, std::make_integer_sequence<int, HI - LO + 1>{});
    }
}

/* Sizes 17..32 (items 0 .. large_items-1): 16-lane segments need up to ~200
 * VGPRs, so this kernel runs 2 waves per SIMD. */
__global__ void __launch_bounds__(kRaggedThreads) __attribute__((amdgpu_waves_per_eu(2)))
    k_ragged_large(RaggedArgs a)
{
    ragged_persistent_loop<kRaggedSmallMax + 1, 32>(a, &a.plan->next_item, a.plan->large_items);
}

/* Sizes 1..16 (items large_items .. total_items-1), held to 4 waves per SIMD
 * (the register budget of its largest size). */
__global__ void __launch_bounds__(kRaggedThreads) __attribute__((amdgpu_waves_per_eu(4)))
    k_ragged_small(RaggedArgs a)
{
    ragged_persistent_loop<1, kRaggedSmallMax>(a, &a.plan->next_small, a.plan->total_items);
}

hipError_t ragged_one_launch(int n, const RaggedArgs &a, int items, hipStream_t st);

struct RaggedWs {
    RaggedPlan *plan = nullptr;
    int32_t *sorted = nullptr;
    int64_t cap = 0;
};

RaggedWs *ragged_ws_create() { return new RaggedWs; }

void ragged_ws_destroy(RaggedWs *ws)
{
    if (ws == nullptr) return;
    hipFree(ws->sorted);
    hipFree(ws->plan);
    delete ws;
}

int ragged_launch_impl(RaggedWs *ws, int64_t batch, const int32_t *n, const int64_t *offA,
                       const int64_t *offB, double *A, double *b, int32_t *ipiv, int32_t *info,
                       bool factors, bool per_size, hipStream_t st)
{
    if (batch > 0x7fffffff) return LUPP_E_UNSUPPORTED;
    if (ws->cap < batch) {
        if (ws->sorted) {
            hipError_t e = hipStreamSynchronize(st);
            if (e != hipSuccess) return hip_err(e);
            hipFree(ws->sorted);
            ws->sorted = nullptr;
            ws->cap = 0;
        }
        const int64_t cap = batch < 65536 ? 65536 : batch;
        hipError_t e = hipMalloc(&ws->sorted, (size_t)cap * sizeof(int32_t));
        if (e != hipSuccess) return e == hipErrorOutOfMemory ? LUPP_E_NOMEM : hip_err(e);
        ws->cap = cap;
    }
    if (ws->plan == nullptr) {
        hipError_t e = hipMalloc(&ws->plan, sizeof(RaggedPlan));
        if (e != hipSuccess) return hip_err(e);
    }
    RaggedArgs a{batch, n, offA, offB, A, b, ipiv, info, factors ? 1 : 0, ws->sorted, ws->plan};
    const unsigned blocks = (unsigned)((batch + 255) / 256);
    hipLaunchKernelGGL(k_ragged_zero, dim3(1), dim3(64), 0, st, ws->plan);
    hipLaunchKernelGGL(k_ragged_hist, dim3(blocks), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_ragged_plan, dim3(1), dim3(64), 0, st, ws->plan);
    hipLaunchKernelGGL(k_ragged_scatter, dim3(blocks), dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_err(e);
    if (!per_size) {
        int dev = 0, cus = 256;
        hipGetDevice(&dev);
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        /* as many workgroups as stay resident: a CU holds 4 SIMDs x (waves per
         * SIMD) waves, 4 waves per workgroup */
        hipLaunchKernelGGL(k_ragged_large, dim3((unsigned)(cus * 2)), dim3(kRaggedThreads), 0, st, a);
        hipLaunchKernelGGL(k_ragged_small, dim3((unsigned)(cus * 4)), dim3(kRaggedThreads), 0, st, a);
        return hip_err(hipGetLastError());
    }
    /* one launch per size: the host reads the plan (a synchronisation) */
    RaggedPlan h;
    e = hipMemcpyAsync(&h, ws->plan, sizeof(h), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_err(e);
    for (int m = 32; m >= 1; --m) {
        const int items = (h.count[m] + ragged_per_item(m) - 1) / ragged_per_item(m);
        e = ragged_one_launch(m, a, items, st);
        if (e != hipSuccess) return hip_err(e);
    }
    return 0;
}

}  // namespace lupp
