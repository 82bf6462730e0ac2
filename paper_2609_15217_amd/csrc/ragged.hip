/* Ragged (mixed-size) batches: device-side grouping by size and one launch
 * per size class (see kernels_ragged.h). */
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

/* Grouping by size. Workgroup g owns the contiguous chunk of systems
 * [g*chunk, (g+1)*chunk), chunk a multiple of 256: a few hundred workgroups,
 * so the per-size global atomics (one per workgroup and size) stay few. */
__device__ __forceinline__ void ragged_chunk(const RaggedArgs &a, int64_t &c0, int64_t &c1)
{
    const int64_t chunk = ((a.batch + gridDim.x - 1) / gridDim.x + 255) / 256 * 256;
    c0 = (int64_t)blockIdx.x * chunk;
    c1 = c0 + chunk < a.batch ? c0 + chunk : a.batch;
}

/* size histogram, privatised in LDS */
__global__ void __launch_bounds__(256) k_ragged_hist(RaggedArgs a)
{
    __shared__ int h[34];
    if (threadIdx.x < 34) h[threadIdx.x] = 0;
    __syncthreads();
    int64_t c0, c1;
    ragged_chunk(a, c0, c1);
    for (int64_t s = c0 + threadIdx.x; s < c1; s += blockDim.x) {
        const int n = a.n[s];
        atomicAdd(&h[(n >= 1 && n <= 32) ? n : 0], 1);
    }
    __syncthreads();
    if (threadIdx.x >= 1 && threadIdx.x <= 32 && h[threadIdx.x] != 0)
        atomicAdd(&a.plan->count[threadIdx.x], h[threadIdx.x]);
    if (threadIdx.x == 0 && h[0] != 0) atomicAdd(&a.plan->bad, h[0]);
}

/* bins in descending size, work items per bin (their size follows the lane
 * count of the size), class boundaries */
__global__ void k_ragged_plan(RaggedArgs a)
{
    if (threadIdx.x != 0) return;
    RaggedPlan *plan = a.plan;
    int start = 0, items = 0;
    for (int n = 32; n >= 1; --n) {
        if (n == ragged_class_hi(ragged_class_of(n))) plan->class_start[ragged_class_of(n)] = items;
        plan->bin_start[n] = start;
        plan->item_start[n] = items;
        plan->cursor[n] = 0;
        const int c = plan->count[n];
        const int per = ragged_per_item(a.lanes[n]);
        start += c;
        items += (c + per - 1) / per;
    }
    plan->class_start[kRaggedClasses] = items;
}

/* scatter system indices into their bins: each workgroup counts its chunk,
 * reserves one range per size with a single global atomic, then places its
 * systems (the order inside a bin does not matter: systems are independent) */
__global__ void __launch_bounds__(256) k_ragged_scatter(RaggedArgs a)
{
    __shared__ int cnt[33], base[33], fill[33];
    if (threadIdx.x < 33) {
        cnt[threadIdx.x] = 0;
        fill[threadIdx.x] = 0;
    }
    __syncthreads();
    int64_t c0, c1;
    ragged_chunk(a, c0, c1);
    for (int64_t s = c0 + threadIdx.x; s < c1; s += blockDim.x) {
        const int n = a.n[s];
        if (n >= 1 && n <= 32) atomicAdd(&cnt[n], 1);
        else a.info[s] = -1;
    }
    __syncthreads();
    if (threadIdx.x >= 1 && threadIdx.x <= 32)
        base[threadIdx.x] =
            cnt[threadIdx.x] ? atomicAdd(&a.plan->cursor[threadIdx.x], cnt[threadIdx.x]) : 0;
    __syncthreads();
    for (int64_t s = c0 + threadIdx.x; s < c1; s += blockDim.x) {
        const int n = a.n[s];
        if (n >= 1 && n <= 32) {
            const int p = atomicAdd(&fill[n], 1);
            a.sorted[a.plan->bin_start[n] + base[n] + p] = (int32_t)s;
        }
    }
}

hipError_t ragged_one_launch(int n, const RaggedArgs &a, int items, hipStream_t st);

/* Workspace of the allocating entry point. Calls on one context may come on
 * different streams: `done` is recorded after each call's last kernel, and
 * the next call on another stream waits for it before its grouping kernels
 * reset the plan and rewrite `sorted` (which the earlier call's solve
 * kernels may still be reading). */
struct RaggedWs {
    RaggedPlan *plan = nullptr;
    int32_t *sorted = nullptr;
    int64_t cap = 0;
    hipEvent_t done = nullptr;
    hipStream_t last = nullptr;
    bool used = false;
};

RaggedWs *ragged_ws_create() { return new RaggedWs; }

void ragged_ws_destroy(RaggedWs *ws)
{
    if (ws == nullptr) return;
    if (ws->done) {
        hipEventSynchronize(ws->done);
        hipEventDestroy(ws->done);
    }
    hipFree(ws->sorted);
    hipFree(ws->plan);
    delete ws;
}

int ragged_enqueue(RaggedPlan *plan, int32_t *sorted, const uint8_t *lanes, int64_t batch,
                   const int32_t *n, const int64_t *offA, const int64_t *offB, double *A, double *b,
                   int32_t *ipiv, int32_t *info, bool factors, bool per_size, hipStream_t st)
{
    RaggedArgs a{batch, n, offA, offB, A, b, ipiv, info, factors ? 1 : 0, sorted, plan, {}};
    for (int m = 0; m <= 32; ++m) a.lanes[m] = m >= 1 ? lanes[m] : 1;
    /* grouping grid: at most 1024 workgroups of 256 threads, each a chunk */
    const int64_t full = (batch + 255) / 256;
    const unsigned blocks = (unsigned)(full < 1024 ? full : 1024);
    hipLaunchKernelGGL(k_ragged_zero, dim3(1), dim3(64), 0, st, plan);
    hipLaunchKernelGGL(k_ragged_hist, dim3(blocks), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_ragged_plan, dim3(1), dim3(64), 0, st, a);
    hipLaunchKernelGGL(k_ragged_scatter, dim3(blocks), dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_err(e);
    if (!per_size) {
        int dev = 0, cus = 256;
        hipGetDevice(&dev);
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        /* each class kernel with as many workgroups as stay resident: a CU
         * holds 4 SIMDs x (waves per SIMD) waves, 4 waves per workgroup */
        e = ragged_c0_launch(a, (unsigned)(cus * ragged_class_waves(0)), st);
        if (e == hipSuccess) e = ragged_c1_launch(a, (unsigned)(cus * ragged_class_waves(1)), st);
        if (e == hipSuccess) e = ragged_c2_launch(a, (unsigned)(cus * ragged_class_waves(2)), st);
        return hip_err(e);
    }
    /* one launch per size: the host reads the plan (a synchronisation) */
    RaggedPlan h;
    e = hipMemcpyAsync(&h, plan, sizeof(h), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_err(e);
    for (int m = 32; m >= 1; --m) {
        const int per = ragged_per_item(a.lanes[m]);
        const int items = (h.count[m] + per - 1) / per;
        e = ragged_one_launch(m, a, items, st);
        if (e != hipSuccess) return hip_err(e);
    }
    return 0;
}

int ragged_launch_impl(RaggedWs *ws, const uint8_t *lanes, int64_t batch, const int32_t *n,
                       const int64_t *offA, const int64_t *offB, double *A, double *b,
                       int32_t *ipiv, int32_t *info, bool factors, bool per_size, hipStream_t st)
{
    if (batch > 0x7fffffff) return LUPP_E_UNSUPPORTED;
    hipError_t e = hipSuccess;
    if (ws->done == nullptr) {
        e = hipEventCreateWithFlags(&ws->done, hipEventDisableTiming);
        if (e != hipSuccess) return hip_err(e);
    }
    if (ws->cap < batch) {
        if (ws->sorted) {
            /* the previous call, on whatever stream, must be done with it */
            e = hipEventSynchronize(ws->done);
            if (e != hipSuccess) return hip_err(e);
            hipFree(ws->sorted);
            ws->sorted = nullptr;
            ws->cap = 0;
        }
        const int64_t cap = batch < 65536 ? 65536 : batch;
        e = hipMalloc(&ws->sorted, (size_t)cap * sizeof(int32_t));
        if (e != hipSuccess) return e == hipErrorOutOfMemory ? LUPP_E_NOMEM : hip_err(e);
        ws->cap = cap;
    }
    if (ws->plan == nullptr) {
        e = hipMalloc(&ws->plan, sizeof(RaggedPlan));
        if (e != hipSuccess) return hip_err(e);
    }
    /* a call being captured into a graph is ordered by the graph, not by
     * the eager event chain */
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    e = hipStreamIsCapturing(st, &cs);
    if (e != hipSuccess) return hip_err(e);
    const bool capturing = cs != hipStreamCaptureStatusNone;
    if (!capturing && ws->used && ws->last != st) {
        e = hipStreamWaitEvent(st, ws->done, 0);
        if (e != hipSuccess) return hip_err(e);
    }
    const int rc = ragged_enqueue(ws->plan, ws->sorted, lanes, batch, n, offA, offB, A, b, ipiv,
                                  info, factors, per_size, st);
    if (capturing) return rc;
    e = hipEventRecord(ws->done, st);
    ws->last = st;
    ws->used = true;
    return rc != 0 ? rc : hip_err(e);
}

/* offsets of a packed single-size batch: system s at s*n*n (matrix) and s*n
 * (right-hand side, pivots) */
__global__ void __launch_bounds__(256) k_ragged_uniform(int64_t batch, int n, int32_t *nv,
                                                        int64_t *offA, int64_t *offB)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= batch) return;
    nv[s] = n;
    offA[s] = s * n * n;
    offB[s] = s * n;
}

int ragged_autotune_impl(RaggedWs *ws, uint8_t *lanes, int n, int64_t batch, const double *A,
                         const double *b, int reps, int *best, float *best_ms, hipStream_t st)
{
    const size_t nA = (size_t)batch * n * n, nB = (size_t)batch * n;
    double *wA = nullptr, *wB = nullptr;
    int32_t *wN = nullptr, *wP = nullptr, *wI = nullptr;
    int64_t *oA = nullptr, *oB = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = 0;
    hipError_t e = hipMalloc(&wA, nA * 8);
    if (e == hipSuccess) e = hipMalloc(&wB, nB * 8);
    if (e == hipSuccess) e = hipMalloc(&wN, (size_t)batch * 4);
    if (e == hipSuccess) e = hipMalloc(&wP, nB * 4);
    if (e == hipSuccess) e = hipMalloc(&wI, (size_t)batch * 4);
    if (e == hipSuccess) e = hipMalloc(&oA, (size_t)batch * 8);
    if (e == hipSuccess) e = hipMalloc(&oB, (size_t)batch * 8);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) rc = e == hipErrorOutOfMemory ? LUPP_E_NOMEM : hip_err(e);
    if (rc == 0) {
        hipLaunchKernelGGL(k_ragged_uniform, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, st,
                           batch, n, wN, oA, oB);
        e = hipGetLastError();
        if (e != hipSuccess) rc = hip_err(e);
    }
    const uint8_t keep = lanes[n];
    int pick = 0;
    float pick_ms = 3.0e38f;
    const int cands[6] = {1, 2, 4, 8, 16, 32};
    for (int c = 0; c < 6 && rc == 0; ++c) {
        if (!ragged_lanes_ok(n, cands[c])) continue;
        lanes[n] = (uint8_t)cands[c];
        float t[64];
        const int r_total = reps + 1 < 64 ? reps + 1 : 64;
        for (int r = 0; r < r_total && rc == 0; ++r) {
            e = hipMemcpyAsync(wA, A, nA * 8, hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess) e = hipMemcpyAsync(wB, b, nB * 8, hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess) e = hipEventRecord(e0, st);
            if (e != hipSuccess) { rc = hip_err(e); break; }
            rc = ragged_launch_impl(ws, lanes, batch, wN, oA, oB, wA, wB, wP, wI, true, false, st);
            if (rc != 0) break;
            e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(&t[r], e0, e1);
            if (e != hipSuccess) rc = hip_err(e);
        }
        if (rc != 0) break;
        /* median of the timed repetitions (the first run is a warm-up) */
        for (int i = 1; i < r_total; ++i)
            for (int j = i + 1; j < r_total; ++j)
                if (t[j] < t[i]) { const float x = t[i]; t[i] = t[j]; t[j] = x; }
        const float med = t[1 + (r_total - 1) / 2];
        if (med < pick_ms) { pick_ms = med; pick = cands[c]; }
    }
    lanes[n] = (rc == 0 && pick != 0) ? (uint8_t)pick : keep;
    if (rc == 0) {
        if (best) *best = pick;
        if (best_ms) *best_ms = pick_ms;
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    hipFree(wA);
    hipFree(wB);
    hipFree(wN);
    hipFree(wP);
    hipFree(wI);
    hipFree(oA);
    hipFree(oB);
    return rc;
}

}  // namespace lupp
