/* Workspace of the allocation-free ragged solve (lupp_batched_solve_ragged_noalloc):
 * a file-scope device array holding the size plan and the sorted system
 * indices of one call, LUPP_NOALLOC_MAX_BATCH systems at most. Each GPU the
 * library runs on holds its own copy until the process ends.
 *
 * Host code never passes `scratch` itself to a kernel or a copy: on the host
 * the name is only a stand-in for the symbol. noalloc_scratch_init resolves
 * the array's device address once per device (with that device current) and
 * keeps it; every later use goes through that address.
 */
#include <mutex>

#include "kernels_ragged.h"

namespace lupp {

constexpr size_t kNoAllocPlanBytes = (sizeof(RaggedPlan) + 255) / 256 * 256;
constexpr size_t kNoAllocBytes = kNoAllocPlanBytes + (size_t)LUPP_NOALLOC_MAX_BATCH * sizeof(int32_t);

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];
int g_scratch_state[kMaxDevices]; /* 0: not resolved, 1: resolved, < 0: the error */
}  // namespace

int noalloc_scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return LUPP_E_UNSUPPORTED;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (g_scratch_state[device] != 0) return g_scratch_state[device] > 0 ? 0 : g_scratch_state[device];
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != device) e = hipSetDevice(device);
    void *p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) hipSetDevice(cur);
    if (e != hipSuccess || p == nullptr) {
        g_scratch_state[device] = e != hipSuccess ? hip_err(e) : LUPP_E_UNSUPPORTED;
        return g_scratch_state[device];
    }
    g_scratch_ptr[device] = p;
    g_scratch_state[device] = 1;
    return 0;
}

int noalloc_ragged_enqueue(int device, const uint8_t *lanes, int64_t batch, const int32_t *n,
                           const int64_t *offA, const int64_t *offB, double *A, double *b,
                           int32_t *ipiv, int32_t *info, bool factors, hipStream_t st)
{
    if (batch > LUPP_NOALLOC_MAX_BATCH) return LUPP_E_TOO_LARGE;
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> g(g_scratch_mu);
        if (device < 0 || device >= kMaxDevices) return LUPP_E_UNSUPPORTED;
        if (g_scratch_state[device] < 0) return g_scratch_state[device];
        if (g_scratch_state[device] == 0) return LUPP_E_UNSUPPORTED;
        base = g_scratch_ptr[device];
    }
    RaggedPlan *plan = static_cast<RaggedPlan *>(base);
    int32_t *sorted = reinterpret_cast<int32_t *>(static_cast<unsigned char *>(base) + kNoAllocPlanBytes);
    /* the zero kernel clears the plan's counters: the array keeps the last
     * call's contents */
    return ragged_enqueue(plan, sorted, lanes, batch, n, offA, offB, A, b, ipiv, info, factors,
                          false, st);
}

}  // namespace lupp
