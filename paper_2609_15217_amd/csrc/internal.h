/* Internal declarations shared by the library's translation units. */
#ifndef LUPP_INTERNAL_H
#define LUPP_INTERNAL_H

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lupp.h"

namespace lupp {

/* Arguments of one batched-solve launch (layout-generic). */
struct SolveArgs {
    int64_t batch;
    double *A;
    int64_t lda;
    int64_t sA;  /* AoS: system stride; SoA: ldbatch */
    double *b;
    int64_t sB;  /* AoS: system stride; SoA: component stride */
    int32_t *ipiv;
    int32_t *info;
    int tile;      /* pivoting rule: 0 textbook, >= 1 tile-local with this tile */
    double thresh; /* tile-local acceptance threshold */
    int fma;       /* 1: fused multiply-add arithmetic (LUPP_FMA), 0: strict */
};

/* Enqueue one batched-solve kernel: layout LUPP_AOS/LUPP_SOA, factors =
 * write L\U back, wpb = wave64s per workgroup (0: default). */
typedef hipError_t (*LaunchFn)(const SolveArgs &, int layout, bool factors, int wpb,
                               hipStream_t);

/* Kernel lookup (registry.cpp): nullptr if the variant is not compiled. */
LaunchFn thread_launcher(int n);
LaunchFn lanes_launcher(int n, int lanes);
const void *thread_kernel_symbol(int n);
const void *lanes_kernel_symbol(int n, int lanes, int layout);
/* Segment widths compiled for size n (ascending), returns the count. */
int lanes_widths(int n, int *out, int cap);
/* Batches below this size use the small-batch dispatch entries. */
constexpr int64_t kSmallBatch = 32768;
/* Autotuned default for (n, layout, batch bucket), compiled in by the build;
 * false if the table has no entry. */
bool tuned_choice(int n, int layout, int bucket, int *variant, int *lanes, int *wpb);
constexpr int kThreadMaxN = 13;

/* CPU-driven batched Newton (batched_newton.hip): workspace owned by a
 * context, and the host-driven iteration loop. */
struct BnWs;
BnWs *bn_ws_create();
void bn_ws_destroy(BnWs *ws);
int constitutive_batched_run(lupp_ctx *ctx, BnWs *ws, const lupp_points *pts, const lupp_law *law,
                             double tol, int maxit, bool graph, hipStream_t st, int *iterations);

/* Constitutive update launcher (constitutive.hip). */
/* lanes: 1 = one lane per point, else lanes per point (see
 * newton_lanes_supported); tangent requests always use one lane per point. */
int constitutive_launch(const lupp_points *pts, const lupp_law *law, double tol, int maxit,
                        int lanes, hipStream_t stream);
bool newton_lanes_supported(int kind, int lanes);
/* Measured default mapping of the fused update per law kind (gfx950). */
int newton_default_lanes(int kind);
const void *constitutive_kernel_symbol(int kind, bool tangent);

/* Ragged batch (ragged.hip): device workspace owned by a context. */
struct RaggedWs;
struct RaggedPlan;
/* Enqueue the grouping kernels and the solve of a ragged batch on st, with
 * the caller's workspace: plan (one RaggedPlan) and sorted (batch int32
 * system indices). Allocates nothing. */
int ragged_enqueue(RaggedPlan *plan, int32_t *sorted, const uint8_t *lanes, int64_t batch,
                   const int32_t *n, const int64_t *offA, const int64_t *offB, double *A, double *b,
                   int32_t *ipiv, int32_t *info, bool factors, bool per_size, hipStream_t st);
RaggedWs *ragged_ws_create();
void ragged_ws_destroy(RaggedWs *ws);
/* lanes[n] (n = 1..32): lanes per system used for size n (ragged_lanes_ok). */
int ragged_launch_impl(RaggedWs *ws, const uint8_t *lanes, int64_t batch, const int32_t *n,
                       const int64_t *offA, const int64_t *offB, double *A, double *b,
                       int32_t *ipiv, int32_t *info, bool factors, bool per_size,
                       hipStream_t stream);
/* Time the ragged path (class launches) on a batch of `batch` systems of size n
 * (AoS, packed) for every lane count compiled for n; lanes[n] is left at the
 * fastest (median of reps timed runs after one warm-up). */
int ragged_autotune_impl(RaggedWs *ws, uint8_t *lanes, int n, int64_t batch, const double *A,
                         const double *b, int reps, int *best, float *best_ms, hipStream_t st);
/* Grouped batches (grouped.hip): enqueue the launches of validated groups. */
int grouped_enqueue(const lupp_group *groups, int ngroups, const uint8_t *lanes, bool factors,
                    hipStream_t st);
/* Allocation-free ragged path (ragged_noalloc.hip): resolve the device
 * address of the fixed workspace on `device` (once per device; lupp_create
 * calls it), and enqueue a ragged solve that uses it. */
int noalloc_scratch_init(int device);
int noalloc_ragged_enqueue(int device, const uint8_t *lanes, int64_t batch, const int32_t *n,
                           const int64_t *offA, const int64_t *offB, double *A, double *b,
                           int32_t *ipiv, int32_t *info, bool factors, hipStream_t st);
/* Measured default lanes per size for the ragged path (compiled in from
 * the autotuner's table); false if the table has no entry for n. */
bool tuned_ragged(int n, int *lanes);

/* Sizes above this one run in the ragged kernels of 16-lane segments. */
constexpr int kRaggedSmallMax = 16;

/* Lane counts compiled into the ragged kernels for size n. Sizes up to 16
 * share one kernel held to 3 waves per SIMD: the thread path up to n = 5 and
 * segments of 2, 4, 8 or 16 lanes where the rows fit; sizes 17..32 run in two
 * kernels (17..23 at 3 waves per SIMD, 24..32 at 2) with 16 lanes, two rows
 * each (one row on each of 32 lanes measured slower at every one of these
 * sizes, standalone and in the ragged kernel, so it is not compiled in: it
 * would double the kernels' code). */
__host__ __device__ constexpr bool ragged_lanes_ok(int n, int T)
{
    if (n < 1 || n > 32) return false;
    if (n > kRaggedSmallMax) return T == 16;
    return (T == 1 && n <= 5) || (T == 2 && n >= 2 && n <= 4) || (T == 4 && n >= 3 && n <= 8) ||
           (T == 8 && n >= 5) || (T == 16 && n >= 9);
}

/* Lanes per size before any measurement: the thread path while the system
 * is tiny, 8-lane segments up to 16, 16-lane segments above. */
__host__ __device__ constexpr int ragged_default_lanes(int n)
{
    return n <= 5 ? 1 : (n <= kRaggedSmallMax ? 8 : 16);
}

/* ------------------------------------------------------------------------ */
/* Device-side memory access through buffer resources.                      */
/*                                                                          */
/* A buffer resource is a 128-bit descriptor (base, size) held in SGPRs; a   */
/* load or store adds a 32-bit per-lane byte offset (VGPR) and a 32-bit      */
/* uniform offset (SGPR). Per-element addresses therefore cost no VGPRs, and */
/* an access at or beyond `bytes` reads 0 / writes nothing, which retires    */
/* the lanes past the end of a batch without branches.                      */
/* ------------------------------------------------------------------------ */
typedef int lupp_v2i __attribute__((ext_vector_type(2)));

/* word 3 of a raw (untyped) buffer descriptor on gfx9-family GPUs: 32-bit
 * data format, no swizzle */
constexpr int kBufferWord3 = 0x00020000;

/* A per-lane byte offset that is out of range for every descriptor the
 * library builds (their extents stay below 2^31 bytes): loads return zero and
 * stores are dropped. */
constexpr uint32_t kOutOfRange = 0x80000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                             kBufferWord3);
}

__device__ __forceinline__ double buf_load_f64(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                               uint32_t soff)
{
    lupp_v2i v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0);
    return __builtin_bit_cast(double, v);
}

__device__ __forceinline__ void buf_store_f64(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                              uint32_t soff, double x)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(lupp_v2i, x), r, (int)voff,
                                          (int)soff, 0);
}

__device__ __forceinline__ void buf_store_i32(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                              uint32_t soff, int x)
{
    __builtin_amdgcn_raw_buffer_store_b32(x, r, (int)voff, (int)soff, 0);
}

/* Workgroups are dispatched to the 8 XCDs round robin (workgroup b runs on
 * XCD b % 8), and each XCD has its own L2. Remapping so that every XCD
 * processes one contiguous range of logical workgroups keeps neighbouring
 * systems - which share cache lines in the interleaved layout - in the same
 * L2. The map is a bijection on [0, G). */
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t G)
{
    constexpr uint32_t X = 8;
    const uint32_t q = G / X, r = G % X, x = b % X, i = b / X;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}

/* Returns p unchanged, but hides its value from the optimiser. Buffer
 * descriptors built from the result cannot be merged with descriptors built
 * earlier from p, so the earlier ones die instead of being kept alive (in
 * spilled SGPRs) across the whole solve. */
template <typename T>
__device__ __forceinline__ T *opaque_ptr(T *p)
{
    const uint64_t v = (uint64_t)p;
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    asm volatile("" : "+s"(lo), "+s"(hi));
    return (T *)(((uint64_t)hi << 32) | lo);
}

/* The same for a uniform 64-bit integer (strides and offsets). */
__device__ __forceinline__ int64_t opaque_i64(int64_t v)
{
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    asm volatile("" : "+s"(lo), "+s"(hi));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

inline int hip_err(hipError_t e) { return e == hipSuccess ? 0 : LUPP_E_HIP_BASE - (int)e; }

}  // namespace lupp

#endif
