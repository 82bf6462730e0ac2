/* Mixed-size (ragged) batches (Section 4.1: a size-aware dispatcher picks the
 * specialised solver for each problem size).
 *
 * Systems are grouped by size on the device: a histogram, a plan that lays
 * the size bins out in descending n (costliest work first) and cuts each bin
 * into work items of one workgroup round, and a scatter of system indices
 * into the bins. The solve is then one launch per size class - classes of
 * sizes with the same register budget, so that each class runs at the
 * occupancy its largest size allows - whose workgroups walk the class's work
 * items with a grid stride (no work counter: the plan gives every workgroup
 * its items), or one launch per size.
 *
 * System s: matrix column-major at A + offA[s] (lda = n[s]), right-hand side
 * and pivots at offset offB[s], info[s].
 */
#ifndef LUPP_KERNELS_RAGGED_H
#define LUPP_KERNELS_RAGGED_H

#include <utility>

#include "internal.h"
#include "lupp_device.h"

namespace lupp {

constexpr int kRaggedWaves = 4;       /* wave64s per workgroup */
constexpr int kRaggedThreads = 64 * kRaggedWaves;

/* Size classes of the ragged and grouped kernels, largest sizes first:
 * 24..32 (16-lane segments, up to 217 VGPRs: 2 waves per SIMD), 17..23
 * (16-lane segments, 164 VGPRs: 3 waves; with n = 24 in it the class kernel
 * spilled) and 1..16. */
constexpr int kRaggedClasses = 3;
__host__ __device__ constexpr int ragged_class_lo(int c) { return c == 0 ? 24 : (c == 1 ? 17 : 1); }
__host__ __device__ constexpr int ragged_class_hi(int c) { return c == 0 ? 32 : (c == 1 ? 23 : 16); }
__host__ __device__ constexpr int ragged_class_of(int n) { return n >= 24 ? 0 : (n >= 17 ? 1 : 2); }

struct RaggedPlan {
    int32_t count[33];      /* systems of each size */
    int32_t bin_start[33];  /* first index of each size in `sorted` */
    int32_t cursor[33];     /* scatter cursors */
    int32_t item_start[33]; /* first work item of each size */
    /* work items of class c: class_start[c] .. class_start[c + 1] - 1 */
    int32_t class_start[kRaggedClasses + 1];
    int32_t bad;            /* systems with n outside 1..32 */
};

struct RaggedArgs {
    int64_t batch;
    const int32_t *n;
    const int64_t *offA, *offB;
    double *A, *b;
    int32_t *ipiv, *info;
    int factors;
    int32_t *sorted;
    RaggedPlan *plan;
    /* lanes per system for each size (ragged_lanes_ok). Words, not bytes:
     * 4-byte-aligned kernel arguments are read by scalar loads, where a byte
     * array is loaded into vector registers (and, in the looping
     * kernels, spilled to scratch memory) */
    int32_t lanes[33];
};

/* systems one workgroup solves at once with T lanes per system: one work
 * item (measured: four rounds per item ran 2-11% slower than one, the
 * workgroup's next loads then waiting for its previous solve) */
__host__ __device__ constexpr int ragged_per_round(int T)
{
    return T == 1 ? kRaggedThreads : kRaggedWaves * (64 / T);
}

__host__ __device__ constexpr int ragged_per_item(int T) { return ragged_per_round(T); }

/* Where the j-th system of a work item lives: matrix (column-major, leading
 * dimension lda()), right-hand side, pivots and info. */
struct SysPtrs {
    double *A, *b;
    int32_t *ipiv, *info;
};

/* Ragged batches: the item's systems are entries of the sorted index list,
 * each at its own offsets, packed (lda = n). */
template <int N>
struct RaggedLoc {
    const RaggedArgs &a;
    const int32_t *idx;
    __device__ __forceinline__ SysPtrs sys(int j) const
    {
        const int64_t s = idx[j];
        return {a.A + a.offA[s], a.b + a.offB[s], a.ipiv + a.offB[s], a.info + s};
    }
    __device__ __forceinline__ int64_t lda() const { return N; }
};

/* Solve the cnt (>= 1) systems of one work item with the whole workgroup, T
 * lanes per system (T == 1: one thread per system). Threads or segments
 * without a system point at system 0, load zeros and store nothing. */
template <int N, int T, typename Loc>
__device__ __forceinline__ void solve_item(const Loc &loc, int cnt, int factors)
{
    const int64_t lda = loc.lda();
    if constexpr (T == 1) {
        const int i = threadIdx.x;
        const bool act = i < cnt;
        const SysPtrs p = loc.sys(act ? i : 0); /* cnt >= 1: system 0 exists */
        double m[N][N], x[N];
        int piv[N];
        static_for<0, N>([&](auto jc) __attribute__((always_inline)) {
            constexpr int j = decltype(jc)::value;
            static_for<0, N>([&](auto ic) __attribute__((always_inline)) {
                constexpr int ii = decltype(ic)::value;
                m[j][ii] = act ? p.A[ii + j * lda] : 0.0;
            });
            x[j] = act ? p.b[j] : 0.0;
        });
        const int inf = thread_getrf_solve<N, true>(m, x, piv);
        if (act) {
            if (factors) {
                static_for<0, N>([&](auto jc) __attribute__((always_inline)) {
                    constexpr int j = decltype(jc)::value;
                    static_for<0, N>([&](auto ic) __attribute__((always_inline)) {
                        constexpr int ii = decltype(ic)::value;
                        p.A[ii + j * lda] = m[j][ii];
                    });
                });
            }
            static_for<0, N>([&](auto kc) __attribute__((always_inline)) {
                constexpr int k = decltype(kc)::value;
                p.ipiv[k] = piv[k];
                if (inf == 0) p.b[k] = x[k];
            });
            *p.info = inf;
        }
    } else {
        constexpr int K = lanes_shape<N, T>::K;
        constexpr int SPW = 64 / T;
        const int lane = (int)__lane_id();
        const int g = lane / T, t = lane % T;
        const int wave = threadIdx.x >> 6;
        const int j0 = wave * SPW + g;
        const bool act = j0 < cnt;
        const SysPtrs p = loc.sys(act ? j0 : 0); /* cnt >= 1: system 0 exists */
        double m[K][N], x[K];
        int pos[K];
        static_for<0, K>([&](auto sc) __attribute__((always_inline)) {
            constexpr int sl = decltype(sc)::value;
            const int r = t + sl * T;
            const bool ok = act && r < N;
            pos[sl] = r < N ? r : -1;
            static_for<0, N>([&](auto jc) __attribute__((always_inline)) {
                constexpr int j = decltype(jc)::value;
                m[sl][j] = ok ? p.A[r + j * lda] : 0.0;
            });
            x[sl] = ok ? p.b[r] : 0.0;
        });
        constexpr int KP = (N + T - 1) / T;
        int pv[KP];
        static_for<0, KP>([&](auto sc) __attribute__((always_inline)) { pv[decltype(sc)::value] = 0; });
        /* 16-column pivot-row broadcasts where 16-lane segments already need
         * more than 168 VGPRs (n >= 26), as in the SoA kernels */
        constexpr int CH = (T == 16 && N >= 26) ? 16 : 8;
        const int inf = lanes_getrf_solve<N, T, false, false, CH>(m, x, pos, g * T, [&](int k, int v) {
            const int c = k / T;
            static_for<0, KP>([&](auto sc) __attribute__((always_inline)) {
                constexpr int cc = decltype(sc)::value;
                if (cc == c) pv[cc] = (t == k % T) ? v : pv[cc];
            });
        });
        if (act) {
            static_for<0, K>([&](auto sc) __attribute__((always_inline)) {
                constexpr int sl = decltype(sc)::value;
                if (pos[sl] >= 0) {
                    if (factors) {
                        static_for<0, N>([&](auto jc) __attribute__((always_inline)) {
                            constexpr int j = decltype(jc)::value;
                            p.A[pos[sl] + j * lda] = m[sl][j];
                        });
                    }
                    if (inf == 0) p.b[pos[sl]] = x[sl];
                }
            });
            static_for<0, KP>([&](auto sc) __attribute__((always_inline)) {
                constexpr int c = decltype(sc)::value;
                if (t + c * T < N) p.ipiv[t + c * T] = pv[c];
            });
            if (t == 0) *p.info = inf;
        }
    }
}

template <int N, int T>
__device__ __forceinline__ void ragged_item(const RaggedArgs &a, int first, int cnt)
{
    const RaggedLoc<N> loc{a, a.sorted + a.plan->bin_start[N] + first};
    solve_item<N, T>(loc, cnt, a.factors);
}

template <int N, int T>
__device__ __forceinline__ void ragged_run_item_t(const RaggedArgs &a, int it)
{
    const int first = (it - a.plan->item_start[N]) * ragged_per_item(T);
    const int rest = a.plan->count[N] - first;
    if (rest > 0) ragged_item<N, T>(a, first, rest < ragged_per_item(T) ? rest : ragged_per_item(T));
}

template <int N, int T>
__device__ __forceinline__ bool ragged_try_lanes(const RaggedArgs &a, int lanes, int it)
{
    if constexpr (ragged_lanes_ok(N, T)) {
        if (lanes == T) {
            ragged_run_item_t<N, T>(a, it);
            return true;
        }
    }
    return false;
}

/* Solve the work item `it` of size N (all threads of the workgroup) with the
 * lane count the table gives for N (uniform across the workgroup). */
template <int N>
__device__ __forceinline__ void ragged_run_item(const RaggedArgs &a, int it)
{
    if constexpr (N > kRaggedSmallMax) {
        /* 16 lanes: the only count compiled for these sizes (ragged_lanes_ok) */
        ragged_run_item_t<N, 16>(a, it);
    } else {
        const int lanes = __builtin_amdgcn_readfirstlane((int)a.lanes[N]);
        (void)(ragged_try_lanes<N, 1>(a, lanes, it) || ragged_try_lanes<N, 2>(a, lanes, it) ||
               ragged_try_lanes<N, 4>(a, lanes, it) || ragged_try_lanes<N, 8>(a, lanes, it) ||
               ragged_try_lanes<N, 16>(a, lanes, it));
    }
}

/* One size per launch: workgroup b solves work item b of size N. */
template <int N>
__global__ void __launch_bounds__(kRaggedThreads) k_ragged_one(RaggedArgs a)
{
    const int it = a.plan->item_start[N] + (int)xcd_block(blockIdx.x, gridDim.x);
    ragged_run_item<N>(a, it);
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

/* The work items of class C (sizes LO..HI): workgroup w of a grid of G
 * takes items class_start[C] + w, + w + G, ... (w remapped so that the
 * workgroups of one XCD take neighbouring items). Items come largest size
 * first and every workgroup gets the same mix, so the grid finishes within
 * about one item of its mean. The size of an item is the smallest m whose
 * first item is at or before it (empty sizes start where the next one does). */
template <int C>
__device__ __forceinline__ void ragged_class_loop(const RaggedArgs &a)
{
    constexpr int LO = ragged_class_lo(C), HI = ragged_class_hi(C);
    const RaggedPlan *plan = a.plan;
    const int end = plan->class_start[C + 1];
    const int G = (int)gridDim.x;
    for (int it = plan->class_start[C] + (int)xcd_block(blockIdx.x, gridDim.x); it < end; it += G) {
        int n = HI;
        for (int m = HI - 1; m >= LO; --m)
            if (plan->item_start[m] <= it) n = m;
        n = __builtin_amdgcn_readfirstlane(n);
        ragged_dispatch<LO>(a, n, it, std::make_integer_sequence<int, HI - LO + 1>{});
    }
}

/* ------------------------------------------------------------------------ */
/* Grouped batches: up to kMaxGroups uniform batches, each with its own size,  */
/* pointers and strides (AoS), solved by one launch per size class. The host   */
/* knows every group's size, so no grouping kernels and no work counter are   */
/* needed: workgroup w takes work item w, and the group table (kernel          */
/* arguments, read with scalar loads) gives its group.                         */
/* ------------------------------------------------------------------------ */
constexpr int kMaxGroups = 32;

struct GroupDesc {
    double *A, *b;
    int32_t *ipiv, *info;
    int64_t lda, sA, sB, batch;
    int32_t n, lanes;
    int32_t item0;   /* first work item of the group in its launch */
    int32_t factors; /* write the factors back (else A is only read) */
};

struct GroupedArgs {
    int32_t ngroups, pad;
    GroupDesc g[kMaxGroups]; /* ascending item0 */
};

/* System s of a group: matrix at A + s*sA (leading dimension lda), right-hand
 * side at b + s*sB, pivots at ipiv + s*n, info[s]. */
template <int N>
struct GroupLoc {
    const GroupDesc &g;
    int64_t first;
    __device__ __forceinline__ SysPtrs sys(int j) const
    {
        const int64_t s = first + j;
        return {g.A + s * g.sA, g.b + s * g.sB, g.ipiv + s * N, g.info + s};
    }
    __device__ __forceinline__ int64_t lda() const { return g.lda; }
};

/* systems of one grouped work item: one round of the workgroup */
__host__ __device__ constexpr int grouped_per_item(int T) { return ragged_per_round(T); }

template <int N, int T>
__device__ __forceinline__ bool grouped_try_lanes(const GroupDesc &g, int lanes, int local,
                                                  int factors)
{
    if constexpr (ragged_lanes_ok(N, T)) {
        if (lanes == T) {
            const int64_t first = (int64_t)local * grouped_per_item(T);
            const int64_t rest = g.batch - first;
            const int cnt = (int)(rest < grouped_per_item(T) ? rest : grouped_per_item(T));
            solve_item<N, T>(GroupLoc<N>{g, first}, cnt, factors);
            return true;
        }
    }
    return false;
}

template <int N>
__device__ __forceinline__ bool grouped_try(const GroupDesc &g, int n, int local, int factors)
{
    if (n != N) return false;
    if constexpr (N > kRaggedSmallMax) {
        (void)grouped_try_lanes<N, 16>(g, 16, local, factors); /* the only count compiled */
    } else {
        const int lanes = __builtin_amdgcn_readfirstlane(g.lanes);
        (void)(grouped_try_lanes<N, 1>(g, lanes, local, factors) ||
               grouped_try_lanes<N, 2>(g, lanes, local, factors) ||
               grouped_try_lanes<N, 4>(g, lanes, local, factors) ||
               grouped_try_lanes<N, 8>(g, lanes, local, factors) ||
               grouped_try_lanes<N, 16>(g, lanes, local, factors));
    }
    return true;
}

template <int LO, int... Ns>
__device__ __forceinline__ void grouped_dispatch(const GroupDesc &g, int n, int local, int factors,
                                                 std::integer_sequence<int, Ns...>)
{
    (void)(grouped_try<LO + Ns>(g, n, local, factors) || ...);
}

/* Work item `it` of a grouped launch over sizes LO..HI (all threads of the
 * workgroup): find its group (uniform), then solve its systems. */
template <int LO, int HI>
__device__ __forceinline__ void grouped_run(const GroupedArgs &a, int it)
{
    int gi = 0;
    for (int k = 1; k < a.ngroups; ++k)
        if (it >= a.g[k].item0) gi = k;
    gi = __builtin_amdgcn_readfirstlane(gi);
    const GroupDesc &g = a.g[gi];
    grouped_dispatch<LO>(g, __builtin_amdgcn_readfirstlane(g.n), it - g.item0, g.factors,
                         std::make_integer_sequence<int, HI - LO + 1>{});
}

/* Grouped kernels (grouped_c0.hip .. grouped_c2.hip), one per size class:
 * one workgroup per work item. */
hipError_t grouped_c0_launch(const GroupedArgs &a, unsigned items, hipStream_t st);
hipError_t grouped_c1_launch(const GroupedArgs &a, unsigned items, hipStream_t st);
hipError_t grouped_c2_launch(const GroupedArgs &a, unsigned items, hipStream_t st);

/* Ragged kernels (ragged_c0.hip .. ragged_c2.hip: separate translation units,
 * compiled in parallel), one per size class: `grid` workgroups each. */
hipError_t ragged_c0_launch(const RaggedArgs &a, unsigned grid, hipStream_t st);
hipError_t ragged_c1_launch(const RaggedArgs &a, unsigned grid, hipStream_t st);
hipError_t ragged_c2_launch(const RaggedArgs &a, unsigned grid, hipStream_t st);
/* waves per SIMD each ragged class kernel is compiled for (its resident
 * grid is compute units x this) */
__host__ __device__ constexpr int ragged_class_waves(int c) { return c == 0 ? 2 : 3; }

}  // namespace lupp

#define LUPP_RAGGED_ONE_INSTANCE(N)                                                 \
    namespace lupp {                                                               \
    hipError_t ragged_one_launch_##N(const RaggedArgs &a, int items, hipStream_t st)   \
    {                                                                              \
        if (items <= 0) return hipSuccess;                                         \
        hipLaunchKernelGGL((k_ragged_one<N>), dim3((unsigned)items), dim3(kRaggedThreads), 0, st, a); \
        return hipGetLastError();                                                  \
    }                                                                              \
    }

#endif
