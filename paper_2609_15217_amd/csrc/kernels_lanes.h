/* Lanes-per-system batched solve: T lanes of a wave64 share one system, each
 * owning K = ceil(n/T) rows in registers (Section 3.2, multi-threaded
 * solvers: register blocking with several rows per thread, several systems
 * per wave, phantom rows when T does not divide n).
 *
 * Lane mapping: wave w of the workgroup serves systems
 * (block*wpb + w)*(64/T) + g for segments g = 0..64/T-1; lane t of segment g
 * owns rows t, t+T, ... .
 * AoS: a segment reads T consecutive doubles of a column per load.
 * SoA: a wave reads 64/T consecutive systems of T rows per load (partial
 * cache lines; the library launches the LDS-staged kernel of
 * kernels_lanes_soa.h for this layout instead).
 * Both layouts are handled by the same code: only the uniform base pointers
 * and the per-lane byte offsets differ. Lanes past the end of the batch and
 * phantom rows use an out-of-range buffer offset, so they load zeros and
 * store nothing.
 */
#ifndef LUPP_KERNELS_LANES_H
#define LUPP_KERNELS_LANES_H

#include "internal.h"
#include "lupp_device.h"

namespace lupp {

template <int N, int T, bool F, bool Tl>
__global__ void __launch_bounds__(256) k_lanes(SolveArgs a, int layout, int factors)
{
    constexpr int K = lanes_shape<N, T>::K;
    constexpr int SPW = 64 / T; /* systems per wave */
    const bool soa = layout == LUPP_SOA;
    const int lane = (int)__lane_id();
    const int g = lane / T, t = lane % T;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t sys0 = ((int64_t)xcd_block(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + wave) * SPW;
    const int64_t rem = a.batch - sys0;
    const int nvalid = (int)(rem <= 0 ? 0 : (rem < SPW ? rem : SPW));
    const bool active = g < nvalid;

    /* uniform bases and extents, per-lane offsets of row r of segment g */
    double *baseA = a.A + (soa ? sys0 : sys0 * a.sA);
    const int64_t colA = soa ? a.lda * a.sA : a.lda; /* elements between columns */
    const uint32_t bytesA = (uint32_t)((soa ? (int64_t)(N - 1) * a.sA + nvalid : (int64_t)nvalid * a.sA) * 8);
    double *baseB = a.b + (soa ? sys0 : sys0 * a.sB);
    const uint32_t bytesB = (uint32_t)((soa ? (int64_t)(N - 1) * a.sB + nvalid : (int64_t)nvalid * a.sB) * 8);
    auto offA = [&](int r) { return (uint32_t)((soa ? (int64_t)r * a.sA + g : (int64_t)g * a.sA + r) * 8); };
    auto offB = [&](int r) { return (uint32_t)((soa ? (int64_t)r * a.sB + g : (int64_t)g * a.sB + r) * 8); };

    double m[K][N];
    double x[K];
    int pos[K];
    uint32_t vo[K];
    static_for<0, K>([&](auto sc) __attribute__((always_inline)) {
        constexpr int s = decltype(sc)::value;
        const int r = t + s * T;
        pos[s] = r < N ? r : -1;
        vo[s] = (active && r < N) ? offA(r) : kOutOfRange;
    });
    static_for<0, N>([&](auto jc) __attribute__((always_inline)) {
        constexpr int j = decltype(jc)::value;
        const auto rc = make_rsrc(baseA + j * colA, bytesA);
        static_for<0, K>([&](auto sc) __attribute__((always_inline)) {
            constexpr int s = decltype(sc)::value;
            m[s][j] = buf_load_f64(rc, vo[s], 0);
        });
    });
    const auto rB = make_rsrc(baseB, bytesB);
    static_for<0, K>([&](auto sc) __attribute__((always_inline)) {
        constexpr int s = decltype(sc)::value;
        const int r = t + s * T;
        x[s] = buf_load_f64(rB, (active && r < N) ? offB(r) : kOutOfRange, 0);
    });

    /* ipiv[k] is stored by lane k % T of the segment: keep it in slot k / T */
    constexpr int KP = (N + T - 1) / T;
    int pv[KP];
    static_for<0, KP>([&](auto sc) __attribute__((always_inline)) { pv[decltype(sc)::value] = 0; });
    constexpr bool kSettle = lanes_settle<N, T>();
    /* the tile-local instances hold the second search's values too: 4-column
     * chunks keep them at three waves per SIMD (n = 32: 170 -> 162 VGPRs) */
    constexpr int CH = (Tl && kSettle) ? 4 : lanes_chunk<N, T>();
    const int inf = lanes_getrf_solve<N, T, F, Tl, CH, kSettle>(m, x, pos, g * T, [&](int k, int v) {
        const int c = k / T;
        static_for<0, KP>([&](auto sc) __attribute__((always_inline)) {
            constexpr int cc = decltype(sc)::value;
            if (cc == c) {
                pv[cc] = (t == k % T) ? v : pv[cc];
                if constexpr (kSettle) settle(pv[cc]);
            }
        });
    }, a.tile, a.thresh);

    baseA = opaque_ptr(baseA);
    baseB = opaque_ptr(baseB);
    const auto rBs = make_rsrc(baseB, bytesB);
    /* slot s holds row pos[s] of the LAPACK-ordered result */
    static_for<0, K>([&](auto sc) __attribute__((always_inline)) {
        constexpr int s = decltype(sc)::value;
        vo[s] = (active && pos[s] >= 0) ? offA(pos[s]) : kOutOfRange;
    });
    if (factors) {
        static_for<0, N>([&](auto jc) __attribute__((always_inline)) {
            constexpr int j = decltype(jc)::value;
            const auto rc = make_rsrc(baseA + j * colA, bytesA);
            static_for<0, K>([&](auto sc) __attribute__((always_inline)) {
                constexpr int s = decltype(sc)::value;
                buf_store_f64(rc, vo[s], 0, m[s][j]);
            });
        });
    }
    static_for<0, K>([&](auto sc) __attribute__((always_inline)) {
        constexpr int s = decltype(sc)::value;
        const bool ok = active && pos[s] >= 0 && inf == 0;
        buf_store_f64(rBs, ok ? offB(pos[s]) : kOutOfRange, 0, x[s]);
    });
    /* AoS ipiv[s*N + k]; SoA ipiv[k*ldbatch + s] */
    const auto rP = make_rsrc(a.ipiv + (soa ? sys0 : sys0 * N),
                              (uint32_t)((soa ? (int64_t)(N - 1) * a.sA + nvalid : (int64_t)nvalid * N) * 4));
    static_for<0, KP>([&](auto sc) __attribute__((always_inline)) {
        constexpr int c = decltype(sc)::value;
        const int k = t + c * T;
        const uint32_t o = (uint32_t)((soa ? (int64_t)k * a.sA + g : (int64_t)g * N + k) * 4);
        buf_store_i32(rP, (active && k < N) ? o : kOutOfRange, 0, pv[c]);
    });
    const auto rI = make_rsrc(a.info + sys0, (uint32_t)nvalid * 4u);
    buf_store_i32(rI, (active && t == 0) ? (uint32_t)g * 4u : kOutOfRange, 0, inf);
}

template <int N, int T>
hipError_t launch_lanes_soa(const SolveArgs &a, bool factors, hipStream_t st);

/* AoS: this kernel with `wpb` waves per workgroup; SoA: the LDS-staged kernel
 * (kernels_lanes_soa.h), whose workgroup shape is fixed (wpb is ignored). */
template <int N, int T>
hipError_t launch_lanes(const SolveArgs &a, int layout, bool factors, int wpb, hipStream_t st)
{
    if (layout == LUPP_SOA) return launch_lanes_soa<N, T>(a, factors, st);
    const int w = wpb > 0 ? wpb : 4;
    const int64_t per_block = (int64_t)w * (64 / T);
    const int64_t blocks = (a.batch + per_block - 1) / per_block;
    /* arithmetic x pivoting instances: strict, FMA, strict + tile-local */
    if (a.fma && a.tile > 0) return hipErrorNotSupported;
    if (a.fma)
        hipLaunchKernelGGL((k_lanes<N, T, true, false>), dim3((unsigned)blocks), dim3(64 * w), 0, st,
                           a, layout, (int)factors);
    else if (a.tile > 0)
        hipLaunchKernelGGL((k_lanes<N, T, false, true>), dim3((unsigned)blocks), dim3(64 * w), 0, st,
                           a, layout, (int)factors);
    else
        hipLaunchKernelGGL((k_lanes<N, T, false, false>), dim3((unsigned)blocks), dim3(64 * w), 0,
                           st, a, layout, (int)factors);
    return hipGetLastError();
}

}  // namespace lupp

/* One registry entry per (n, T), defined in the translation unit that
 * instantiates the kernel. */
#define LUPP_LANES_INSTANCE(N, T)                                                   \
    namespace lupp {                                                               \
    LaunchFn lanes_fn_##N##_##T() { return launch_lanes<N, T>; }                   \
    const void *lanes_sym_##N##_##T(int layout)                                    \
    {                                                                              \
        return layout == LUPP_SOA ? reinterpret_cast<const void *>(&k_lanes_soa<N, T, false, false>) \
                                  : reinterpret_cast<const void *>(&k_lanes<N, T, false, false>); \
    }                                                                              \
    }

#endif
