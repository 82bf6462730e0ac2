/* Thread-per-system batched solve: one lane factors and solves one system
 * held entirely in its registers (Section 3.2, single-threaded solvers: the
 * matrix never leaves the register file, so the data-dependent pivot row
 * costs select instructions, not memory accesses).
 *
 * Element e = i + j*lda of the system served by lane `tid` of the workgroup
 * starting at system s0 is read at  base + e*E + tid*V  with
 *   SoA: base = A + s0,        E = ldbatch, V = 1   (a wave reads 512
 *        contiguous bytes per element);
 *   AoS: base = A + s0*strideA, E = 1,       V = strideA (each lane walks its
 *        own matrix; the wave's accesses are served through L1/L2 lines).
 * The uniform part goes into the buffer descriptor, the per-lane part into
 * one VGPR shared by all elements.
 */
#ifndef LUPP_KERNELS_THREAD_H
#define LUPP_KERNELS_THREAD_H

#include "internal.h"
#include "lupp_device.h"

namespace lupp {

template <int N>
__global__ void __launch_bounds__(256) k_thread(SolveArgs a, int layout, int factors)
{
    const bool soa = layout == LUPP_SOA;
    const int64_t s0 = (int64_t)blockIdx.x * blockDim.x;
    const int64_t rem = a.batch - s0;
    const uint32_t nvalid = (uint32_t)(rem < (int64_t)blockDim.x ? rem : blockDim.x);
    const uint32_t tid = threadIdx.x;

    const int64_t EA = soa ? a.sA : 1, EB = soa ? a.sB : 1;
    const double *bA = a.A + (soa ? s0 : s0 * a.sA);
    const double *bB = a.b + (soa ? s0 : s0 * a.sB);
    /* bytes reachable from one element's base by the block's valid lanes */
    const uint32_t nbA = soa ? nvalid * 8u : nvalid * (uint32_t)a.sA * 8u;
    const uint32_t nbB = soa ? nvalid * 8u : nvalid * (uint32_t)a.sB * 8u;
    const uint32_t voA = soa ? tid * 8u : tid * (uint32_t)a.sA * 8u;
    const uint32_t voB = soa ? tid * 8u : tid * (uint32_t)a.sB * 8u;

    double m[N][N];
    double x[N];
    int piv[N];
    static_for<0, N>([&](auto jc) __attribute__((always_inline)) {
        constexpr int j = decltype(jc)::value;
        static_for<0, N>([&](auto ic) __attribute__((always_inline)) {
            constexpr int i = decltype(ic)::value;
            m[j][i] = buf_load_f64(make_rsrc(bA + (i + j * a.lda) * EA, nbA), voA, 0);
        });
    });
    static_for<0, N>([&](auto ic) __attribute__((always_inline)) {
        constexpr int i = decltype(ic)::value;
        x[i] = buf_load_f64(make_rsrc(bB + i * EB, nbB), voB, 0);
    });

    const int inf = thread_getrf_solve<N, true>(m, x, piv);

    if (factors) {
        static_for<0, N>([&](auto jc) __attribute__((always_inline)) {
            constexpr int j = decltype(jc)::value;
            static_for<0, N>([&](auto ic) __attribute__((always_inline)) {
                constexpr int i = decltype(ic)::value;
                buf_store_f64(make_rsrc(bA + (i + j * a.lda) * EA, nbA), voA, 0, m[j][i]);
            });
        });
    }
    const uint32_t vx = inf == 0 ? voB : kOutOfRange;
    static_for<0, N>([&](auto ic) __attribute__((always_inline)) {
        constexpr int i = decltype(ic)::value;
        buf_store_f64(make_rsrc(bB + i * EB, nbB), vx, 0, x[i]);
    });
    /* AoS ipiv[s*N + k]; SoA ipiv[k*ldbatch + s] */
    const int32_t *bP = a.ipiv + (soa ? s0 : s0 * N);
    const int64_t EP = soa ? a.sA : 1;
    const uint32_t nbP = soa ? nvalid * 4u : nvalid * N * 4u;
    const uint32_t voP = soa ? tid * 4u : tid * N * 4u;
    static_for<0, N>([&](auto kc) __attribute__((always_inline)) {
        constexpr int k = decltype(kc)::value;
        buf_store_i32(make_rsrc(bP + k * EP, nbP), voP, 0, piv[k]);
    });
    buf_store_i32(make_rsrc(a.info + s0, nvalid * 4u), tid * 4u, 0, inf);
}

template <int N>
hipError_t launch_thread(const SolveArgs &a, int layout, bool factors, int wpb, hipStream_t st)
{
    const int threads = 64 * (wpb > 0 ? wpb : 4);
    const int64_t blocks = (a.batch + threads - 1) / threads;
    hipLaunchKernelGGL((k_thread<N>), dim3((unsigned)blocks), dim3(threads), 0, st, a, layout,
                       (int)factors);
    return hipGetLastError();
}

}  // namespace lupp

#define LUPP_THREAD_INSTANCE(N)                                                      \
    namespace lupp {                                                                \
    LaunchFn thread_fn_##N() { return launch_thread<N>; }                           \
    const void *thread_sym_##N() { return reinterpret_cast<const void *>(&k_thread<N>); } \
    }

#endif
