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
 * The uniform part goes into the buffer descriptor and its offset field,
 * the per-lane part into one VGPR shared by all elements.
 */
#ifndef LUPP_KERNELS_THREAD_H
#define LUPP_KERNELS_THREAD_H

#include "internal.h"
#include "lupp_device.h"

namespace lupp {

/* Occupancy target per size: the register-resident matrix takes 2*N*N VGPRs.
 * Each value is the highest occupancy the compiler reaches for that size
 * without scratch memory (gfx950: n <= 6 at 4 or more waves per SIMD, n = 7
 * and 8 at 3, n = 9 and 10 at 2 - 208 and 250 VGPRs -, n >= 11 at 1). */
template <int N>
constexpr int thread_waves_per_eu() { return N <= 6 ? 4 : (N <= 8 ? 3 : (N <= 10 ? 2 : 1)); }

template <int N, bool F, bool Tl>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(thread_waves_per_eu<N>())))
    k_thread(SolveArgs a, int layout, int factors)
{
    const bool soa = layout == LUPP_SOA;
    const int64_t s0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x;
    const int64_t rem = a.batch - s0;
    const uint32_t nvalid = (uint32_t)(rem < (int64_t)blockDim.x ? rem : blockDim.x);
    const uint32_t tid = threadIdx.x;
    const bool active = tid < nvalid;

    /* Element (i, j) of this lane's system sits at
     *   base + j*C + i*R + tid*V   (elements),
     * SoA: base = A + s0, C = lda*ldbatch, R = ldbatch, V = 1;
     * AoS: base = A + s0*strideA, C = lda, R = 1, V = strideA.
     * Every element gets its own descriptor based at base + j*C + i*R (a
     * uniform 64-bit address built with scalar adds), so the descriptor
     * extent covers only the workgroup's lanes - nvalid*V elements - whatever
     * the strides: an interleaved batch may span any number of bytes. Lanes
     * past the batch get an out-of-range lane offset. */
    double *bA = a.A + (soa ? s0 : s0 * a.sA);
    double *bB = a.b + (soa ? s0 : s0 * a.sB);
    const int64_t C = soa ? a.lda * a.sA : a.lda;
    const int64_t R = soa ? a.sA : 1;
    const int64_t RB = soa ? a.sB : 1;
    const uint32_t nbA = nvalid * (uint32_t)(soa ? 8 : a.sA * 8);
    const uint32_t nbB = nvalid * (uint32_t)(soa ? 8 : a.sB * 8);
    const uint32_t voA = !active ? kOutOfRange : (soa ? tid * 8u : tid * (uint32_t)a.sA * 8u);
    const uint32_t voB = !active ? kOutOfRange : (soa ? tid * 8u : tid * (uint32_t)a.sB * 8u);

    double m[N][N];
    double x[N];
    int piv[N];
    static_for<0, N>([&](auto jc) __attribute__((always_inline)) {
        constexpr int j = decltype(jc)::value;
        static_for<0, N>([&](auto ic) __attribute__((always_inline)) {
            constexpr int i = decltype(ic)::value;
            m[j][i] = buf_load_f64(make_rsrc(bA + j * C + i * R, nbA), voA, 0);
        });
        asm volatile("" ::: "memory");
    });
    {
        static_for<0, N>([&](auto ic) __attribute__((always_inline)) {
            constexpr int i = decltype(ic)::value;
            x[i] = buf_load_f64(make_rsrc(bB + i * RB, nbB), voB, 0);
        });
    }

    const int inf = thread_getrf_solve<N, true, F, Tl>(m, x, piv, a.tile, a.thresh);

    /* fresh copies of the bases and strides: the store addresses are then
     * rebuilt here instead of being kept live (in SGPRs) across the solve */
    bA = opaque_ptr(bA);
    bB = opaque_ptr(bB);
    const int64_t Cs = opaque_i64(C), Rs = opaque_i64(R), RBs = opaque_i64(RB);
    if (factors) {
        static_for<0, N>([&](auto jc) __attribute__((always_inline)) {
            constexpr int j = decltype(jc)::value;
            static_for<0, N>([&](auto ic) __attribute__((always_inline)) {
                constexpr int i = decltype(ic)::value;
                buf_store_f64(make_rsrc(bA + j * Cs + i * Rs, nbA), voA, 0, m[j][i]);
            });
            asm volatile("" ::: "memory");
        });
    }
    {
        const uint32_t vx = inf == 0 ? voB : kOutOfRange;
        static_for<0, N>([&](auto ic) __attribute__((always_inline)) {
            constexpr int i = decltype(ic)::value;
            buf_store_f64(make_rsrc(bB + i * RBs, nbB), vx, 0, x[i]);
        });
    }
    /* AoS ipiv[s*N + k]; SoA ipiv[k*ldbatch + s] */
    {
        int32_t *bP = opaque_ptr(a.ipiv + (soa ? s0 : s0 * N));
        const uint32_t nbP = nvalid * (soa ? 4u : N * 4u);
        const uint32_t voP = !active ? kOutOfRange : (soa ? tid * 4u : tid * N * 4u);
        const int64_t RP = soa ? a.sA : 1;
        static_for<0, N>([&](auto kc) __attribute__((always_inline)) {
            constexpr int k = decltype(kc)::value;
            buf_store_i32(make_rsrc(bP + k * RP, nbP), voP, 0, piv[k]);
        });
    }
    buf_store_i32(make_rsrc(a.info + s0, nvalid * 4u), tid * 4u, 0, inf);
}

template <int N>
hipError_t launch_thread(const SolveArgs &a, int layout, bool factors, int wpb, hipStream_t st)
{
    const int threads = 64 * (wpb > 0 ? wpb : 4);
    const int64_t blocks = (a.batch + threads - 1) / threads;
    /* arithmetic x pivoting instances: strict, FMA, strict + tile-local */
    if (a.fma && a.tile > 0) return hipErrorNotSupported;
    if (a.fma)
        hipLaunchKernelGGL((k_thread<N, true, false>), dim3((unsigned)blocks), dim3(threads), 0, st,
                           a, layout, (int)factors);
    else if (a.tile > 0)
        hipLaunchKernelGGL((k_thread<N, false, true>), dim3((unsigned)blocks), dim3(threads), 0, st,
                           a, layout, (int)factors);
    else
        hipLaunchKernelGGL((k_thread<N, false, false>), dim3((unsigned)blocks), dim3(threads), 0, st,
                           a, layout, (int)factors);
    return hipGetLastError();
}

}  // namespace lupp

#define LUPP_THREAD_INSTANCE(N)                                                      \
    namespace lupp {                                                                \
    LaunchFn thread_fn_##N() { return launch_thread<N>; }                           \
    const void *thread_sym_##N() { return reinterpret_cast<const void *>(&k_thread<N, false, false>); } \
    }

#endif
