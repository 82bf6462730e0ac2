/* Lanes-per-system batched solve for the interleaved (SoA) layout, with the
 * global traffic staged through LDS (Section 3: coalesced accesses to the
 * batch; Section 3.2: several rows per thread, several systems per wave).
 *
 * The solve itself is the one of k_lanes (T lanes per system, K = ceil(n/T)
 * rows per lane, logical pivoting). What differs is how the matrices move
 * between HBM and registers. In the interleaved layout element (i, j) of
 * consecutive systems is contiguous, but a wave holds only 64/T systems, so a
 * direct load of one element per lane touches T rows x (64/T) systems: T
 * partial cache lines per instruction, and the rest of every line is read by
 * other waves. Here a workgroup owns S = 16 consecutive systems (one 128-byte
 * line per matrix element) and moves column chunks of its S matrices through
 * LDS: every global load or store instruction covers whole lines, and the
 * transposition into the lanes' row ownership happens in LDS.
 *
 * LDS tile of a column chunk: element (column c, row i, system y) at
 *     (c * NP + i) * S + (y ^ sw(i)),
 * NP = rows padded to whole segments. The XOR swizzle sw(i) permutes the
 * systems of each row so that both access patterns are free of bank
 * conflicts within each half-wave (32 lanes x 8 bytes = all 64 banks):
 *   - cooperative side: 32 consecutive (row, system) pairs, systems fastest;
 *   - lane side: 32/T systems x T consecutive rows of a segment slot.
 * sw(i) = ((i >> max(0, 5 - log2 S)) << log2(32/T)) & (S - 1).
 *
 * Rows past n and systems past the batch end use an out-of-range buffer
 * offset: they load zeros (as in k_lanes) and store nothing.
 */
#ifndef LUPP_KERNELS_LANES_SOA_H
#define LUPP_KERNELS_LANES_SOA_H

#include "internal.h"
#include "lupp_device.h"

namespace lupp {

__host__ __device__ constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }

template <int N, int T>
struct soa_shape {
    static constexpr int SPW = 64 / T;                   /* systems per wave */
    static constexpr int S = SPW > 16 ? SPW : 16;        /* systems per workgroup */
    static constexpr int WPB = S / SPW;                  /* waves per workgroup */
    static constexpr int NT = 64 * WPB;                  /* threads = S * T */
    static constexpr int K = (N + T - 1) / T;
    static constexpr int NP = K * T;                     /* rows padded to segments */
    static constexpr int LOG_S = ilog2c(S);
    static constexpr int LOG_SPH = ilog2c(T >= 32 ? 1 : 32 / T); /* systems per half-wave */
    static constexpr int SH = LOG_S >= 5 ? 0 : 5 - LOG_S;
    /* columns per LDS chunk: about 4 KB of tile per wave */
    static constexpr int CJ0 = (4096 * WPB) / (NP * S * 8);
    static constexpr int CJ = CJ0 < 1 ? 1 : (CJ0 > N ? N : CJ0);
    static constexpr int NCH = (N + CJ - 1) / CJ;        /* chunks */
    /* 512-thread workgroups (T = 32) need two per CU: at most 128 VGPRs;
     * 16 lanes (two rows per lane up to n = 32) fit 168 VGPRs, three waves
     * per SIMD */
    static constexpr int MIN_WAVES_EU = WPB >= 8 ? 4 : (T == 16 ? 3 : 1);
    /* pivot-row broadcast chunk (columns) */
    static constexpr int CH = lanes_chunk<N, T>();
    /* global loads in flight during the staging: this many column chunks
     * ahead of the one being transposed */
    static constexpr int LA = 2;
    static_assert(NT == S * T, "shape");
};

template <int N, int T>
__device__ __forceinline__ int soa_sw(int i)
{
    using Sh = soa_shape<N, T>;
    return ((i >> Sh::SH) << Sh::LOG_SPH) & (Sh::S - 1);
}

template <int N, int T, bool F, bool Tl>
__global__ void __launch_bounds__((soa_shape<N, T>::NT))
    __attribute__((amdgpu_waves_per_eu(soa_shape<N, T>::MIN_WAVES_EU))) k_lanes_soa(SolveArgs a, int factors)
{
    using Sh = soa_shape<N, T>;
    constexpr int S = Sh::S, K = Sh::K, NP = Sh::NP, CJ = Sh::CJ, NCH = Sh::NCH;
    constexpr int QB = NP / T; /* cooperative accesses per column and thread */
    __shared__ double tile[CJ * NP * S];
    __shared__ double xb[NP * S];
    __shared__ int ipl[NP * S];
    __shared__ int infl[S];

    int tid = (int)threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t sys0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * S;
    const int64_t rem = a.batch - sys0;
    const int nvalid = (int)(rem < S ? rem : S);

    /* Lane geometry, all derived from tid (rebuilt after the solve from a
     * fenced copy of tid, so that none of it stays live across the solve):
     * lane side: segment g, lane t of the segment, system yl, rows t + s*T;
     * cooperative side: system yw, rows ci0 + multiples of T. */
    int g, t, yl, yw, ci0;
    auto set_geometry = [&]() __attribute__((always_inline)) {
        const int lane = tid & 63;
        g = lane / T;
        t = lane % T;
        yl = wave * Sh::SPW + g;
        yw = tid & (S - 1);
        ci0 = tid >> Sh::LOG_S;
    };
    set_geometry();

    /* The cooperative rows of a wave are ci0 = cw .. cw + 64/S - 1, so each
     * descriptor is based at the wave's first row (a uniform address) and
     * its extent spans 64/S rows: the per-lane offsets stay below 2^31
     * bytes for any ldbatch under 2^31 / (8 * (64/S - 1) + 8). */
    const int cw = (wave * 64) >> Sh::LOG_S;
    double *baseA = a.A + sys0 + (int64_t)cw * a.sA;
    double *baseB = a.b + sys0 + (int64_t)cw * a.sB;
    const int64_t colA = a.lda * a.sA;
    constexpr int RW = 64 / S; /* cooperative rows per wave */
    const uint32_t bytesA = (uint32_t)(((int64_t)(RW - 1) * a.sA + nvalid) * 8);
    const uint32_t bytesB = (uint32_t)(((int64_t)(RW - 1) * a.sB + nvalid) * 8);
    auto coop_off = [&](int64_t ld, int w) __attribute__((always_inline)) {
        return yw < nvalid ? (uint32_t)(((int64_t)(ci0 - cw) * ld + yw) * w) : kOutOfRange;
    };
    uint32_t vA = coop_off(a.sA, 8), vB = coop_off(a.sB, 8);
    /* per-lane offset of the cooperative row ci0 + ib (out of range for rows past n) */
    auto rowv = [&](uint32_t v, int ib) -> uint32_t {
        return (ib + T <= N || ci0 < N - ib) ? v : kOutOfRange;
    };
    /* LDS index of the cooperative element (chunk column c, row block ib) */
    auto cidx = [&](int c, int ib) { const int i = ci0 + ib; return (c * NP + i) * S + (yw ^ soa_sw<N, T>(i)); };
    /* LDS index of a lane-side element (chunk column c, row i) */
    auto lidx = [&](int c, int i) { return (c * NP + i) * S + (yl ^ soa_sw<N, T>(i)); };

    /* ---------------------------------------------------------- load */
    double m[K][N];
    double x[K];
    int pos[K];
    static_for<0, K>(LUPP_SF(sc) {
        constexpr int s = decltype(sc)::value;
        pos[s] = t + s * T < N ? t + s * T : -1;
    });
    /* the loads of column chunk c + LA are issued before chunk c is
     * transposed, so LA + 1 chunks are in flight per wave while the staging
     * registers of a chunk die as its matrix registers fill (the whole
     * matrix in flight would hold 2*n*n/T extra VGPRs: a wave per SIMD) */
    double v[N * QB];
    double vb[QB];
    auto load_chunk = [&](auto chc) __attribute__((always_inline)) {
        constexpr int ch = decltype(chc)::value;
        if constexpr (ch < NCH) {
            constexpr int j0 = ch * CJ;
            constexpr int cj = (j0 + CJ <= N) ? CJ : N - j0;
            static_for<j0 * QB, (j0 + cj) * QB>(LUPP_SF(qc) {
                constexpr int q = decltype(qc)::value;
                constexpr int j = q / QB, ib = (q % QB) * T;
                const auto rc = make_rsrc(baseA + (int64_t)j * colA + (int64_t)ib * a.sA, bytesA);
                v[q] = buf_load_f64(rc, rowv(vA, ib), 0);
            });
        }
    };
    static_for<0, Sh::LA>(load_chunk);
    {
        static_for<0, QB>(LUPP_SF(qc) {
            constexpr int ib = decltype(qc)::value * T;
            vb[decltype(qc)::value] =
                buf_load_f64(make_rsrc(baseB + (int64_t)ib * a.sB, bytesB), rowv(vB, ib), 0);
        });
    }
    static_for<0, NCH>(LUPP_SF(chc) {
        constexpr int ch = decltype(chc)::value;
        load_chunk(std::integral_constant<int, ch + Sh::LA>{});
        constexpr int j0 = ch * CJ;
        constexpr int cj = (j0 + CJ <= N) ? CJ : N - j0;
        static_for<0, cj * QB>(LUPP_SF(qc) {
            constexpr int q = decltype(qc)::value;
            tile[cidx(q / QB, (q % QB) * T)] = v[j0 * QB + q];
        });
        if constexpr (ch == NCH - 1) {
            static_for<0, QB>(LUPP_SF(qc) {
                constexpr int q = decltype(qc)::value;
                xb[cidx(0, q * T)] = vb[q];
            });
        }
        __syncthreads();
        static_for<0, cj>(LUPP_SF(cc) {
            constexpr int c = decltype(cc)::value;
            static_for<0, K>(LUPP_SF(sc) {
                constexpr int s = decltype(sc)::value;
                m[s][j0 + c] = tile[lidx(c, t + s * T)];
            });
        });
        if constexpr (ch == NCH - 1) {
            static_for<0, K>(LUPP_SF(sc) {
                constexpr int s = decltype(sc)::value;
                x[s] = xb[lidx(0, t + s * T)];
            });
        }
        __syncthreads();
    });

    /* ---------------------------------------------------------- solve */
    constexpr int KP = (N + T - 1) / T;
    int pv[KP];
    static_for<0, KP>(LUPP_SF(sc) { pv[decltype(sc)::value] = 0; });
    constexpr bool kSettle = lanes_settle<N, T>();
    const int inf = lanes_getrf_solve<N, T, F, Tl, Sh::CH, kSettle>(m, x, pos, g * T, [&](int k, int val) {
        const int c = k / T;
        static_for<0, KP>(LUPP_SF(sc) {
            constexpr int cc = decltype(sc)::value;
            if (cc == c) {
                pv[cc] = (t == k % T) ? val : pv[cc];
                if constexpr (kSettle) settle(pv[cc]);
            }
        });
    }, a.tile, a.thresh);

    /* ---------------------------------------------------------- store */
    baseA = opaque_ptr(baseA);
    baseB = opaque_ptr(baseB);
    const int64_t sAs = opaque_i64(a.sA), sBs = opaque_i64(a.sB);
    settle(tid);
    set_geometry();
    vA = coop_off(sAs, 8);
    vB = coop_off(sBs, 8);
    if (factors) {
        static_for<0, NCH>(LUPP_SF(chc) {
            constexpr int j0 = decltype(chc)::value * CJ;
            constexpr int cj = (j0 + CJ <= N) ? CJ : N - j0;
            /* slot s holds row pos[s] of the LAPACK-ordered factors */
            static_for<0, K>(LUPP_SF(sc) {
                constexpr int s = decltype(sc)::value;
                if (pos[s] >= 0) {
                    static_for<0, cj>(LUPP_SF(cc) {
                        constexpr int c = decltype(cc)::value;
                        tile[lidx(c, pos[s])] = m[s][j0 + c];
                    });
                }
            });
            __syncthreads();
            static_for<0, cj * QB>(LUPP_SF(qc) {
                constexpr int q = decltype(qc)::value;
                constexpr int c = q / QB, ib = (q % QB) * T;
                const auto rc = make_rsrc(baseA + (int64_t)(j0 + c) * colA + (int64_t)ib * sAs, bytesA);
                buf_store_f64(rc, rowv(vA, ib), 0, tile[cidx(c, ib)]);
            });
            __syncthreads();
        });
    }
    static_for<0, K>(LUPP_SF(sc) {
        constexpr int s = decltype(sc)::value;
        if (pos[s] >= 0) xb[lidx(0, pos[s])] = x[s];
    });
    static_for<0, KP>(LUPP_SF(sc) {
        constexpr int c = decltype(sc)::value;
        const int k = t + c * T;
        if (k < N) ipl[lidx(0, k)] = pv[c];
    });
    if (t == 0) infl[yl] = inf;
    __syncthreads();
    {
        const bool ok = infl[yw] == 0;
        int32_t *baseP = a.ipiv + sys0 + (int64_t)cw * sAs;
        const uint32_t bytesP = (uint32_t)(((int64_t)(RW - 1) * sAs + nvalid) * 4);
        const uint32_t vP = coop_off(sAs, 4);
        static_for<0, QB>(LUPP_SF(qc) {
            constexpr int ib = decltype(qc)::value * T;
            buf_store_f64(make_rsrc(baseB + (int64_t)ib * sBs, bytesB), ok ? rowv(vB, ib) : kOutOfRange,
                          0, xb[cidx(0, ib)]);
            buf_store_i32(make_rsrc(baseP + (int64_t)ib * sAs, bytesP), rowv(vP, ib), 0,
                          ipl[cidx(0, ib)]);
        });
        const auto ri = make_rsrc(a.info + sys0, (uint32_t)nvalid * 4u);
        if (tid < S) buf_store_i32(ri, (uint32_t)tid * 4u, 0, infl[tid]);
    }
}

template <int N, int T>
hipError_t launch_lanes_soa(const SolveArgs &a, bool factors, hipStream_t st)
{
    using Sh = soa_shape<N, T>;
    const int64_t blocks = (a.batch + Sh::S - 1) / Sh::S;
    /* arithmetic x pivoting instances: strict, FMA, strict + tile-local */
    if (a.fma && a.tile > 0) return hipErrorNotSupported;
    if (a.fma)
        hipLaunchKernelGGL((k_lanes_soa<N, T, true, false>), dim3((unsigned)blocks), dim3(Sh::NT), 0,
                           st, a, (int)factors);
    else if (a.tile > 0)
        hipLaunchKernelGGL((k_lanes_soa<N, T, false, true>), dim3((unsigned)blocks), dim3(Sh::NT), 0,
                           st, a, (int)factors);
    else
        hipLaunchKernelGGL((k_lanes_soa<N, T, false, false>), dim3((unsigned)blocks), dim3(Sh::NT),
                           0, st, a, (int)factors);
    return hipGetLastError();
}

}  // namespace lupp

#endif
