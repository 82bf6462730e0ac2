/* Device-callable LU with partial pivoting for tiny systems (n <= 32), HIP for
 * gfx950 (CDNA4, wave64).
 *
 * This header is the device-side half of the library: a user kernel includes
 * it and calls a solver from inside its own per-system or per-point code, as
 * the paper's device-callable solvers are called from inside the fused
 * constitutive-law kernel (Section 3.2 and Section 3.3; Algorithm 2).
 *
 * Arithmetic contract (strict mode, the default):
 *   - LU with partial pivoting as in Section 2.2: at step k the pivot is the
 *     candidate of largest magnitude in column k, lowest current row position
 *     on ties; rows are interchanged (physically in the thread path, logically
 *     in the lanes path, with the factors written back in the interchanged
 *     order), multipliers are l_ik = a_ik / a_kk (a true, correctly rounded
 *     division), and the trailing update is a_ij = a_ij - l_ik * u_kj as one
 *     rounded multiply followed by one rounded subtract;
 *   - forward substitution applies b_i = b_i - l_ik * y_k in ascending k, back
 *     substitution divides by u_jj and then eliminates column j above the
 *     diagonal, for j descending.
 * Every element therefore receives the same sequence of rounded operations as
 * the textbook algorithm, so results are bitwise reproducible across thread
 * and lanes mappings, layouts, batch compositions and launches. Translation
 * units that use this header must be compiled with -ffp-contract=off.
 * FMA mode (the solvers' kFMA parameter): every multiply-subtract of the
 * elimination and of both substitutions is one fused multiply-add instead;
 * divisions and pivoting are unchanged, so the results are again the same
 * for every mapping (and differ from strict mode in the last bits).
 *
 * info: 0, or k+1 for the first step k whose pivot is exactly zero (the
 * factorisation still completes; the solution is then not computed).
 * ipiv: LAPACK convention, ipiv[k] = 1-based row exchanged with row k.
 */
#ifndef LUPP_DEVICE_H
#define LUPP_DEVICE_H

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace lupp {

/* ------------------------------------------------------------------------ */
/* Thread-per-system solver: the whole system lives in one lane's registers. */
/* Indices into the register arrays are compile-time constants after full    */
/* unrolling; the data-dependent pivot row is selected with compare/select   */
/* chains so that nothing spills to scratch memory.                          */
/* ------------------------------------------------------------------------ */

/* a[j][i] holds element (i, j) (column-major), b the right-hand side.
 * kFactors: interchange whole rows (all n columns) so that a[][] ends holding
 * the LAPACK-ordered factors L\U; otherwise only the trailing columns move and
 * the columns left of the diagonal are garbage on return (enough for a
 * solve-only caller such as a Newton loop).
 * On return with info == 0, b holds the solution. ipiv receives the LAPACK
 * interchange sequence (1-based). */
/* Compile-time loop: f(integral_constant<int, I>) for I in [B, E). Every
 * register-array index derived from the loop variable is a constant
 * expression, so the arrays stay in registers whatever the loop size. */
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

/* Descending variant: I = E-1 down to B. */
template <int B, int E, typename F>
__device__ __forceinline__ void static_for_down(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, E - 1>{});
        static_for_down<B, E - 1>(f);
    }
}

#define LUPP_SF(v) [&](auto v) __attribute__((always_inline))

/* Register-lifetime fence: an empty asm statement that takes x and hands it
 * back, so whatever produces x is computed at this point. The solvers fence
 * values that are final long before their only use (a stored multiplier, the
 * running info, an interchange index kept for the store): left alone, the
 * compiler may keep every step's operands live and form such values at the
 * use, which costs registers (16 lanes per system at n = 32: 195 VGPRs, two
 * waves per SIMD, against 168 and three). No instruction is emitted and no
 * result changes. */
template <typename V>
__device__ __forceinline__ void settle(V &x)
{
    asm volatile("" : "+v"(x));
}

/* Whether the batched lanes kernels fence the solver's per-step results,
 * and their pivot-row broadcast chunk: the fence is used where it buys a
 * wave per SIMD and the wave pays - 16 lanes per system from n = 27
 * (195 -> 168 VGPRs at n = 32: three waves) and n = 20..24 with 4-column
 * chunks (<= 128 VGPRs: four waves instead of three; 4-7% faster at 2^19
 * systems, while n = 17..19 lost 1-3%). Elsewhere it would only hold the
 * scheduler back (n = 24 at three waves either way: 3.06 -> 3.23 ms). */
template <int N, int T>
constexpr bool lanes_settle()
{
    return T == 16 && (N >= 27 || (N >= 20 && N <= 24));
}

template <int N, int T>
constexpr int lanes_chunk()
{
    return (T == 16 && N >= 20 && N <= 24) ? 4 : 8;
}

/* a - l*u: in strict mode one rounded multiply then one rounded subtract;
 * with kFMA one fused multiply-add (fma(-l, u, a), a single rounding). */
template <bool kFMA>
__device__ __forceinline__ double msub(double a, double l, double u)
{
    if constexpr (kFMA) return __builtin_fma(-l, u, a);
    else return a - l * u;
}

/* Last row + 1 of the pivot candidates tried first at step k: the end of the
 * diagonal tile of size `tile` holding k (tile-local pivoting, the Tiled
 * solvers' rule, Section 3.2.2), or n for textbook partial pivoting
 * (tile <= 0). tile is uniform across the wave. */
__device__ __forceinline__ int pivot_tile_end(int k, int n, int tile)
{
    if (tile <= 0) return n;
    const int e = (k / tile + 1) * tile;
    return e < n ? e : n;
}

/* Pivot of column k over rows k .. N-1 (element (i, k) at a[k][i]): the
 * largest magnitude, the lowest row among equal ones, by a pairwise (tree)
 * reduction in which the right (higher) half wins only when strictly larger:
 * the choice of a left-to-right scan for any non-NaN column, with
 * ceil(log2(N - k)) dependent compare/select levels instead of N - k - 1.
 * best, pv, p: magnitude, signed value and row of the pivot. */
template <int N, int k>
__device__ __forceinline__ void thread_pivot_tree(const double (&a)[N][N], double &best, double &pv,
                                                  int &p)
{
    constexpr int M = N - k;
    double mg[M], vl[M];
    int id[M];
    static_for<0, M>(LUPP_SF(ic) {
        constexpr int i = decltype(ic)::value;
        mg[i] = fabs(a[k][k + i]);
        vl[i] = a[k][k + i];
        id[i] = k + i;
    });
    static_for<0, 6>(LUPP_SF(lc) {
        constexpr int st = 1 << decltype(lc)::value;
        if constexpr (st < M) {
            static_for<0, (M + 2 * st - 1) / (2 * st)>(LUPP_SF(pc) {
                constexpr int i = decltype(pc)::value * 2 * st;
                if constexpr (i + st < M) {
                    const bool gt = mg[i + st] > mg[i];
                    mg[i] = gt ? mg[i + st] : mg[i];
                    vl[i] = gt ? vl[i + st] : vl[i];
                    id[i] = gt ? id[i + st] : id[i];
                }
            });
        }
    });
    best = mg[0];
    pv = vl[0];
    p = id[0];
}

/* Pivoting rule (all solvers): textbook partial pivoting unless the kTile
 * parameter is set (then tile >= 1 is required): tile-local pivoting, where
 * the candidates at step k are first the rows k .. pivot_tile_end - 1, and
 * only if the best of them has magnitude below `thresh` are all rows
 * k .. n-1 searched; ties go to the lowest row (position) either way.
 * Without kTile the solvers contain no tile code at all.
 *
 * Search shape (thread solver): a running left-to-right scan where the
 * factors are kept (fewer values live: n = 8 stays free of scratch at three
 * waves per SIMD), a pairwise tree for solve-only calls such as the Newton
 * steps (a dependent chain of ceil(log2(n - k)) compare/selects instead of
 * n - k - 1). Both pick the same row unless the column holds a NaN.
 *
 * Interchange: the pivot row p is data while register indices are not, so
 * rows k and p are swapped by selects, one candidate row i at a time, and
 * the swap with row i runs only if some lane of the wave chose it (a
 * wave-uniform branch on a ballot). A wave whose systems pivot alike - the
 * Jacobians of one law at neighbouring points, which nearly always pivot on
 * row k or the flow-rule row - skips most of the selects; for unrelated
 * random systems every row is some lane's pivot, and the branches still
 * bound how far the compiler interleaves the swaps: measured on gfx950 this
 * form needs far fewer registers than selecting the pivot row out of all
 * candidates column by column (n = 8: 170 VGPRs against 256 plus scratch;
 * n = 13: no scratch against 1204 bytes per lane).
 *
 * kRecip (solve only, kFactors false): one division per step - the pivot's
 * reciprocal - by which the multipliers are formed and, stored in the
 * pivot's place, the back substitution multiplies: 13 divisions instead of
 * 91 at n = 13. The rounding differs from the true divisions of the default
 * (and of the oracle). */
template <int N, bool kFactors, bool kFMA = false, bool kTile = false, bool kRecip = false>
__device__ __forceinline__ int thread_getrf_solve(double (&a)[N][N], double (&b)[N],
                                                  int (&ipiv)[N], int tile = 0,
                                                  double thresh = 0.0)
{
    static_assert(!(kRecip && kFactors), "the reciprocal form overwrites the pivots");
    int info = 0;
    static_for<0, N>(LUPP_SF(kc) {
        constexpr int k = decltype(kc)::value;
        /* pivot search over rows k .. k1-1 of column k, then, if needed, over
         * every row k .. N-1 */
        const int k1 = kTile ? pivot_tile_end(k, N, tile) : N;
        double best = fabs(a[k][k]);
        double pv = a[k][k];
        int p = k;
        if constexpr (!kTile && !kFactors) {
            thread_pivot_tree<N, k>(a, best, pv, p);
        } else {
            static_for<k + 1, N>(LUPP_SF(ic) {
                constexpr int i = decltype(ic)::value;
                const double v = fabs(a[k][i]);
                bool gt = v > best;
                if constexpr (kTile) gt = gt & (i < k1);
                best = gt ? v : best;
                pv = gt ? a[k][i] : pv;
                p = gt ? i : p;
            });
        }
        if (kTile && __ballot(best < thresh) != 0) {
            const bool wide = best < thresh;
            double bw = fabs(a[k][k]);
            double pw = a[k][k];
            int qw = k;
            static_for<k + 1, N>(LUPP_SF(ic) {
                constexpr int i = decltype(ic)::value;
                const double v = fabs(a[k][i]);
                const bool gt = v > bw;
                bw = gt ? v : bw;
                pw = gt ? a[k][i] : pw;
                qw = gt ? i : qw;
            });
            best = wide ? bw : best;
            pv = wide ? pw : pv;
            p = wide ? qw : p;
        }
        ipiv[k] = p + 1;
        const bool zero = (pv == 0.0);
        info = (zero && info == 0) ? k + 1 : info;
        /* solve-only calls on systems that spill into AGPRs (the 13 x 13
         * Newton steps): fenced, see settle - 190 -> 146 AGPRs, no VGPR
         * spill, 2991 -> 2891 us; at 7 x 7 it removes registers without
         * adding a wave (641 vs 632 us) */
        if constexpr (!kFactors && N >= 10) settle(info);
        /* kRecip: the reciprocal needs only the pivot value, so its latency
         * runs under the interchange below (a zero pivot gives an unused
         * infinity) */
        const double rp = kRecip ? 1.0 / pv : 0.0;

        /* interchange rows k and p: exactly one candidate i matches p in a
         * lane, so the conditional swaps compose to the single interchange */
        static_for<k + 1, N>(LUPP_SF(ic) {
            constexpr int i = decltype(ic)::value;
            const bool hit = (p == i);
            if (__ballot(hit) != 0) {
                static_for<(kFactors ? 0 : k), N>(LUPP_SF(jc) {
                    constexpr int j = decltype(jc)::value;
                    const double rk = a[j][k], ri = a[j][i];
                    a[j][k] = hit ? ri : rk;
                    a[j][i] = hit ? rk : ri;
                });
                const double bk = b[k], bi = b[i];
                b[k] = hit ? bi : bk;
                b[i] = hit ? bk : bi;
            }
        });

        if (!zero) {
            /* multipliers, Schur-complement update, forward substitution */
            if constexpr (kRecip) {
                /* one division per step: the multipliers take the pivot's
                 * reciprocal, which then replaces the pivot for the back
                 * substitution */
                static_for<k + 1, N>(LUPP_SF(ic) {
                    constexpr int i = decltype(ic)::value;
                    a[k][i] = a[k][i] * rp;
                });
                a[k][k] = rp;
            } else {
                static_for<k + 1, N>(LUPP_SF(ic) {
                    constexpr int i = decltype(ic)::value;
                    a[k][i] = a[k][i] / pv;
                });
            }
            static_for<k + 1, N>(LUPP_SF(jc) {
                constexpr int j = decltype(jc)::value;
                static_for<k + 1, N>(LUPP_SF(ic) {
                    constexpr int i = decltype(ic)::value;
                    a[j][i] = msub<kFMA>(a[j][i], a[k][i], a[j][k]);
                });
            });
            static_for<k + 1, N>(LUPP_SF(ic) {
                constexpr int i = decltype(ic)::value;
                b[i] = msub<kFMA>(b[i], a[k][i], b[k]);
            });
        }
    });
    if (info == 0) {
        static_for_down<0, N>(LUPP_SF(jc) {
            constexpr int j = decltype(jc)::value;
            if constexpr (kRecip) b[j] = b[j] * a[j][j];
            else b[j] = b[j] / a[j][j];
            static_for<0, j>(LUPP_SF(ic) {
                constexpr int i = decltype(ic)::value;
                b[i] = msub<kFMA>(b[i], a[j][i], b[j]);
            });
        });
    }
    return info;
}

/* Row permutation of a LAPACK interchange sequence (1-based ipiv): row i of
 * P A is row perm[i] of A. */
template <int N>
__device__ __forceinline__ void thread_ipiv_to_perm(const int (&ipiv)[N], int (&perm)[N])
{
    static_for<0, N>(LUPP_SF(ic) { perm[decltype(ic)::value] = decltype(ic)::value; });
    static_for<0, N>(LUPP_SF(kc) {
        constexpr int k = decltype(kc)::value;
        const int p = ipiv[k] - 1;
        int vp = perm[k];
        static_for<k + 1, N>(LUPP_SF(ic) {
            constexpr int i = decltype(ic)::value;
            vp = (p == i) ? perm[i] : vp;
        });
        const int vk = perm[k];
        static_for<k + 1, N>(LUPP_SF(ic) {
            constexpr int i = decltype(ic)::value;
            perm[i] = (p == i) ? vk : perm[i];
        });
        perm[k] = vp;
    });
}

/* x = A^-1 e_c from the LAPACK-ordered factors lu[j][i] (element (i, j)) of
 * thread_getrf_solve<N, true> and the row permutation of its ipiv: P e_c,
 * then forward substitution with the unit lower factor (column-oriented,
 * ascending) and back substitution with the upper one (divide, then
 * eliminate the column above, descending) - the operation order of the
 * one-right-hand-side solve. Used for multi-right-hand-side solves with unit
 * vectors, such as a consistent tangent operator. */
template <int N, bool kFMA = false>
__device__ __forceinline__ void thread_solve_unit(const double (&lu)[N][N], const int (&perm)[N],
                                                  int c, double (&x)[N])
{
    static_for<0, N>(LUPP_SF(ic) {
        constexpr int i = decltype(ic)::value;
        x[i] = (perm[i] == c) ? 1.0 : 0.0;
    });
    static_for<0, N>(LUPP_SF(jc) {
        constexpr int j = decltype(jc)::value;
        static_for<j + 1, N>(LUPP_SF(ic) {
            constexpr int i = decltype(ic)::value;
            x[i] = msub<kFMA>(x[i], lu[j][i], x[j]);
        });
    });
    static_for_down<0, N>(LUPP_SF(jc) {
        constexpr int j = decltype(jc)::value;
        x[j] = x[j] / lu[j][j];
        static_for<0, j>(LUPP_SF(ic) {
            constexpr int i = decltype(ic)::value;
            x[i] = msub<kFMA>(x[i], lu[j][i], x[j]);
        });
    });
}

/* Solve-only convenience entry: the device-callable solve of one system held
 * by the calling thread (a is destroyed). Returns info. */
template <int N>
__device__ __forceinline__ int lupp_solve_n(double (&a)[N][N], double (&b)[N], int (&ipiv)[N])
{
    return thread_getrf_solve<N, false>(a, b, ipiv);
}

/* ------------------------------------------------------------------------ */
/* Lanes-per-system solver: T consecutive lanes of a wave64 (a "segment",    */
/* T a power of two <= 32) cooperate on one system. Lane t owns rows         */
/* r = t + s*T for slots s = 0..K-1 (round robin, K = ceil(N/T)); a slot     */
/* with r >= N is a phantom row that takes no part. Rows never move          */
/* (logical pivoting): pos[s] is the row's current position in LAPACK's      */
/* interchange order, so the candidates at step k are the rows with          */
/* pos >= k and ties go to the lowest position. The pivot search is a        */
/* butterfly reduction inside the segment; the pivot row is broadcast with   */
/* ds_bpermute.                                                              */
/* ------------------------------------------------------------------------ */
template <int N, int T>
struct lanes_shape {
    static_assert(T == 1 || T == 2 || T == 4 || T == 8 || T == 16 || T == 32, "T");
    static constexpr int K = (N + T - 1) / T;
};

__device__ __forceinline__ double bcast_f64(double v, int src_lane)
{
    const int addr = src_lane << 2;
    const int2 w = __builtin_bit_cast(int2, v);
    int2 r;
    r.x = __builtin_amdgcn_ds_bpermute(addr, w.x);
    r.y = __builtin_amdgcn_ds_bpermute(addr, w.y);
    return __builtin_bit_cast(double, r);
}

__device__ __forceinline__ int bcast_i32(int v, int src_lane)
{
    return __builtin_amdgcn_ds_bpermute(src_lane << 2, v);
}

/* Butterfly exchange inside aligned groups of 2^(L+1) lanes, all on the VALU:
 * L = 0, 1: quad permutes (lane ^ 1, lane ^ 2); L = 2: mirror inside 8 lanes;
 * L = 3: mirror inside 16 lanes; L = 4: rows of 16 exchanged in pairs.
 * Each lane receives the value of a partner in the other half of its group;
 * the callers combine own and partner values with a commutative operation, so
 * after levels 0..L every lane of a group holds the group's result. */
template <int L>
__device__ __forceinline__ void pair_u32(unsigned v, unsigned &a, unsigned &b)
{
    /* every lane has a valid source lane in these patterns, so the plain DPP
     * move (no "old" operand to initialise) is enough */
    if constexpr (L == 0) { a = v; b = __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false); }
    else if constexpr (L == 1) { a = v; b = __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false); }
    else if constexpr (L == 2) { a = v; b = __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false); }
    else if constexpr (L == 3) { a = v; b = __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, false); }
    else {
        /* {a, b} = {own, partner} in some order */
        auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        a = r[0];
        b = r[1];
    }
}

template <int L>
__device__ __forceinline__ double max_round(double v)
{
    const uint2 w = __builtin_bit_cast(uint2, v);
    uint2 a, b;
    pair_u32<L>(w.x, a.x, b.x);
    pair_u32<L>(w.y, a.y, b.y);
    return fmax(__builtin_bit_cast(double, a), __builtin_bit_cast(double, b));
}

template <int L>
__device__ __forceinline__ int min_round(int v)
{
    unsigned a, b;
    pair_u32<L>((unsigned)v, a, b);
    return min((int)a, (int)b);
}

/* Maximum of v over the T lanes of a segment (v >= -1, no NaN). */
template <int T>
__device__ __forceinline__ double segment_max(double v)
{
    if constexpr (T > 1) v = max_round<0>(v);
    if constexpr (T > 2) v = max_round<1>(v);
    if constexpr (T > 4) v = max_round<2>(v);
    if constexpr (T > 8) v = max_round<3>(v);
    if constexpr (T > 16) v = max_round<4>(v);
    return v;
}

template <int T>
__device__ __forceinline__ int segment_min(int v)
{
    if constexpr (T > 1) v = min_round<0>(v);
    if constexpr (T > 2) v = min_round<1>(v);
    if constexpr (T > 4) v = min_round<2>(v);
    if constexpr (T > 8) v = min_round<3>(v);
    if constexpr (T > 16) v = min_round<4>(v);
    return v;
}

/* Pivot search of step k inside a segment: the segment maximum M of |a_rk|
 * over candidate rows (pos >= k) is found with a VALU butterfly; a ballot of
 * the lanes holding it gives the owner directly, and only when two lanes of
 * some segment hold the same maximum (a tie, rare for non-integer data) does
 * a second reduction pick the lowest position. Returns the owner's lane
 * within the segment; lpos / ls are this lane's best candidate position and
 * slot (meaningful in the owner). */
template <int N, int T, int k, bool kTile>
__device__ __forceinline__ int lanes_pivot_owner(const double (&a)[(N + T - 1) / T][N],
                                                 const int (&pos)[(N + T - 1) / T], int seg_base,
                                                 double &M, int &lpos, int &ls, int tile,
                                                 double thresh)
{
    constexpr int K = lanes_shape<N, T>::K;
    const unsigned lowmask = T >= 32 ? 0xffffffffu : ((1u << (T & 31)) - 1u);
    /* local candidate: largest |a_rk| among rows with k <= pos < k1, lowest
     * pos on ties; k1 = N unless the pivoting is tile-local */
    /* in_tile: candidates also need pos < hi (tile-local pivoting); without
     * it every row with pos >= k is a candidate */
    auto local_best = [&](auto in_tile, int hi, double &mag, int &lp, int &sl)
                          __attribute__((always_inline)) {
        mag = -1.0;
        lp = 0x7fffffff;
        sl = 0;
        static_for<0, K>(LUPP_SF(sc) {
            constexpr int s = decltype(sc)::value;
            const double v = fabs(a[s][k]);
            bool cand = pos[s] >= k;
            if constexpr (decltype(in_tile)::value) cand = cand & (pos[s] < hi);
            /* non-short-circuit logic: selects, not branches */
            const bool take = cand & ((v > mag) | ((v == mag) & (pos[s] < lp)));
            mag = take ? v : mag;
            lp = take ? pos[s] : lp;
            sl = take ? s : sl;
        });
    };
    double mag;
    if constexpr (kTile)
        local_best(std::true_type{}, pivot_tile_end(k, N, tile), mag, lpos, ls);
    else
        local_best(std::false_type{}, N, mag, lpos, ls);
    M = segment_max<T>(mag);
    if (kTile && __ballot(M < thresh) != 0) {
        /* tile-local pivoting: segments whose in-tile best is below the
         * threshold search every remaining row */
        const bool wide = M < thresh;
        double mw;
        int lw, sw;
        local_best(std::false_type{}, N, mw, lw, sw);
        const double Mw = segment_max<T>(mw);
        mag = wide ? mw : mag;
        lpos = wide ? lw : lpos;
        ls = wide ? sw : ls;
        M = wide ? Mw : M;
    }
    const uint64_t hits = __ballot(mag == M);
    const unsigned sb = (unsigned)(hits >> (unsigned)seg_base) & lowmask;
    /* sb != 0 for finite data; lane 0 keeps the owner inside the segment
     * otherwise (NaN entries, outside the solver's contract) */
    int tp = sb ? (int)__builtin_ctz(sb) : 0;
    if (__ballot(__builtin_popcount(sb) > 1) != 0) {
        /* a tie between lanes in some segment: lowest position wins */
        const int pmin = segment_min<T>(mag == M ? lpos : 0x7fffffff);
        const unsigned s2 =
            (unsigned)(__ballot(mag == M && lpos == pmin) >> (unsigned)seg_base) & lowmask;
        tp = s2 ? (int)__builtin_ctz(s2) : tp;
    }
    /* a lane without candidate (only with NaN entries) reports the last row */
    lpos = lpos < N ? lpos : N - 1;
    return tp;
}

/* Back substitution, column j descending: x_j lives in the row at position j;
 * its owner divides, broadcasts x_j, and the rows above eliminate it. Every
 * lane of the segment sees every x_j: x_sink(j, x_j) is called by all lanes
 * (a solver whose callers need the whole solution in every lane gets it
 * without further communication). */
template <int N, int T, bool kFMA, bool kRecip, typename XSink>
__device__ __forceinline__ void lanes_back_subst(const double (&a)[(N + T - 1) / T][N],
                                                 double (&b)[(N + T - 1) / T],
                                                 const int (&pos)[(N + T - 1) / T], int seg_base,
                                                 XSink x_sink)
{
    constexpr int K = lanes_shape<N, T>::K;
    const unsigned lowmask = T >= 32 ? 0xffffffffu : ((1u << (T & 31)) - 1u);
    static_for_down<0, N>(LUPP_SF(jc) {
        constexpr int j = decltype(jc)::value;
        bool mine = false;
        double bs = 0.0, us = 1.0;
        static_for<0, K>(LUPP_SF(sc) {
            constexpr int s = decltype(sc)::value;
            const bool hit = pos[s] == j;
            mine = mine || hit;
            bs = hit ? b[s] : bs;
            us = hit ? a[s][j] : us;
        });
        /* kRecip: the row holds the pivot's reciprocal in place of u_jj */
        const double xl = kRecip ? bs * us : bs / us;
        const unsigned ob = (unsigned)(__ballot(mine) >> (unsigned)seg_base) & lowmask;
        const int owner = seg_base + (int)__builtin_ctz(ob | (1u << 31));
        const double x = bcast_f64(xl, owner);
        x_sink(j, x);
        static_for<0, K>(LUPP_SF(sc) {
            constexpr int s = decltype(sc)::value;
            if (pos[s] == j) b[s] = x;
            else if (pos[s] >= 0 && pos[s] < j) b[s] = msub<kFMA>(b[s], a[s][j], x);
        });
    });
}

/* Factor (and solve, on info == 0) the system owned by this segment.
 * a[s][j]: row t+s*T, column j; b[s]: its right-hand side entry; pos[s] must
 * be initialised to the row index (or -1 for a phantom row). On return
 * pos[s] is the row's final position: the factors/solution entry held in
 * slot s belong to row pos[s] of the LAPACK-ordered result. seg_base is the
 * wave lane of the segment's lane 0. ipiv_k(k, v) is called by every lane
 * with the segment-uniform interchange ipiv[k] = v (1-based).
 *
 * The pivot row reaches the other lanes of the segment by ds_bpermute, and
 * the trailing update runs under the exec mask of the trailing rows
 * (pos > k). No LDS allocation is needed. lanes_getrf_solve_x also calls
 * x_sink(j, x_j) in every lane for every solution entry; tile / thresh
 * select the pivoting rule (see thread_getrf_solve). CH is the number of
 * pivot-row columns broadcast (and held in registers) at a time within a
 * step: larger chunks expose more independent broadcasts per wait at the
 * cost of 2*CH VGPRs. Results do not depend on it. kRecip: one division per
 * step (the pivot's reciprocal, by which the multipliers are formed and the
 * back substitution multiplies) instead of one per multiplier, as
 * thread_getrf_solve with kRecip; the factors are then not LAPACK's. */
template <int N, int T, bool kFMA = false, bool kTile = false, int CH = 8, bool kRecip = false,
          bool kSettle = false, typename IpivSink, typename XSink>
__device__ __forceinline__ int lanes_getrf_solve_x(double (&a)[(N + T - 1) / T][N],
                                                   double (&b)[(N + T - 1) / T],
                                                   int (&pos)[(N + T - 1) / T], int seg_base,
                                                   IpivSink ipiv_k, XSink x_sink, int tile = 0,
                                                   double thresh = 0.0)
{
    constexpr int K = lanes_shape<N, T>::K;
    static_assert(CH >= 1, "CH: pivot-row columns broadcast per chunk");
    const int lane_in_seg = (int)__lane_id() - seg_base;
    int info = 0;
    static_for<0, N>(LUPP_SF(kc) {
        constexpr int k = decltype(kc)::value;
        double M;
        int lpos, ls;
        const int tp =
            lanes_pivot_owner<N, T, k, kTile>(a, pos, seg_base, M, lpos, ls, tile, thresh);
        const int src = seg_base + tp;
        /* Every lane reads its own best candidate slot (ls); the owner's
         * slot is the pivot row, so broadcasting from the owner needs no
         * earlier exchange of the slot index: the pivot value and the row go
         * out right after the reduction, and the pivot's position q (for the
         * bookkeeping and ipiv) travels beside them, off the critical path. */
        double sel = a[0][k];
        static_for<1, K>(LUPP_SF(sc) {
            constexpr int s = decltype(sc)::value;
            sel = (ls == s) ? a[s][k] : sel;
        });
        const double pv = bcast_f64(sel, src);
        const int q = bcast_i32(lpos, src); /* current position of the pivot row */
        ipiv_k(k, q + 1);

        /* trailing rows: every candidate row except the pivot row (the row at
         * position k, if it is not the pivot, moves to q > k) */
        const bool own = lane_in_seg == tp;
        bool trail[K];
        static_for<0, K>(LUPP_SF(sc) {
            constexpr int s = decltype(sc)::value;
            const bool piv = own && ls == s;
            trail[s] = !piv && pos[s] >= k;
            /* positions: the row at position k moves to q, the pivot row takes k */
            const int ps = pos[s];
            pos[s] = piv ? k : ((ps == k) ? q : ps);
        });
        const bool zero = (M == 0.0);
        info = (zero && info == 0) ? k + 1 : info;
        if constexpr (kSettle) settle(info);

        if (!zero) {
            double l[K];
            if constexpr (kRecip) {
                const double r = 1.0 / pv;
                static_for<0, K>(LUPP_SF(sc) {
                    constexpr int s = decltype(sc)::value;
                    l[s] = a[s][k] * r;
                    a[s][k] = trail[s] ? l[s] : ((own && ls == s) ? r : a[s][k]);
                    if constexpr (kSettle) settle(a[s][k]);
                });
            } else {
                static_for<0, K>(LUPP_SF(sc) {
                    constexpr int s = decltype(sc)::value;
                    l[s] = a[s][k] / pv;
                    a[s][k] = trail[s] ? l[s] : a[s][k];
                    if constexpr (kSettle) settle(a[s][k]);
                });
            }
            double ys = b[0];
            static_for<1, K>(LUPP_SF(sc) {
                constexpr int s = decltype(sc)::value;
                ys = (ls == s) ? b[s] : ys;
            });
            const double y = bcast_f64(ys, src);
            static_for<0, (N - k - 1 + CH - 1) / CH>(LUPP_SF(cc) {
                constexpr int j0 = k + 1 + decltype(cc)::value * CH;
                constexpr int j1 = (j0 + CH < N) ? j0 + CH : N;
                double u[CH];
                static_for<j0, j1>(LUPP_SF(jc) {
                    constexpr int j = decltype(jc)::value;
                    double us = a[0][j];
                    static_for<1, K>(LUPP_SF(sc) {
                        constexpr int s = decltype(sc)::value;
                        us = (ls == s) ? a[s][j] : us;
                    });
                    u[j - j0] = bcast_f64(us, src);
                });
                static_for<0, K>(LUPP_SF(sc) {
                    constexpr int s = decltype(sc)::value;
                    if (trail[s]) {
                        static_for<j0, j1>(LUPP_SF(jc) {
                            constexpr int j = decltype(jc)::value;
                            a[s][j] = msub<kFMA>(a[s][j], l[s], u[j - j0]);
                        });
                        if constexpr (decltype(cc)::value == 0) b[s] = msub<kFMA>(b[s], l[s], y);
                    }
                });
            });
            if constexpr (k + 1 >= N) {
                static_for<0, K>(LUPP_SF(sc) {
                    constexpr int s = decltype(sc)::value;
                    if (trail[s]) b[s] = msub<kFMA>(b[s], l[s], y);
                });
            }
        }
    });
    if (info == 0) lanes_back_subst<N, T, kFMA, kRecip>(a, b, pos, seg_base, x_sink);
    return info;
}

template <int N, int T, bool kFMA = false, bool kTile = false, int CH = 8, bool kSettle = false,
          typename IpivSink>
__device__ __forceinline__ int lanes_getrf_solve(double (&a)[(N + T - 1) / T][N],
                                                 double (&b)[(N + T - 1) / T],
                                                 int (&pos)[(N + T - 1) / T], int seg_base,
                                                 IpivSink ipiv_k, int tile = 0, double thresh = 0.0)
{
    return lanes_getrf_solve_x<N, T, kFMA, kTile, CH, false, kSettle>(a, b, pos, seg_base, ipiv_k,
                                                      [](int, double) {}, tile, thresh);
}

}  // namespace lupp

#endif
