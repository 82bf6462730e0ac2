/* Fused per-point Newton constitutive update (Section 2.1, equations 1-3;
 * Section 3.3 and Algorithm 2: the whole Newton loop of every integration
 * point runs inside one kernel and calls the device-callable LU solver, so
 * nothing goes back to the host between iterations). The laws are in law.h.
 *
 * One lane per integration point; points are stored component-major (SoA):
 * component c of point p at ptr[c*ld + p].
 */
#include "law.h"
#include "serving.h"

namespace lupp {

/* One workgroup of 256 points, the first at p0: the whole Newton loop of
 * every point, then its stress, state (on convergence), iterations, status
 * and optionally its tangent. */
template <int NU, bool TAN>
__device__ __forceinline__ void newton_block(const lupp_points &pts, const LawK &P, double tol,
                                             int maxit, int64_t p0)
{
    constexpr bool kTangent = TAN;
    const int64_t rem = pts.count - p0;
    const uint32_t nvalid = (uint32_t)(rem < (int64_t)blockDim.x ? rem : blockDim.x);
    const uint32_t tid = threadIdx.x;
    const uint32_t nb = nvalid * 8u, vo = tid * 8u;
    /* The strain increment, the state at the start of the step and the
     * unknowns live in LDS, one column of 256 doubles per component (each
     * lane reads its own entries: no bank conflicts, no barrier), and are
     * read at the start of every iteration: the registers stay free for the
     * Jacobian and its factorisation (13 unknowns: 169 doubles). */
    __shared__ double sh[(6 + 2 * NU) * 256];
    auto DE = [&](int c) -> double & { return sh[c * 256 + tid]; };
    auto ST = [&](int c) -> double & { return sh[(6 + c) * 256 + tid]; };
    auto Y = [&](int c) -> double & { return sh[(6 + NU + c) * 256 + tid]; };
#pragma unroll
    for (int c = 0; c < 6; ++c) DE(c) = buf_load_f64(make_rsrc(pts.deps + c * pts.ld + p0, nb), vo, 0);
#pragma unroll
    for (int c = 0; c < NU; ++c) {
        ST(c) = buf_load_f64(make_rsrc(pts.state + c * pts.ld + p0, nb), vo, 0);
        Y(c) = 0.0;
    }
    auto read_inputs = [&](double (&de)[6], double (&st)[NU], double (&y)[NU])
                           __attribute__((always_inline)) {
#pragma unroll
        for (int c = 0; c < 6; ++c) de[c] = DE(c);
#pragma unroll
        for (int c = 0; c < NU; ++c) {
            st[c] = ST(c);
            y[c] = Y(c);
        }
    };

    int status = 1, it = 0;
    for (;; ++it) {
        /* keeps the reads inside the loop (no hoisting into registers) */
        asm volatile("" ::: "memory");
        double de[6], st[NU], y[NU], F[NU], sig[6];
        double J[NU][NU];
        read_inputs(de, st, y);
        law_assemble<NU>(P, de, st, y, F, J, sig);
        bool finite = true;
        double nrm = 0.0;
#pragma unroll
        for (int i = 0; i < NU; ++i) {
            finite = finite && __builtin_isfinite(F[i]);
            nrm = fmax(nrm, fabs(F[i]));
        }
        if (!finite) { status = 3; break; }
        if (nrm < tol) { status = 0; break; }
        if (it == maxit) { status = 1; break; }
        double dx[NU];
        int piv[NU];
#pragma unroll
        for (int i = 0; i < NU; ++i) dx[i] = -F[i];
        if (thread_getrf_solve<NU, false, kNewtonFMA, false, kNewtonRecip>(J, dx, piv) != 0) {
            status = 2;
            break;
        }
#pragma unroll
        for (int i = 0; i < NU; ++i) Y(i) = Y(i) + dx[i];
    }

    asm volatile("" ::: "memory");
    double de[6], st[NU], y[NU], sig[6];
    read_inputs(de, st, y);
    law_stress<NU>(P, st, y, sig); /* the stress of the returned iterate */
#pragma unroll
    for (int c = 0; c < 6; ++c) buf_store_f64(make_rsrc(pts.sig + c * pts.ld + p0, nb), vo, 0, sig[c]);
    const uint32_t vs = status == 0 ? vo : kOutOfRange;
#pragma unroll
    for (int c = 0; c < NU; ++c)
        buf_store_f64(make_rsrc(pts.state + c * pts.ld + p0, nb), vs, 0, st[c] + y[c]);
    buf_store_i32(make_rsrc(pts.iters + p0, nvalid * 4u), tid * 4u, 0, it);
    buf_store_i32(make_rsrc(pts.status + p0, nvalid * 4u), tid * 4u, 0, status);

    if constexpr (kTangent) {
        if (status == 0) {
            if constexpr (NU == 7) newton_tangent7(P, de, st, y, pts, p0, nb, vo);
            else newton_tangent13(P, de, st, y, pts, p0, nb, vo);
        }
    }
}

/* Occupancy: 7 unknowns fit 3 waves per SIMD without scratch (146 VGPRs; 4
 * waves would spill 52 bytes per lane); 13 unknowns take the whole register
 * file of one wave (VGPRs and AGPRs) and no scratch. */
template <int NU>
constexpr int newton_waves_per_eu() { return NU == 7 ? 3 : 1; }

template <int NU, bool TAN>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(newton_waves_per_eu<NU>())))
    k_newton(lupp_points pts, LawK P, double tol, int maxit)
{
    newton_block<NU, TAN>(pts, P, tol, maxit, (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x);
}

/* Several point sets of one law in one launch (the serving loop's merged
 * updates): workgroup w takes block w of the concatenated sets, and the
 * set table in the kernel arguments (scalar loads) gives its set. */
constexpr int kMaxNewtonGroups = 24;
struct NewtonGroups {
    int32_t nsets;
    int32_t block0[kMaxNewtonGroups]; /* first workgroup of each set, ascending */
    lupp_points pts[kMaxNewtonGroups];
};

template <int NU, bool TAN>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(newton_waves_per_eu<NU>())))
    k_newton_grouped(NewtonGroups g, LawK P, double tol, int maxit)
{
    const int b = (int)xcd_block(blockIdx.x, gridDim.x);
    int gi = 0;
    for (int k = 1; k < g.nsets; ++k)
        if (b >= g.block0[k]) gi = k;
    gi = __builtin_amdgcn_readfirstlane(gi);
    newton_block<NU, TAN>(g.pts[gi], P, tol, maxit, (int64_t)(b - g.block0[gi]) * blockDim.x);
}

/* Lanes-per-point form of the same fused update (Section 3.2.1 and Section
 * 3.3: a multi-threaded device-callable solver embedded in the law, with the
 * law's work partitioned across the cooperating threads). T lanes of a wave
 * share one point: every lane evaluates the law's common part and the whole
 * residual redundantly (so the stop rules need no communication), builds
 * only the Jacobian rows it owns (rows t, t + T, ...), and the segment solves
 * with the lanes LU, whose back substitution hands every x_j to every lane.
 * The Jacobian entries, the pivots and the operation order are those of the
 * one-lane-per-point kernel, so the results are bitwise the same; the
 * per-lane register footprint is a fraction of the 13 x 13 matrix.
 * The tangent is left to the one-lane-per-point kernel. */
template <int NU, int T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
    k_newton_lanes(lupp_points pts, LawK P, double tol, int maxit)
{
    constexpr int K = (NU + T - 1) / T, SPW = 64 / T;
    const int lane = (int)__lane_id();
    const int g = lane / T, t = lane % T;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t p0 = ((int64_t)xcd_block(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + wave) * SPW;
    const int64_t rem = pts.count - p0;
    const uint32_t nvalid = (uint32_t)(rem <= 0 ? 0 : (rem < SPW ? rem : SPW));
    const uint32_t nb = nvalid * 8u;
    const uint32_t vo = (uint32_t)g < nvalid ? (uint32_t)g * 8u : kOutOfRange;

    double de[6], st[NU], y[NU];
#pragma unroll
    for (int c = 0; c < 6; ++c) de[c] = buf_load_f64(make_rsrc(pts.deps + c * pts.ld + p0, nb), vo, 0);
#pragma unroll
    for (int c = 0; c < NU; ++c) {
        st[c] = buf_load_f64(make_rsrc(pts.state + c * pts.ld + p0, nb), vo, 0);
        y[c] = 0.0;
    }

    LawC<NU> C;
    int status = 1, it = 0;
    for (;; ++it) {
        law_common<NU>(P, de, st, y, C);
        bool finite = true;
        double nrm = 0.0;
#pragma unroll
        for (int i = 0; i < NU; ++i) {
            finite = finite && __builtin_isfinite(C.F[i]);
            nrm = fmax(nrm, fabs(C.F[i]));
        }
        if (!finite) { status = 3; break; }
        if (nrm < tol) { status = 0; break; }
        if (it == maxit) { status = 1; break; }
        double a[K][NU], b[K];
        int pos[K];
        static_for<0, K>(LUPP_SF(sc) {
            constexpr int s = decltype(sc)::value;
            const int r = t + s * T;
            pos[s] = r < NU ? r : -1;
            if (r < NU) {
                law_jac_row<NU>(P, C, r, a[s]);
                b[s] = -select_at<NU>(C.F, r);
            } else {
#pragma unroll
                for (int c = 0; c < NU; ++c) a[s][c] = 0.0;
                b[s] = 0.0;
            }
        });
        /* x += dx as the back substitution hands out each dx_j (a zero pivot
         * skips the substitution, so y is then unchanged) */
        const int inf = lanes_getrf_solve_x<NU, T, kNewtonFMA, false, 8, kNewtonRecip>(
            a, b, pos, g * T, [](int, int) {}, [&](int j, double x) { y[j] = y[j] + x; });
        if (inf != 0) { status = 2; break; }
    }

    /* lane 0 of each segment writes the point's results */
    const uint32_t vw = t == 0 ? vo : kOutOfRange;
#pragma unroll
    for (int c = 0; c < 6; ++c) buf_store_f64(make_rsrc(pts.sig + c * pts.ld + p0, nb), vw, 0, C.sig[c]);
    const uint32_t vs = status == 0 ? vw : kOutOfRange;
#pragma unroll
    for (int c = 0; c < NU; ++c)
        buf_store_f64(make_rsrc(pts.state + c * pts.ld + p0, nb), vs, 0, st[c] + y[c]);
    const uint32_t vi = t == 0 && (uint32_t)g < nvalid ? (uint32_t)g * 4u : kOutOfRange;
    buf_store_i32(make_rsrc(pts.iters + p0, nvalid * 4u), vi, 0, it);
    buf_store_i32(make_rsrc(pts.status + p0, nvalid * 4u), vi, 0, status);
}

template <int NU, int T>
static void launch_newton_lanes(const lupp_points *pts, const LawK &P, double tol, int maxit,
                                hipStream_t stream)
{
    constexpr int per_block = 4 * (64 / T); /* 4 waves */
    const int64_t blocks = (pts->count + per_block - 1) / per_block;
    hipLaunchKernelGGL((k_newton_lanes<NU, T>), dim3((unsigned)blocks), dim3(256), 0, stream, *pts, P,
                       tol, maxit);
}

/* Default mapping per law, measured on gfx950 (2^20 points of the benchmark
 * increments, mean 17.7 solves per point): one lane per point wins for both
 * laws - 7 unknowns: 1.33 ms against 4.5 ms (4 lanes) and 6.6 ms (8 lanes);
 * 13 unknowns: 7.6 ms, despite 512 VGPRs with some scratch and one wave per
 * SIMD, against 17.9 ms (8 lanes) and 23 ms (16 lanes, 247 VGPRs, two
 * waves). Every lane of a group repeats the law's common part (pow, sqrt,
 * divisions), and the lanes LU's pivot search and broadcasts cost more than
 * the occupancy they buy back. */
int newton_default_lanes(int) { return 1; }

bool newton_lanes_supported(int kind, int lanes)
{
    if (lanes == 1) return true;
    if (kind == LUPP_LAW_NORTON7) return lanes == 4 || lanes == 8;
    if (kind == LUPP_LAW_NORTON_AF13) return lanes == 8 || lanes == 16;
    return false;
}

int constitutive_launch(const lupp_points *pts, const lupp_law *law, double tol, int maxit,
                        int lanes, hipStream_t stream)
{
    const LawK P = law_constants(law);
    const bool tan = pts->tangent != nullptr;
    if (!tan && lanes > 1) {
        if (law->kind == LUPP_LAW_NORTON7) {
            if (lanes == 4) launch_newton_lanes<7, 4>(pts, P, tol, maxit, stream);
            else launch_newton_lanes<7, 8>(pts, P, tol, maxit, stream);
        } else {
            if (lanes == 8) launch_newton_lanes<13, 8>(pts, P, tol, maxit, stream);
            else launch_newton_lanes<13, 16>(pts, P, tol, maxit, stream);
        }
        return hip_err(hipGetLastError());
    }
    const int threads = 256;
    const int64_t blocks = (pts->count + threads - 1) / threads;
    const dim3 g((unsigned)blocks), b(threads);
    if (law->kind == LUPP_LAW_NORTON7) {
        if (tan) hipLaunchKernelGGL((k_newton<7, true>), g, b, 0, stream, *pts, P, tol, maxit);
        else hipLaunchKernelGGL((k_newton<7, false>), g, b, 0, stream, *pts, P, tol, maxit);
    } else {
        if (tan) hipLaunchKernelGGL((k_newton<13, true>), g, b, 0, stream, *pts, P, tol, maxit);
        else hipLaunchKernelGGL((k_newton<13, false>), g, b, 0, stream, *pts, P, tol, maxit);
    }
    return hip_err(hipGetLastError());
}

int constitutive_launch_grouped(const lupp_points *sets, int nsets, const lupp_law *law,
                                double tol, int maxit, hipStream_t stream)
{
    const LawK P = law_constants(law);
    const bool tan = nsets > 0 && sets[0].tangent != nullptr;
    for (int i0 = 0; i0 < nsets; i0 += kMaxNewtonGroups) {
        NewtonGroups g{};
        int64_t blocks = 0;
        for (int i = i0; i < nsets && g.nsets < kMaxNewtonGroups; ++i) {
            if (sets[i].count <= 0) continue;
            g.block0[g.nsets] = (int32_t)blocks;
            g.pts[g.nsets] = sets[i];
            ++g.nsets;
            blocks += (sets[i].count + 255) / 256;
        }
        if (g.nsets == 0) continue;
        const dim3 grid((unsigned)blocks), blk(256);
        if (law->kind == LUPP_LAW_NORTON7) {
            if (tan) hipLaunchKernelGGL((k_newton_grouped<7, true>), grid, blk, 0, stream, g, P, tol, maxit);
            else hipLaunchKernelGGL((k_newton_grouped<7, false>), grid, blk, 0, stream, g, P, tol, maxit);
        } else {
            if (tan) hipLaunchKernelGGL((k_newton_grouped<13, true>), grid, blk, 0, stream, g, P, tol, maxit);
            else hipLaunchKernelGGL((k_newton_grouped<13, false>), grid, blk, 0, stream, g, P, tol, maxit);
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_err(e);
    }
    return 0;
}

const void *constitutive_kernel_symbol(int kind, bool tangent)
{
    if (kind == LUPP_LAW_NORTON7)
        return tangent ? reinterpret_cast<const void *>(&k_newton<7, true>)
                       : reinterpret_cast<const void *>(&k_newton<7, false>);
    if (kind == LUPP_LAW_NORTON_AF13)
        return tangent ? reinterpret_cast<const void *>(&k_newton<13, true>)
                       : reinterpret_cast<const void *>(&k_newton<13, false>);
    return nullptr;
}

}  // namespace lupp
