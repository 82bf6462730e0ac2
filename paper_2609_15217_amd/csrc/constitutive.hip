/* Fused per-point Newton constitutive update (Section 2.1, equations 1-3;
 * Section 3.3 and Algorithm 2: the whole Newton loop of every integration
 * point runs inside one kernel and calls the device-callable LU solver, so
 * nothing goes back to the host between iterations). The laws are in law.h.
 *
 * One lane per integration point; points are stored component-major (SoA):
 * component c of point p at ptr[c*ld + p].
 */
#include "law.h"

namespace lupp {

template <int NU, bool TAN>
__global__ void __launch_bounds__(256) k_newton(lupp_points pts, LawK P, double tol, int maxit)
{
    constexpr bool kTangent = TAN;
    const int64_t p0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x;
    const int64_t rem = pts.count - p0;
    const uint32_t nvalid = (uint32_t)(rem < (int64_t)blockDim.x ? rem : blockDim.x);
    const uint32_t tid = threadIdx.x;
    const uint32_t nb = nvalid * 8u, vo = tid * 8u;

    double de[6], st[NU], y[NU], F[NU], sig[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) de[c] = buf_load_f64(make_rsrc(pts.deps + c * pts.ld + p0, nb), vo, 0);
#pragma unroll
    for (int c = 0; c < NU; ++c) {
        st[c] = buf_load_f64(make_rsrc(pts.state + c * pts.ld + p0, nb), vo, 0);
        y[c] = 0.0;
    }

    int status = 1, it = 0;
    for (;; ++it) {
        double J[NU][NU];
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
        if (thread_getrf_solve<NU, false>(J, dx, piv) != 0) { status = 2; break; }
#pragma unroll
        for (int i = 0; i < NU; ++i) y[i] = y[i] + dx[i];
    }

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

int constitutive_launch(const lupp_points *pts, const lupp_law *law, double tol, int maxit,
                        hipStream_t stream)
{
    const LawK P = law_constants(law);
    const int threads = 256;
    const int64_t blocks = (pts->count + threads - 1) / threads;
    const bool tan = pts->tangent != nullptr;
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
