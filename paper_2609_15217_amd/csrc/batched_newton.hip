/* CPU-driven batched Newton constitutive update (Algorithm 1; Section 2.5):
 * every Newton iteration is three launches - assemble F and J for all points,
 * one batched LU solve of all the Jacobians, update the unknowns and apply the
 * stop rules - and the host reads one counter after each iteration to decide
 * whether to go on. The batched solve is the library's register-resident
 * thread solver over the interleaved Jacobians, in the Newton arithmetic of
 * law.h (the standalone batched solve has no reciprocal-pivot mode). Points
 * that have finished are carried through the remaining batched solves (the
 * batched paradigm's dragging, Section 2.5) but no longer change, so every
 * point follows exactly the iteration sequence of the fused kernel and the
 * results are bitwise those of constitutive_update.
 *
 * Workspace (owned by the context, grown on demand), all interleaved (SoA,
 * point index fastest) so that every kernel's accesses are coalesced:
 * unknowns y [NU][count], Jacobians [NU*NU][count] (element (r, c) at row
 * r + c*NU), right-hand sides [NU][count], info, per-point state and the
 * active-point counter.
 */
#include "law.h"

namespace lupp {

struct BnArgs {
    int64_t count;
    double *y;        /* [NU][count] */
    double *J;        /* [NU*NU][count] */
    double *rhs;      /* [NU][count] */
    int32_t *info;    /* [count] */
    int32_t *st;      /* [count] -1 while iterating, else the final status */
    int32_t *it;      /* [count] linear solves done */
    int32_t *active;  /* points still iterating after this iteration's assembly */
};

__global__ void __launch_bounds__(256) k_bn_init(BnArgs w, int nu)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0) *w.active = 0;
    if (p >= w.count) return;
    for (int c = 0; c < nu; ++c) w.y[c * w.count + p] = 0.0;
    w.st[p] = -1;
    w.it[p] = 0;
}

/* counter reset as a kernel (graph-safe: no memory-set node) */
__global__ void k_bn_zero(int32_t *active)
{
    if (threadIdx.x == 0) *active = 0;
}

/* Assemble F, J at the current iterate of every point still iterating; apply
 * the stop rules of the fused loop in its order (non-finite residual,
 * ||F||_inf < tol, maxit); a finished point writes its outputs once and
 * leaves an identity system behind for the remaining batched solves. */
template <int NU, bool TAN>
__global__ void __launch_bounds__(256) k_bn_assemble(lupp_points pts, LawK P, BnArgs w, double tol,
                                                     int maxit)
{
    const int64_t p0 = (int64_t)blockIdx.x * blockDim.x;
    const int64_t p = p0 + threadIdx.x;
    const int64_t rem = pts.count - p0;
    const uint32_t nvalid = (uint32_t)(rem < (int64_t)blockDim.x ? rem : blockDim.x);
    const uint32_t nb = nvalid * 8u, vo = threadIdx.x * 8u;
    const bool live = p < pts.count && w.st[p] == -1;
    int still = 0;
    if (live) {
        double de[6], st[NU], y[NU], F[NU], sig[6], J[NU][NU];
#pragma unroll
        for (int c = 0; c < 6; ++c) de[c] = pts.deps[c * pts.ld + p];
#pragma unroll
        for (int c = 0; c < NU; ++c) {
            st[c] = pts.state[c * pts.ld + p];
            y[c] = w.y[c * w.count + p];
        }
        law_assemble<NU>(P, de, st, y, F, J, sig);
#pragma unroll
        for (int c = 0; c < 6; ++c) pts.sig[c * pts.ld + p] = sig[c];
        bool finite = true;
        double nrm = 0.0;
#pragma unroll
        for (int i = 0; i < NU; ++i) {
            finite = finite && __builtin_isfinite(F[i]);
            nrm = fmax(nrm, fabs(F[i]));
        }
        const int it = w.it[p];
        const int status = !finite ? 3 : (nrm < tol ? 0 : (it == maxit ? 1 : -1));
        double *Jp = w.J + p;
        double *rp = w.rhs + p;
        const int64_t C = w.count;
        if (status == -1) {
            still = 1;
#pragma unroll
            for (int c = 0; c < NU; ++c)
#pragma unroll
                for (int r = 0; r < NU; ++r) Jp[(c * NU + r) * C] = J[c][r];
#pragma unroll
            for (int r = 0; r < NU; ++r) rp[r * C] = -F[r];
        } else {
            w.st[p] = status;
            pts.status[p] = status;
            pts.iters[p] = it;
            if (status == 0) {
#pragma unroll
                for (int c = 0; c < NU; ++c) pts.state[c * pts.ld + p] = st[c] + y[c];
                if constexpr (TAN) {
                    if constexpr (NU == 7) newton_tangent7(P, de, st, y, pts, p0, nb, vo);
                    else newton_tangent13(P, de, st, y, pts, p0, nb, vo);
                }
            }
            /* an identity system for the solves this point is dragged through */
#pragma unroll
            for (int c = 0; c < NU; ++c) {
#pragma unroll
                for (int r = 0; r < NU; ++r) Jp[(c * NU + r) * C] = (c == r) ? 1.0 : 0.0;
                rp[c * C] = 0.0;
            }
        }
    }
    /* one atomic per wave */
    const uint64_t b = __ballot(still != 0);
    if (__lane_id() == 0 && b != 0) atomicAdd(w.active, (int)__builtin_popcountll(b));
}

/* The batched solve: point p's Jacobian and right-hand side, solved in
 * registers (J dx = -F, dx overwriting the right-hand side where the
 * factorisation has no zero pivot), info[p]. */
template <int NU>
__global__ void __launch_bounds__(256) k_bn_solve(BnArgs w)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= w.count) return;
    const int64_t C = w.count;
    double a[NU][NU], x[NU];
    int piv[NU];
#pragma unroll
    for (int c = 0; c < NU; ++c) {
#pragma unroll
        for (int r = 0; r < NU; ++r) a[c][r] = w.J[(r + c * NU) * C + p];
        x[c] = w.rhs[c * C + p];
    }
    const int inf = thread_getrf_solve<NU, false, kNewtonFMA, false, kNewtonRecip>(a, x, piv);
    if (inf == 0) {
#pragma unroll
        for (int c = 0; c < NU; ++c) w.rhs[c * C + p] = x[c];
    }
    w.info[p] = inf;
}

/* x += dx for the points that iterated; a zero pivot stops a point with
 * status 2 (its iterate is not updated, as in the fused loop). */
template <int NU>
__global__ void __launch_bounds__(256) k_bn_update(lupp_points pts, BnArgs w)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= w.count || w.st[p] != -1) return;
    if (w.info[p] != 0) {
        w.st[p] = 2;
        pts.status[p] = 2;
        pts.iters[p] = w.it[p];
        return;
    }
#pragma unroll
    for (int c = 0; c < NU; ++c) w.y[c * w.count + p] = w.y[c * w.count + p] + w.rhs[c * w.count + p];
    w.it[p] = w.it[p] + 1;
}

struct BnWs {
    int64_t cap = 0;
    int nu = 0;
    double *y = nullptr, *J = nullptr, *rhs = nullptr;
    int32_t *info = nullptr, *st = nullptr, *it = nullptr, *active = nullptr;
    int32_t *host_active = nullptr; /* pinned */
};

BnWs *bn_ws_create() { return new BnWs; }

static void bn_ws_release(BnWs *ws)
{
    hipFree(ws->y);
    hipFree(ws->J);
    hipFree(ws->rhs);
    hipFree(ws->info);
    hipFree(ws->st);
    hipFree(ws->it);
    hipFree(ws->active);
    ws->y = ws->J = ws->rhs = nullptr;
    ws->info = ws->st = ws->it = ws->active = nullptr;
    ws->cap = 0;
    ws->nu = 0;
}

void bn_ws_destroy(BnWs *ws)
{
    if (ws == nullptr) return;
    bn_ws_release(ws);
    if (ws->host_active) hipHostFree(ws->host_active);
    delete ws;
}

static hipError_t bn_ws_reserve(BnWs *ws, int64_t count, int nu, hipStream_t st)
{
    if (ws->cap >= count && ws->nu >= nu && ws->y != nullptr) return hipSuccess;
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    bn_ws_release(ws);
    const size_t C = (size_t)count;
    e = hipMalloc(&ws->y, C * nu * 8);
    if (e == hipSuccess) e = hipMalloc(&ws->J, C * nu * nu * 8);
    if (e == hipSuccess) e = hipMalloc(&ws->rhs, C * nu * 8);
    if (e == hipSuccess) e = hipMalloc(&ws->info, C * 4);
    if (e == hipSuccess) e = hipMalloc(&ws->st, C * 4);
    if (e == hipSuccess) e = hipMalloc(&ws->it, C * 4);
    if (e == hipSuccess) e = hipMalloc(&ws->active, 256);
    if (e == hipSuccess && ws->host_active == nullptr)
        e = hipHostMalloc(&ws->host_active, sizeof(int32_t), hipHostMallocDefault);
    if (e != hipSuccess) {
        bn_ws_release(ws);
        return e;
    }
    ws->cap = count;
    ws->nu = nu;
    return hipSuccess;
}

template <int NU, bool TAN>
static hipError_t bn_iteration(lupp_ctx *ctx, const lupp_points &pts, const LawK &P, const BnArgs &w,
                               const BnWs &ws, double tol, int maxit, hipStream_t st, int *rc)
{
    (void)ctx;
    (void)ws;
    const unsigned blocks = (unsigned)((pts.count + 255) / 256);
    hipLaunchKernelGGL(k_bn_zero, dim3(1), dim3(64), 0, st, w.active);
    hipLaunchKernelGGL((k_bn_assemble<NU, TAN>), dim3(blocks), dim3(256), 0, st, pts, P, w, tol, maxit);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_bn_solve<NU>), dim3(blocks), dim3(256), 0, st, w);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    *rc = 0;
    hipLaunchKernelGGL((k_bn_update<NU>), dim3(blocks), dim3(256), 0, st, pts, w);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return hipMemcpyAsync(ws.host_active, w.active, sizeof(int32_t), hipMemcpyDeviceToHost, st);
}

template <int NU, bool TAN>
static int bn_run(lupp_ctx *ctx, BnWs *ws, const lupp_points &pts, const LawK &P, double tol,
                  int maxit, bool graph, hipStream_t st, int *iterations)
{
    hipError_t e = bn_ws_reserve(ws, pts.count, NU, st);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? LUPP_E_NOMEM : hip_err(e);
    const BnArgs w{pts.count, ws->y, ws->J, ws->rhs, ws->info, ws->st, ws->it, ws->active};
    const unsigned blocks = (unsigned)((pts.count + 255) / 256);
    hipLaunchKernelGGL(k_bn_init, dim3(blocks), dim3(256), 0, st, w, NU);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_err(e);
    int rc = 0;
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    if (graph) {
        /* one Newton iteration (assemble, batched solve, update, counter copy)
         * captured once and replayed */
        hipStream_t cs = nullptr;
        e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            e = bn_iteration<NU, TAN>(ctx, pts, P, w, *ws, tol, maxit, cs, &rc);
            const hipError_t e2 = hipStreamEndCapture(cs, &g);
            if (e == hipSuccess) e = e2;
        }
        if (e == hipSuccess && rc == 0) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        if (cs) hipStreamDestroy(cs);
    }
    /* every point stops after at most maxit + 1 assemblies */
    int k = 0;
    for (; e == hipSuccess && rc == 0 && k <= maxit + 1; ++k) {
        if (graph) e = hipGraphLaunch(ge, st);
        else e = bn_iteration<NU, TAN>(ctx, pts, P, w, *ws, tol, maxit, st, &rc);
        if (e == hipSuccess && rc == 0) e = hipStreamSynchronize(st);
        if (e == hipSuccess && rc == 0 && *ws->host_active == 0) {
            ++k;
            break;
        }
    }
    if (ge) hipGraphExecDestroy(ge);
    if (g) hipGraphDestroy(g);
    if (iterations) *iterations = k;
    if (rc != 0) return rc;
    return hip_err(e);
}

int constitutive_batched_run(lupp_ctx *ctx, BnWs *ws, const lupp_points *pts, const lupp_law *law,
                             double tol, int maxit, bool graph, hipStream_t st, int *iterations)
{
    const LawK P = law_constants(law);
    const bool tan = pts->tangent != nullptr;
    if (law->kind == LUPP_LAW_NORTON7)
        return tan ? bn_run<7, true>(ctx, ws, *pts, P, tol, maxit, graph, st, iterations)
                   : bn_run<7, false>(ctx, ws, *pts, P, tol, maxit, graph, st, iterations);
    return tan ? bn_run<13, true>(ctx, ws, *pts, P, tol, maxit, graph, st, iterations)
               : bn_run<13, false>(ctx, ws, *pts, P, tol, maxit, graph, st, iterations);
}

}  // namespace lupp
