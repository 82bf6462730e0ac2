/* Time-step sweeps of the fused constitutive update, captured once in a HIP
 * graph and replayed with one launch.
 *
 * An implicit constitutive update runs at every step of the global solution
 * (Section 2.5); each step is one fused Newton kernel over all points
 * (Section 3.3, Algorithm 2) that commits the state the next step starts
 * from. For small point counts the per-step launch cost matters, so the
 * steps are recorded as kernel nodes of one graph. The capture records only
 * kernels (no memory-set nodes), and every replay recomputes from the state
 * buffer's current contents. */
#include <new>

#include "internal.h"

struct lupp_sweep {
    int device = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

using namespace lupp;

extern "C" {

int lupp_sweep_create(lupp_ctx *ctx, const lupp_points *pts, const lupp_law *law, double tol,
                      int maxit, int steps, int64_t deps_step, lupp_sweep **out)
{
    if (out == nullptr) return -8;
    *out = nullptr;
    if (ctx == nullptr) return -1;
    if (pts == nullptr || pts->count < 0 || pts->ld < pts->count) return -2;
    if (law == nullptr || (law->kind != LUPP_LAW_NORTON7 && law->kind != LUPP_LAW_NORTON_AF13))
        return -3;
    if (!(tol >= 0.0)) return -4;
    if (maxit < 0 || maxit > LUPP_MAXIT_LIMIT) return -5;
    if (steps < 1) return -6;
    if (deps_step != 0 && deps_step < 6 * pts->ld) return -7;
    if (pts->count > 0 && (pts->deps == nullptr || pts->state == nullptr || pts->sig == nullptr ||
                           pts->iters == nullptr || pts->status == nullptr))
        return -2;
    int dev = 0;
    lupp_get_device(ctx, &dev);
    int cur = 0;
    hipGetDevice(&cur);
    if (cur != dev) hipSetDevice(dev);
    lupp_sweep *sw = new (std::nothrow) lupp_sweep;
    if (sw == nullptr) return LUPP_E_NOMEM;
    sw->device = dev;
    hipStream_t st = nullptr;
    int rc = 0;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        for (int t = 0; t < steps && rc == 0 && pts->count > 0; ++t) {
            lupp_points p = *pts;
            p.deps = pts->deps + (int64_t)t * deps_step;
            int lanes = 1;
            lupp_get_newton_variant(ctx, law->kind, &lanes);
            rc = constitutive_launch(&p, law, tol, maxit, lanes, st);
        }
        /* always end the capture, also after a failed launch */
        const hipError_t e2 = hipStreamEndCapture(st, &sw->graph);
        if (rc == 0 && e2 != hipSuccess) e = e2;
    }
    if (rc == 0 && e == hipSuccess) e = hipGraphInstantiate(&sw->exec, sw->graph, nullptr, nullptr, 0);
    if (rc == 0 && e != hipSuccess) rc = hip_err(e);
    if (st) hipStreamDestroy(st);
    if (cur != dev) hipSetDevice(cur);
    if (rc != 0) {
        lupp_sweep_destroy(sw);
        return rc;
    }
    *out = sw;
    return 0;
}

int lupp_sweep_launch(lupp_sweep *sw, void *stream)
{
    if (sw == nullptr) return -1;
    int cur = 0;
    hipGetDevice(&cur);
    if (cur != sw->device) hipSetDevice(sw->device);
    const hipError_t e = hipGraphLaunch(sw->exec, (hipStream_t)stream);
    if (cur != sw->device) hipSetDevice(cur);
    return hip_err(e);
}

void lupp_sweep_destroy(lupp_sweep *sw)
{
    if (sw == nullptr) return;
    if (sw->exec) hipGraphExecDestroy(sw->exec);
    if (sw->graph) hipGraphDestroy(sw->graph);
    delete sw;
}

}  // extern "C"
