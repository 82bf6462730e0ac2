/* C-ABI entry points of liblupp: argument validation, the per-size dispatch
 * table (Section 4.1: a size-aware dispatcher selects the specialised kernel
 * for each problem size), and launch. */
#include <cstdio>
#include <cstring>
#include <new>

#include "internal.h"

namespace lupp {

struct Choice {
    int variant;  /* LUPP_VARIANT_THREAD / LUPP_VARIANT_LANES */
    int lanes;
    int wpb;
};

}  // namespace lupp

struct lupp_ctx {
    int device;
    int forced_variant = LUPP_VARIANT_AUTO;
    int forced_lanes = 0;
    int forced_wpb = 0;
    lupp::Choice table[33][2];
    void *ragged_ws = nullptr;   /* device workspace of the ragged path */
    size_t ragged_ws_bytes = 0;
};

namespace lupp {

/* Defaults before autotuning: registers-only thread path while a system fits
 * one lane comfortably, then one row per lane. */
static Choice default_choice(int n, int layout)
{
    (void)layout;
    if (n <= 8) return {LUPP_VARIANT_THREAD, 1, 4};
    if (n <= 16) return {LUPP_VARIANT_LANES, 16, 4};
    return {LUPP_VARIANT_LANES, 32, 4};
}

static bool fits_offsets(int n, int64_t batch, int layout, int variant, int lanes,
                         int64_t sA, int64_t sB)
{
    const int64_t lim = (int64_t)1 << 31;
    if (layout == LUPP_SOA) {
        if (variant == LUPP_VARIANT_THREAD) return true;
        (void)batch;
        return ((int64_t)(n - 1) * sA + 64) * 8 < lim && ((int64_t)(n - 1) * sB + 64) * 8 < lim;
    }
    const int64_t per = variant == LUPP_VARIANT_THREAD ? 256 : 64 / (lanes > 0 ? lanes : 1);
    return per * sA * 8 < lim && per * sB * 8 < lim && per * n * 4 < lim;
}

static LaunchFn pick(int n, const Choice &c)
{
    if (c.variant == LUPP_VARIANT_THREAD) return thread_launcher(n);
    if (c.variant == LUPP_VARIANT_LANES) return lanes_launcher(n, c.lanes);
    return nullptr;
}

}  // namespace lupp

using namespace lupp;

extern "C" {

int lupp_create(lupp_ctx **ctx, int device)
{
    if (ctx == nullptr) return -1;
    *ctx = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return hip_err(e);
    if (device < 0 || device >= count) return -2;
    lupp_ctx *c = new (std::nothrow) lupp_ctx;
    if (c == nullptr) return LUPP_E_NOMEM;
    c->device = device;
    for (int n = 0; n <= 32; ++n)
        for (int l = 0; l < 2; ++l) c->table[n][l] = default_choice(n < 1 ? 1 : n, l);
    *ctx = c;
    return 0;
}

void lupp_destroy(lupp_ctx *ctx)
{
    if (ctx == nullptr) return;
    if (ctx->ragged_ws != nullptr) {
        int cur = 0;
        hipGetDevice(&cur);
        hipSetDevice(ctx->device);
        hipFree(ctx->ragged_ws);
        hipSetDevice(cur);
    }
    delete ctx;
}

int lupp_force_variant(lupp_ctx *ctx, int variant, int lanes, int wpb)
{
    if (ctx == nullptr) return -1;
    if (variant != LUPP_VARIANT_AUTO && variant != LUPP_VARIANT_THREAD &&
        variant != LUPP_VARIANT_LANES)
        return -2;
    if (variant == LUPP_VARIANT_LANES && lanes != 2 && lanes != 4 && lanes != 8 && lanes != 16 &&
        lanes != 32)
        return -3;
    if (wpb != 0 && wpb != 1 && wpb != 2 && wpb != 4) return -4;
    ctx->forced_variant = variant;
    ctx->forced_lanes = lanes;
    ctx->forced_wpb = wpb;
    return 0;
}

int lupp_set_dispatch(lupp_ctx *ctx, int n, int layout, int variant, int lanes, int wpb)
{
    if (ctx == nullptr) return -1;
    if (n < 1 || n > 32) return -2;
    if (layout != LUPP_AOS && layout != LUPP_SOA) return -3;
    if (variant != LUPP_VARIANT_THREAD && variant != LUPP_VARIANT_LANES) return -4;
    const Choice c{variant, lanes, wpb};
    if (pick(n, c) == nullptr) return -5;
    if (wpb != 0 && wpb != 1 && wpb != 2 && wpb != 4) return -6;
    ctx->table[n][layout] = c;
    return 0;
}

int lupp_get_dispatch(lupp_ctx *ctx, int n, int layout, int *variant, int *lanes, int *wpb)
{
    if (ctx == nullptr) return -1;
    if (n < 1 || n > 32) return -2;
    if (layout != LUPP_AOS && layout != LUPP_SOA) return -3;
    const Choice &c = ctx->table[n][layout];
    if (variant) *variant = c.variant;
    if (lanes) *lanes = c.lanes;
    if (wpb) *wpb = c.wpb;
    return 0;
}

int lupp_check_solve_args(int n, int64_t batch, int layout, const double *A, int64_t lda,
                          int64_t strideA, const double *b, int64_t strideB, const int32_t *ipiv,
                          const int32_t *info, unsigned flags)
{
    if (n < 1 || n > 32) return -2;
    if (batch < 0) return -3;
    if (layout != LUPP_AOS && layout != LUPP_SOA) return -4;
    if (A == nullptr && batch > 0) return -5;
    if (lda < n) return -6;
    if (layout == LUPP_AOS ? strideA < lda * n : strideA < batch) return -7;
    if (b == nullptr && batch > 0) return -8;
    if (layout == LUPP_AOS ? strideB < n : strideB < batch) return -9;
    if (ipiv == nullptr && batch > 0) return -10;
    if (info == nullptr && batch > 0) return -11;
    if ((flags & ~LUPP_KEEP_A) != 0) return -12;
    return 0;
}

int lupp_batched_solve(lupp_ctx *ctx, int n, int64_t batch, int layout, double *A, int64_t lda,
                       int64_t strideA, double *b, int64_t strideB, int32_t *ipiv,
                       int32_t *info, unsigned flags, void *stream)
{
    if (ctx == nullptr) return -1;
    const int bad = lupp_check_solve_args(n, batch, layout, A, lda, strideA, b, strideB, ipiv,
                                          info, flags);
    if (bad != 0) return bad;
    if (batch == 0) return 0;

    Choice c = ctx->table[n][layout];
    if (ctx->forced_variant != LUPP_VARIANT_AUTO)
        c = Choice{ctx->forced_variant, ctx->forced_lanes, ctx->forced_wpb};
    LaunchFn fn = pick(n, c);
    if (fn == nullptr) return LUPP_E_UNSUPPORTED;
    if (!fits_offsets(n, batch, layout, c.variant, c.lanes, strideA, strideB)) {
        /* the thread path has no 32-bit offset limit in SoA */
        const Choice t{LUPP_VARIANT_THREAD, 1, 4};
        if (ctx->forced_variant != LUPP_VARIANT_AUTO || thread_launcher(n) == nullptr ||
            !fits_offsets(n, batch, layout, t.variant, t.lanes, strideA, strideB))
            return LUPP_E_UNSUPPORTED;
        c = t;
        fn = thread_launcher(n);
    }
    int cur = 0;
    hipGetDevice(&cur);
    if (cur != ctx->device) hipSetDevice(ctx->device);
    SolveArgs a{batch, A, lda, strideA, b, strideB, ipiv, info};
    const hipError_t e = fn(a, layout, (flags & LUPP_KEEP_A) == 0, c.wpb, (hipStream_t)stream);
    if (cur != ctx->device) hipSetDevice(cur);
    return hip_err(e);
}

int lupp_batched_solve_ragged(lupp_ctx *ctx, int64_t batch, const int32_t *n,
                              const int64_t *offA, const int64_t *offB, double *A, double *b,
                              int32_t *ipiv, int32_t *info, unsigned flags, void *stream)
{
    if (ctx == nullptr) return -1;
    if (batch < 0) return -2;
    if (batch > 0 && n == nullptr) return -3;
    if (batch > 0 && offA == nullptr) return -4;
    if (batch > 0 && offB == nullptr) return -5;
    if (batch > 0 && A == nullptr) return -6;
    if (batch > 0 && b == nullptr) return -7;
    if (batch > 0 && ipiv == nullptr) return -8;
    if (batch > 0 && info == nullptr) return -9;
    if ((flags & ~LUPP_KEEP_A) != 0) return -10;
    if (batch == 0) return 0;
    int cur = 0;
    hipGetDevice(&cur);
    if (cur != ctx->device) hipSetDevice(ctx->device);
    const int rc = ragged_launch(ctx, batch, n, offA, offB, A, b, ipiv, info,
                                 (flags & LUPP_KEEP_A) == 0, (hipStream_t)stream);
    if (cur != ctx->device) hipSetDevice(cur);
    return rc;
}

int lupp_variant_info(int n, int layout, int variant, int lanes, int keep_a,
                      lupp_kernel_info *out)
{
    (void)layout;
    (void)keep_a;
    if (out == nullptr) return -6;
    const void *sym = nullptr;
    if (variant == LUPP_VARIANT_THREAD) sym = thread_kernel_symbol(n);
    else if (variant == LUPP_VARIANT_LANES) sym = lanes_kernel_symbol(n, lanes);
    else if (variant == 100 + LUPP_LAW_NORTON7 || variant == 100 + LUPP_LAW_NORTON_AF13)
        sym = constitutive_kernel_symbol(variant - 100);
    if (sym == nullptr) return LUPP_E_UNSUPPORTED;
    hipFuncAttributes fa;
    std::memset(&fa, 0, sizeof(fa));
    const hipError_t e = hipFuncGetAttributes(&fa, sym);
    if (e != hipSuccess) return hip_err(e);
    out->vgprs = fa.numRegs;
    out->agprs = -1;
    out->sgprs = -1;
    out->scratch_bytes = (int)fa.localSizeBytes;
    out->lds_bytes = (int)fa.sharedSizeBytes;
    out->max_threads = fa.maxThreadsPerBlock;
    return 0;
}

int constitutive_update(lupp_ctx *ctx, const lupp_points *pts, const lupp_law *law, double tol,
                        int maxit, void *stream)
{
    if (ctx == nullptr) return -1;
    if (pts == nullptr || pts->count < 0 || pts->ld < pts->count) return -2;
    if (law == nullptr || (law->kind != LUPP_LAW_NORTON7 && law->kind != LUPP_LAW_NORTON_AF13))
        return -3;
    if (!(tol >= 0.0)) return -4;
    if (maxit < 0 || maxit > LUPP_MAXIT_LIMIT) return -5;
    if (pts->count == 0) return 0;
    if (pts->deps == nullptr || pts->state == nullptr || pts->sig == nullptr ||
        pts->iters == nullptr || pts->status == nullptr)
        return -2;
    int cur = 0;
    hipGetDevice(&cur);
    if (cur != ctx->device) hipSetDevice(ctx->device);
    const int rc = constitutive_launch(pts, law, tol, maxit, (hipStream_t)stream);
    if (cur != ctx->device) hipSetDevice(cur);
    return rc;
}

const char *lupp_error_string(int code)
{
    static thread_local char buf[96];
    if (code == 0) return "success";
    if (code == LUPP_E_UNSUPPORTED) return "request not supported by this build";
    if (code == LUPP_E_NOMEM) return "out of memory";
    if (code <= LUPP_E_HIP_BASE) {
        std::snprintf(buf, sizeof(buf), "HIP error %d: %s", LUPP_E_HIP_BASE - code,
                      hipGetErrorString((hipError_t)(LUPP_E_HIP_BASE - code)));
        return buf;
    }
    if (code < 0) {
        std::snprintf(buf, sizeof(buf), "argument %d is invalid", -code);
        return buf;
    }
    return "unknown code";
}

}  // extern "C"
