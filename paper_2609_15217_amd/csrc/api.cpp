/* C-ABI entry points of liblupp: argument validation, the per-size dispatch
 * table (Section 4.1: a size-aware dispatcher selects the specialised kernel
 * for each problem size), and launch. */
#include <cstdio>
#include <cstring>
#include <new>

#include "internal.h"
#include "serving.h"

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
    lupp::Choice table[33][2][2]; /* [n][layout][batch bucket] */
    lupp::RaggedWs *ragged_ws = nullptr; /* device workspace of the ragged path */
    lupp::BnWs *bn_ws = nullptr;         /* device workspace of the batched Newton */
    int newton_lanes[2] = {lupp::newton_default_lanes(LUPP_LAW_NORTON7),
                           lupp::newton_default_lanes(LUPP_LAW_NORTON_AF13)};
    int tile = 0;          /* pivoting of lupp_batched_solve: 0 textbook, else tile-local */
    double thresh = 0.0;
    uint8_t ragged_lanes[33] = {}; /* lanes per system of the ragged path, per size */
};

namespace lupp {

/* Default dispatch: the table the autotuner measured on gfx950 (compiled in
 * by the build from dispatch_gfx950.json), else registers-only thread path
 * while a system fits one lane comfortably, then one row per lane. */
static Choice default_choice(int n, int layout, int bucket)
{
    int v = 0, l = 0, w = 0;
    if (tuned_choice(n, layout, bucket, &v, &l, &w)) return {v, l, w};
    if (n <= 8) return {LUPP_VARIANT_THREAD, 1, 4};
    if (n <= 16) return {LUPP_VARIANT_LANES, 16, 4};
    return {LUPP_VARIANT_LANES, 32, 4};
}

static bool fits_offsets(int n, int64_t batch, int layout, int variant, int lanes,
                         int64_t sA, int64_t sB)
{
    const int64_t lim = (int64_t)1 << 31;
    (void)batch;
    (void)n;
    if (layout == LUPP_SOA) {
        /* the thread kernel bases one descriptor at every element: its
         * extents cover one workgroup's systems, any ldbatch fits */
        if (variant == LUPP_VARIANT_THREAD) return true;
        /* the staged kernel's descriptors span the rows one wave moves:
         * 64/S rows of S systems, S = max(64/lanes, 16) */
        const int64_t S = 64 / lanes > 16 ? 64 / lanes : 16;
        const int64_t rows = 64 / S;
        return ((rows - 1) * sA + S) * 8 < lim && ((rows - 1) * sB + S) * 8 < lim;
    }
    const int64_t per = variant == LUPP_VARIANT_THREAD ? 256 : 64 / (lanes > 0 ? lanes : 1);
    return per * sA * 8 < lim && per * sB * 8 < lim && per * n * 4 < lim;
}

/* Batch-size bucket of the dispatch table: small batches (latency-bound,
 * the GPU is not filled) and large ones. */
static int bucket_of(int64_t batch) { return batch < kSmallBatch ? 0 : 1; }

static LaunchFn pick(int n, const Choice &c)
{
    if (c.variant == LUPP_VARIANT_THREAD) return thread_launcher(n);
    if (c.variant == LUPP_VARIANT_LANES) return lanes_launcher(n, c.lanes);
    return nullptr;
}

void ctx_copy_settings(lupp_ctx *dst, const lupp_ctx *src)
{
    dst->forced_variant = src->forced_variant;
    dst->forced_lanes = src->forced_lanes;
    dst->forced_wpb = src->forced_wpb;
    std::memcpy(dst->table, src->table, sizeof(dst->table));
    dst->newton_lanes[0] = src->newton_lanes[0];
    dst->newton_lanes[1] = src->newton_lanes[1];
    dst->tile = src->tile;
    dst->thresh = src->thresh;
    std::memcpy(dst->ragged_lanes, src->ragged_lanes, sizeof(dst->ragged_lanes));
}

bool ctx_textbook_dispatch(const lupp_ctx *ctx)
{
    return ctx->tile == 0 && ctx->forced_variant == LUPP_VARIANT_AUTO;
}

const uint8_t *ctx_ragged_lanes(const lupp_ctx *ctx) { return ctx->ragged_lanes; }

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
        for (int l = 0; l < 2; ++l)
            for (int bk = 0; bk < 2; ++bk) c->table[n][l][bk] = default_choice(n < 1 ? 1 : n, l, bk);
    for (int n = 1; n <= 32; ++n) {
        int t = 0;
        c->ragged_lanes[n] = (uint8_t)((tuned_ragged(n, &t) && ragged_lanes_ok(n, t))
                                           ? t : ragged_default_lanes(n));
    }
    /* set-up of the allocation-free ragged path: resolve its workspace on
     * this device (once per device); a failure surfaces only in that call */
    (void)noalloc_scratch_init(device);
    *ctx = c;
    return 0;
}

void lupp_destroy(lupp_ctx *ctx)
{
    if (ctx == nullptr) return;
    if (ctx->ragged_ws != nullptr || ctx->bn_ws != nullptr) {
        int cur = 0;
        hipGetDevice(&cur);
        hipSetDevice(ctx->device);
        ragged_ws_destroy(ctx->ragged_ws);
        bn_ws_destroy(ctx->bn_ws);
        hipSetDevice(cur);
    }
    delete ctx;
}

int lupp_get_device(const lupp_ctx *ctx, int *device)
{
    if (ctx == nullptr) return -1;
    if (device == nullptr) return -2;
    *device = ctx->device;
    return 0;
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

int lupp_set_dispatch(lupp_ctx *ctx, int n, int layout, int64_t batch, int variant, int lanes,
                      int wpb)
{
    if (ctx == nullptr) return -1;
    if (n < 1 || n > 32) return -2;
    if (layout != LUPP_AOS && layout != LUPP_SOA) return -3;
    if (batch < 0) return -4;
    if (variant != LUPP_VARIANT_THREAD && variant != LUPP_VARIANT_LANES) return -5;
    const Choice c{variant, lanes, wpb};
    if (pick(n, c) == nullptr) return -6;
    if (wpb != 0 && wpb != 1 && wpb != 2 && wpb != 4) return -7;
    ctx->table[n][layout][bucket_of(batch)] = c;
    return 0;
}

int lupp_get_dispatch(lupp_ctx *ctx, int n, int layout, int64_t batch, int *variant, int *lanes,
                      int *wpb)
{
    if (ctx == nullptr) return -1;
    if (n < 1 || n > 32) return -2;
    if (layout != LUPP_AOS && layout != LUPP_SOA) return -3;
    if (batch < 0) return -4;
    const Choice &c = ctx->table[n][layout][bucket_of(batch)];
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
    if ((flags & ~(LUPP_KEEP_A | LUPP_FMA)) != 0) return -12;
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

    /* compiled instances: strict, FMA, strict with tile-local pivoting */
    if ((flags & LUPP_FMA) != 0 && ctx->tile > 0) return LUPP_E_UNSUPPORTED;
    Choice c = ctx->table[n][layout][bucket_of(batch)];
    if (ctx->forced_variant != LUPP_VARIANT_AUTO)
        c = Choice{ctx->forced_variant, ctx->forced_lanes, ctx->forced_wpb};
    LaunchFn fn = pick(n, c);
    if (fn == nullptr) return LUPP_E_UNSUPPORTED;
    if (!fits_offsets(n, batch, layout, c.variant, c.lanes, strideA, strideB)) {
        /* an interleaved batch too far apart for the staged lanes kernel:
         * the thread kernel takes any ldbatch (sizes it is compiled for) */
        if (layout != LUPP_SOA || n > kThreadMaxN) return LUPP_E_UNSUPPORTED;
        c = Choice{LUPP_VARIANT_THREAD, 1, 0};
        fn = pick(n, c);
        if (fn == nullptr) return LUPP_E_UNSUPPORTED;
    }
    int cur = 0;
    hipGetDevice(&cur);
    if (cur != ctx->device) hipSetDevice(ctx->device);
    SolveArgs a{batch, A, lda, strideA, b, strideB, ipiv, info, ctx->tile, ctx->thresh,
                (flags & LUPP_FMA) != 0 ? 1 : 0};
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
    if ((flags & ~(LUPP_KEEP_A | LUPP_RAGGED_PER_SIZE)) != 0) return -10;
    if (batch == 0) return 0;
    int cur = 0;
    hipGetDevice(&cur);
    if (cur != ctx->device) hipSetDevice(ctx->device);
    if (ctx->ragged_ws == nullptr) ctx->ragged_ws = ragged_ws_create();
    const int rc = ragged_launch_impl(ctx->ragged_ws, ctx->ragged_lanes, batch, n, offA, offB, A,
                                      b, ipiv, info, (flags & LUPP_KEEP_A) == 0,
                                      (flags & LUPP_RAGGED_PER_SIZE) != 0, (hipStream_t)stream);
    if (cur != ctx->device) hipSetDevice(cur);
    return rc;
}

int lupp_batched_solve_grouped(lupp_ctx *ctx, int ngroups, const lupp_group *groups,
                               unsigned flags, void *stream)
{
    if (ctx == nullptr) return -1;
    if (ngroups < 0) return -2;
    if (ngroups > 0 && groups == nullptr) return -3;
    for (int i = 0; i < ngroups; ++i) {
        const lupp_group &g = groups[i];
        if (g.n < 1 || g.n > 32 || g.batch < 0 || g.batch > 0x7fffffff) return -3;
        if (g.batch == 0) continue;
        if (g.A == nullptr || g.b == nullptr || g.ipiv == nullptr || g.info == nullptr) return -3;
        if (g.lda < g.n || g.strideA < g.lda * g.n || g.strideB < g.n) return -3;
    }
    if ((flags & ~LUPP_KEEP_A) != 0) return -4;
    if (ngroups == 0) return 0;
    int cur = 0;
    hipGetDevice(&cur);
    if (cur != ctx->device) hipSetDevice(ctx->device);
    const int rc = grouped_enqueue(groups, ngroups, ctx->ragged_lanes, (flags & LUPP_KEEP_A) == 0,
                                   (hipStream_t)stream);
    if (cur != ctx->device) hipSetDevice(cur);
    return rc;
}

int lupp_batched_solve_ragged_noalloc(lupp_ctx *ctx, int64_t batch, const int32_t *n,
                                      const int64_t *offA, const int64_t *offB, double *A,
                                      double *b, int32_t *ipiv, int32_t *info, unsigned flags,
                                      void *stream)
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
    if (batch > LUPP_NOALLOC_MAX_BATCH) return LUPP_E_TOO_LARGE;
    if (batch == 0) return 0;
    int cur = 0;
    hipGetDevice(&cur);
    if (cur != ctx->device) hipSetDevice(ctx->device);
    const int rc = noalloc_ragged_enqueue(ctx->device, ctx->ragged_lanes, batch, n, offA, offB, A,
                                          b, ipiv, info, (flags & LUPP_KEEP_A) == 0,
                                          (hipStream_t)stream);
    if (cur != ctx->device) hipSetDevice(cur);
    return rc;
}

int lupp_ragged_lanes_supported(int n, int lanes) { return ragged_lanes_ok(n, lanes) ? 1 : 0; }

int lupp_set_ragged_lanes(lupp_ctx *ctx, int n, int lanes)
{
    if (ctx == nullptr) return -1;
    if (n < 1 || n > 32) return -2;
    if (!ragged_lanes_ok(n, lanes)) return -3;
    ctx->ragged_lanes[n] = (uint8_t)lanes;
    return 0;
}

int lupp_get_ragged_lanes(const lupp_ctx *ctx, int n)
{
    if (ctx == nullptr) return -1;
    if (n < 1 || n > 32) return -2;
    return ctx->ragged_lanes[n];
}

int lupp_autotune_ragged(lupp_ctx *ctx, int n, int64_t batch, const double *A, const double *b,
                         int reps, int *lanes, float *ms, void *stream)
{
    if (ctx == nullptr) return -1;
    if (n < 1 || n > 32) return -2;
    if (batch < 1 || batch > 0x7fffffff) return -3;
    if (A == nullptr) return -4;
    if (b == nullptr) return -5;
    if (reps < 1) return -6;
    int cur = 0;
    hipGetDevice(&cur);
    if (cur != ctx->device) hipSetDevice(ctx->device);
    if (ctx->ragged_ws == nullptr) ctx->ragged_ws = ragged_ws_create();
    const int rc = ragged_autotune_impl(ctx->ragged_ws, ctx->ragged_lanes, n, batch, A, b, reps,
                                        lanes, ms, (hipStream_t)stream);
    if (cur != ctx->device) hipSetDevice(cur);
    return rc;
}

int lupp_autotune(lupp_ctx *ctx, int n, int64_t batch, int layout, const double *A, int64_t lda,
                  int64_t strideA, const double *b, int64_t strideB, int reps, int *variant,
                  int *lanes, int *wpb, float *ms, void *stream)
{
    if (ctx == nullptr) return -1;
    const int bad = lupp_check_solve_args(n, batch, layout, A, lda, strideA, b, strideB,
                                          (const int32_t *)1, (const int32_t *)1, 0);
    if (bad != 0) return bad;
    if (batch == 0) return -3;
    if (reps < 1) return -10;
    int cur = 0;
    hipGetDevice(&cur);
    if (cur != ctx->device) hipSetDevice(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    const size_t nA = layout == LUPP_AOS ? (size_t)batch * strideA : (size_t)n * lda * strideA;
    const size_t nB = layout == LUPP_AOS ? (size_t)batch * strideB : (size_t)n * strideB;
    const size_t nP = layout == LUPP_AOS ? (size_t)batch * n : (size_t)n * strideA;
    double *wA = nullptr, *wB = nullptr;
    int32_t *wP = nullptr, *wI = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = 0;
    hipError_t e = hipMalloc(&wA, nA * 8);
    if (e == hipSuccess) e = hipMalloc(&wB, nB * 8);
    if (e == hipSuccess) e = hipMalloc(&wP, nP * 4);
    if (e == hipSuccess) e = hipMalloc(&wI, (size_t)batch * 4);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) rc = e == hipErrorOutOfMemory ? LUPP_E_NOMEM : hip_err(e);

    Choice best{0, 0, 0};
    float best_ms = 3.0e38f;
    int widths[8];
    const int nw = lanes_widths(n, widths, 8);
    Choice cands[64];
    int nc = 0;
    for (int w = 1; w <= 4; w <<= 1) {
        if (thread_launcher(n) != nullptr) cands[nc++] = {LUPP_VARIANT_THREAD, 1, w};
        /* the SoA lanes kernel has one workgroup shape */
        if (layout == LUPP_SOA && w > 1) continue;
        for (int i = 0; i < nw; ++i)
            cands[nc++] = {LUPP_VARIANT_LANES, widths[i], layout == LUPP_SOA ? 0 : w};
    }
    SolveArgs a{batch, wA, lda, strideA, wB, strideB, wP, wI, ctx->tile, ctx->thresh, 0};
    for (int c = 0; c < nc && rc == 0; ++c) {
        if (!fits_offsets(n, batch, layout, cands[c].variant, cands[c].lanes, strideA, strideB))
            continue;
        LaunchFn fn = pick(n, cands[c]);
        float t[64];
        const int r_total = reps + 1 < 64 ? reps + 1 : 64;
        for (int r = 0; r < r_total && rc == 0; ++r) {
            e = hipMemcpyAsync(wA, A, nA * 8, hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess) e = hipMemcpyAsync(wB, b, nB * 8, hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess) e = hipEventRecord(e0, st);
            if (e == hipSuccess) e = fn(a, layout, true, cands[c].wpb, st);
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(&t[r], e0, e1);
            if (e != hipSuccess) rc = hip_err(e);
        }
        if (rc != 0) break;
        /* median of the timed repetitions (the first launch is a warm-up) */
        for (int i = 1; i < r_total; ++i)
            for (int j = i + 1; j < r_total; ++j)
                if (t[j] < t[i]) { float x = t[i]; t[i] = t[j]; t[j] = x; }
        const float med = t[1 + (r_total - 1) / 2];
        if (med < best_ms) { best_ms = med; best = cands[c]; }
    }
    if (rc == 0 && best.variant != 0) {
        ctx->table[n][layout][bucket_of(batch)] = best;
        if (variant) *variant = best.variant;
        if (lanes) *lanes = best.lanes;
        if (wpb) *wpb = best.wpb;
        if (ms) *ms = best_ms;
    } else if (rc == 0) {
        rc = LUPP_E_UNSUPPORTED;
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    hipFree(wA);
    hipFree(wB);
    hipFree(wP);
    hipFree(wI);
    if (cur != ctx->device) hipSetDevice(cur);
    return rc;
}

int lupp_variant_info(int n, int layout, int variant, int lanes, int keep_a,
                      lupp_kernel_info *out)
{
    if (out == nullptr) return -6;
    const void *sym = nullptr;
    if (variant == LUPP_VARIANT_THREAD) sym = thread_kernel_symbol(n);
    else if (variant == LUPP_VARIANT_LANES) sym = lanes_kernel_symbol(n, lanes, layout);
    else if (variant == 100 + LUPP_LAW_NORTON7 || variant == 100 + LUPP_LAW_NORTON_AF13)
        sym = constitutive_kernel_symbol(variant - 100, keep_a != 0);
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
    const int lanes = ctx->newton_lanes[law->kind == LUPP_LAW_NORTON7 ? 0 : 1];
    const int rc = constitutive_launch(pts, law, tol, maxit, lanes, (hipStream_t)stream);
    if (cur != ctx->device) hipSetDevice(cur);
    return rc;
}

int lupp_set_pivoting(lupp_ctx *ctx, int tile, double threshold)
{
    if (ctx == nullptr) return -1;
    if (tile < 0 || tile > 32) return -2;
    if (!(threshold >= 0.0)) return -3;
    ctx->tile = tile;
    ctx->thresh = tile > 0 ? threshold : 0.0;
    return 0;
}

int lupp_get_pivoting(const lupp_ctx *ctx, int *tile, double *threshold)
{
    if (ctx == nullptr) return -1;
    if (tile) *tile = ctx->tile;
    if (threshold) *threshold = ctx->thresh;
    return 0;
}

int lupp_set_newton_variant(lupp_ctx *ctx, int kind, int lanes)
{
    if (ctx == nullptr) return -1;
    if (kind != LUPP_LAW_NORTON7 && kind != LUPP_LAW_NORTON_AF13) return -2;
    if (lanes == 0) lanes = newton_default_lanes(kind);
    if (!newton_lanes_supported(kind, lanes)) return -3;
    ctx->newton_lanes[kind == LUPP_LAW_NORTON7 ? 0 : 1] = lanes;
    return 0;
}

int lupp_get_newton_variant(const lupp_ctx *ctx, int kind, int *lanes)
{
    if (ctx == nullptr) return -1;
    if (kind != LUPP_LAW_NORTON7 && kind != LUPP_LAW_NORTON_AF13) return -2;
    if (lanes == nullptr) return -3;
    *lanes = ctx->newton_lanes[kind == LUPP_LAW_NORTON7 ? 0 : 1];
    return 0;
}

int constitutive_update_batched(lupp_ctx *ctx, const lupp_points *pts, const lupp_law *law,
                                double tol, int maxit, unsigned flags, void *stream,
                                int *iterations)
{
    if (iterations) *iterations = 0;
    if (ctx == nullptr) return -1;
    if (pts == nullptr || pts->count < 0 || pts->ld < pts->count) return -2;
    if (law == nullptr || (law->kind != LUPP_LAW_NORTON7 && law->kind != LUPP_LAW_NORTON_AF13))
        return -3;
    if (!(tol >= 0.0)) return -4;
    if (maxit < 0 || maxit > LUPP_MAXIT_LIMIT) return -5;
    if ((flags & ~LUPP_BATCHED_GRAPH) != 0) return -6;
    if (pts->count == 0) return 0;
    if (pts->deps == nullptr || pts->state == nullptr || pts->sig == nullptr ||
        pts->iters == nullptr || pts->status == nullptr)
        return -2;
    int cur = 0;
    hipGetDevice(&cur);
    if (cur != ctx->device) hipSetDevice(ctx->device);
    if (ctx->bn_ws == nullptr) ctx->bn_ws = bn_ws_create();
    const int rc = constitutive_batched_run(ctx, ctx->bn_ws, pts, law, tol, maxit,
                                            (flags & LUPP_BATCHED_GRAPH) != 0,
                                            (hipStream_t)stream, iterations);
    if (cur != ctx->device) hipSetDevice(cur);
    return rc;
}

const char *lupp_error_string(int code)
{
    static thread_local char buf[96];
    if (code == 0) return "success";
    if (code == LUPP_E_UNSUPPORTED) return "request not supported by the compiled kernels";
    if (code == LUPP_E_NOMEM) return "out of memory";
    if (code == LUPP_E_TOO_LARGE)
        return "batch exceeds the allocation-free workspace (LUPP_NOALLOC_MAX_BATCH systems)";
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
