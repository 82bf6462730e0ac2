/* Serving loop: continuous batching of standalone-solve and constitutive-
 * update requests under an HBM budget.
 *
 * A request names its inputs and outputs by pointer (host or device). The
 * scheduler thread admits waiting requests in submission order while an
 * in-flight slot is free and the arena (a device allocation the size of the
 * HBM budget) holds their staging buffers, and runs everything admitted in
 * one scheduling pass together on one of the server's streams:
 *   - every solve request of the pass becomes one group of one grouped solve
 *     (lupp_batched_solve_grouped: a launch per size class for all of them);
 *   - the update requests of the pass with the same law, tol, maxit and
 *     tangent choice become one grouped fused-Newton launch over their point
 *     sets;
 *   - one host callback on the stream then completes every request of the
 *     pass.
 * Successive passes go to successive streams, so they overlap on the GPU.
 * Device-resident data is used in place: a device A is only read (the factors
 * go to the request's lu, or nowhere), right-hand sides are copied into a
 * device x and solved there, device outputs are written directly. Only host
 * buffers (and outputs the request does not want) take arena space: host
 * inputs are copied in, host outputs copied out. Integration-point state
 * lives on the device in registered point sets that update requests advance;
 * requests on the same set run in submission order. Latency runs from submit
 * to the completion of the pass that holds the request.
 */
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "serving.h"

namespace lupp {

using Clock = std::chrono::steady_clock;

/* first-fit allocator over [0, size) with 256-byte granules */
class Arena {
  public:
    explicit Arena(size_t size) : size_(size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = (bytes + 255) & ~(size_t)255;
        if (bytes == 0) {
            *off = 0;
            return true;
        }
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = (bytes + 255) & ~(size_t)255;
        if (bytes == 0) return;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t size() const { return size_; }

  private:
    size_t size_, used_ = 0;
    std::map<size_t, size_t> free_;
};

struct PointSet {
    int kind = 0;
    int64_t count = 0;
    double *state = nullptr; /* [kind][count] device, owned */
    bool busy = false;       /* a request on this set is admitted */
};

static bool is_device(const void *p)
{
    if (p == nullptr) return false;
    hipPointerAttribute_t a;
    std::memset(&a, 0, sizeof(a));
    if (hipPointerGetAttributes(&a, p) == hipSuccess && a.type == hipMemoryTypeDevice) return true;
    (void)hipGetLastError();
    return false;
}

static size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr size_t kNone = ~(size_t)0;

/* Where each buffer of a request lives during its pass: a caller pointer
 * used in place, or an arena slot (offset; kNone = not staged). */
struct Staging {
    size_t fac = kNone, rhs = kNone, piv = kNone, inf = kNone;      /* solve */
    size_t deps = kNone, sig = kNone, its = kNone, sts = kNone, tan = kNone; /* update */
    size_t bytes = 0;
};

struct Req {
    int64_t ticket = 0;
    lupp_request r{};
    lupp_law law{};
    Staging sg;
    bool dev_A = false, dev_x = false, dev_lu = false, dev_ipiv = false, dev_info = false;
    bool dev_deps = false, dev_sig = false, dev_it = false, dev_st = false, dev_tan = false;
    size_t off = 0; /* arena base of the staging slots */
    double *set_state = nullptr;
    Clock::time_point t_submit, t_done;
    int status = 0; /* 0 ok or a lupp error */
    bool done = false;
};

/* The staging slots a request needs, from where its pointers live. */
static void plan_staging(Req &q)
{
    Staging &s = q.sg;
    size_t at = 0;
    auto slot = [&](size_t bytes) {
        const size_t o = at;
        at += round256(bytes);
        return o;
    };
    const lupp_request &r = q.r;
    if (r.kind == LUPP_REQ_SOLVE) {
        const size_t n = (size_t)r.n, B = (size_t)r.batch;
        /* factors: to the caller's device lu, else staged (host lu, or a
         * host A to read) */
        if (r.lu != nullptr ? !q.dev_lu : !q.dev_A) s.fac = slot(B * n * n * 8);
        if (!q.dev_x) s.rhs = slot(B * n * 8);
        if (!q.dev_ipiv) s.piv = slot(B * n * 4);
        if (!q.dev_info) s.inf = slot(B * 4);
    } else {
        const size_t P = (size_t)r.count;
        if (!q.dev_deps) s.deps = slot(P * 48);
        if (!q.dev_sig) s.sig = slot(P * 48);
        if (!q.dev_it) s.its = slot(P * 4);
        if (!q.dev_st) s.sts = slot(P * 4);
        if (r.tangent != nullptr && !q.dev_tan) s.tan = slot(P * 288);
    }
    s.bytes = at;
}

struct Pass;

}  // namespace lupp

using namespace lupp;

struct lupp_server {
    lupp_ctx *ctx = nullptr;
    int device = 0;
    lupp_server_config cfg{};
    void *dev_base = nullptr;
    Arena *arena = nullptr;
    std::vector<hipStream_t> streams;
    int next_stream = 0;

    std::mutex mu;
    std::condition_variable cv_sched, cv_done;
    std::deque<Req *> pending;
    std::deque<Pass *> completed_q;
    std::unordered_map<int64_t, Req *> by_ticket;
    std::unordered_map<int64_t, PointSet> sets;
    int64_t next_ticket = 1, next_set = 1;
    int inflight = 0;
    bool stopping = false;
    std::thread sched;

    /* statistics */
    std::vector<double> lat_ms;
    int64_t submitted = 0, completed = 0, rejected = 0, failed = 0, passes = 0, launches = 0;
    size_t peak_bytes = 0;
    int peak_inflight = 0;
    Clock::time_point t_first_submit, t_last_done;
    bool any = false;
};

namespace lupp {

struct Pass {
    lupp_server *srv = nullptr;
    std::vector<Req *> reqs;
    int stream = 0;
};

static void pass_done(void *p)
{
    Pass *ps = static_cast<Pass *>(p);
    lupp_server *s = ps->srv;
    std::lock_guard<std::mutex> g(s->mu);
    s->completed_q.push_back(ps);
    s->cv_sched.notify_all();
}

static hipMemcpyKind dir(bool dst_dev, bool src_dev)
{
    if (dst_dev) return src_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    return src_dev ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
}

/* Buffers of a solve request during its pass. */
struct SolveBufs {
    double *fac, *rhs;
    int32_t *piv, *inf;
    bool factors;
};

static SolveBufs solve_bufs(const Req &q, char *base)
{
    const lupp_request &r = q.r;
    SolveBufs b;
    b.factors = r.lu != nullptr;
    if (q.sg.fac != kNone) b.fac = reinterpret_cast<double *>(base + q.sg.fac);
    else b.fac = const_cast<double *>(b.factors ? r.lu : r.A);
    b.rhs = q.sg.rhs != kNone ? reinterpret_cast<double *>(base + q.sg.rhs) : r.x;
    b.piv = q.sg.piv != kNone ? reinterpret_cast<int32_t *>(base + q.sg.piv) : r.ipiv;
    b.inf = q.sg.inf != kNone ? reinterpret_cast<int32_t *>(base + q.sg.inf) : r.info;
    return b;
}

static lupp_points update_points(const Req &q, char *base)
{
    const lupp_request &r = q.r;
    lupp_points p;
    p.count = r.count;
    p.ld = r.count;
    p.deps = q.sg.deps != kNone ? reinterpret_cast<double *>(base + q.sg.deps) : r.deps;
    p.state = q.set_state;
    p.sig = q.sg.sig != kNone ? reinterpret_cast<double *>(base + q.sg.sig) : r.sig;
    p.iters = q.sg.its != kNone ? reinterpret_cast<int32_t *>(base + q.sg.its) : r.iters;
    p.status = q.sg.sts != kNone ? reinterpret_cast<int32_t *>(base + q.sg.sts) : r.status;
    p.tangent = r.tangent == nullptr ? nullptr
                : (q.sg.tan != kNone ? reinterpret_cast<double *>(base + q.sg.tan) : r.tangent);
    return p;
}

/* Copies that bring a request's inputs where its kernels read them. */
static hipError_t stage_in(const Req &q, char *base, hipStream_t st)
{
    const lupp_request &r = q.r;
    hipError_t e = hipSuccess;
    if (r.kind == LUPP_REQ_SOLVE) {
        const size_t n = (size_t)r.n, B = (size_t)r.batch;
        const SolveBufs b = solve_bufs(q, base);
        if (b.fac != r.A)
            e = hipMemcpyAsync(b.fac, r.A, B * n * n * 8, dir(true, q.dev_A), st);
        if (e == hipSuccess && b.rhs != r.b)
            e = hipMemcpyAsync(b.rhs, r.b, B * n * 8, dir(true, is_device(r.b)), st);
    } else if (q.sg.deps != kNone) {
        e = hipMemcpyAsync(base + q.sg.deps, r.deps, (size_t)r.count * 48, hipMemcpyHostToDevice, st);
    }
    return e;
}

/* Copies of staged outputs to the caller's host buffers. */
static hipError_t stage_out(const Req &q, char *base, hipStream_t st)
{
    const lupp_request &r = q.r;
    hipError_t e = hipSuccess;
    auto out = [&](void *dst, size_t slot, size_t bytes) {
        if (e == hipSuccess && dst != nullptr && slot != kNone)
            e = hipMemcpyAsync(dst, base + slot, bytes, hipMemcpyDeviceToHost, st);
    };
    if (r.kind == LUPP_REQ_SOLVE) {
        const size_t n = (size_t)r.n, B = (size_t)r.batch;
        out(r.x, q.sg.rhs, B * n * 8);
        out(r.ipiv, q.sg.piv, B * n * 4);
        out(r.info, q.sg.inf, B * 4);
        if (r.lu != nullptr) out(r.lu, q.sg.fac, B * n * n * 8);
    } else {
        const size_t P = (size_t)r.count;
        out(r.sig, q.sg.sig, P * 48);
        out(r.iters, q.sg.its, P * 4);
        out(r.status, q.sg.sts, P * 4);
        out(r.tangent, q.sg.tan, P * 288);
    }
    return e;
}

static bool same_update_key(const Req &a, const Req &b)
{
    const lupp_law &x = a.law, &y = b.law;
    return x.kind == y.kind && x.E == y.E && x.nu == y.nu && x.A == y.A && x.m == y.m &&
           x.C == y.C && x.D == y.D && x.dt == y.dt && a.r.tol == b.r.tol &&
           a.r.maxit == b.r.maxit && (a.r.tangent != nullptr) == (b.r.tangent != nullptr);
}

/* Enqueue a pass: inputs, the merged launches, outputs, completion. Called
 * WITHOUT the server lock (a copy from pageable host memory may wait for
 * earlier work on the stream, whose completion callbacks take the lock).
 * Point-set state pointers are stable while their sets are busy. */
static int run_pass(lupp_server *s, Pass *ps)
{
    int launches = 0;
    hipStream_t st = s->streams[ps->stream];
    char *base0 = static_cast<char *>(s->dev_base);
    const bool merge = s->cfg.mode == LUPP_SERVE_MERGED;
    const bool grouped_ok = merge && ctx_textbook_dispatch(s->ctx);
    int pass_err = 0;

    std::vector<Req *> solves, updates;
    for (Req *q : ps->reqs) {
        char *base = base0 + q->off;
        const hipError_t e = stage_in(*q, base, st);
        if (e != hipSuccess) q->status = hip_err(e);
        else (q->r.kind == LUPP_REQ_SOLVE ? solves : updates).push_back(q);
    }

    /* solves: the small ones of the pass in one grouped solve, the others
     * one call each (a batch of kSmallBatch systems or more fills the GPU by
     * itself, and the per-size dispatch table's kernels are faster than the
     * grouped kernel's plain loads there) */
    if (!solves.empty()) {
        std::vector<lupp_group> groups;
        std::vector<uint8_t> fac;
        for (Req *q : solves) {
            const SolveBufs b = solve_bufs(*q, base0 + q->off);
            const lupp_request &r = q->r;
            if (grouped_ok && r.batch < kSmallBatch) {
                groups.push_back({r.n, r.batch, b.fac, r.n, (int64_t)r.n * r.n, b.rhs, r.n, b.piv,
                                  b.inf});
                fac.push_back(b.factors ? 1 : 0);
            } else {
                q->status = lupp_batched_solve(s->ctx, r.n, r.batch, LUPP_AOS, b.fac, r.n,
                                               (int64_t)r.n * r.n, b.rhs, r.n, b.piv, b.inf,
                                               b.factors ? 0u : LUPP_KEEP_A, st);
                ++launches;
            }
        }
        if (!groups.empty()) {
            const int rc = grouped_enqueue_each(groups.data(), fac.data(), true, (int)groups.size(),
                                                ctx_ragged_lanes(s->ctx), st);
            ++launches;
            if (rc != 0)
                for (Req *q : solves)
                    if (q->r.batch < kSmallBatch) q->status = rc;
        }
    }

    /* updates: one grouped launch per (law, tol, maxit, tangent), or one
     * call each */
    std::vector<bool> taken(updates.size(), false);
    for (size_t i = 0; i < updates.size(); ++i) {
        if (taken[i]) continue;
        std::vector<Req *> same;
        for (size_t j = i; j < updates.size(); ++j)
            if (!taken[j] && (j == i || (merge && same_update_key(*updates[i], *updates[j])))) {
                same.push_back(updates[j]);
                taken[j] = true;
            }
        std::vector<lupp_points> pts;
        for (Req *q : same) pts.push_back(update_points(*q, base0 + q->off));
        const Req &k = *same.front();
        int rc;
        if (merge)
            rc = constitutive_launch_grouped(pts.data(), (int)pts.size(), &k.law, k.r.tol, k.r.maxit, st);
        else
            rc = constitutive_update(s->ctx, &pts[0], &k.law, k.r.tol, k.r.maxit, st);
        ++launches;
        if (rc != 0)
            for (Req *q : same) q->status = rc;
    }

    for (Req *q : ps->reqs) {
        if (q->status != 0) continue;
        const hipError_t e = stage_out(*q, base0 + q->off, st);
        if (e != hipSuccess) q->status = hip_err(e);
    }
    /* completion always flows through the stream, after all of the pass */
    const hipError_t e = hipLaunchHostFunc(st, pass_done, ps);
    if (e != hipSuccess) {
        hipStreamSynchronize(st);
        pass_err = hip_err(e);
        for (Req *q : ps->reqs)
            if (q->status == 0) q->status = pass_err;
        std::lock_guard<std::mutex> g(s->mu);
        s->completed_q.push_back(ps);
    }
    return launches;
}

/* Admit waiting requests in submission order (called with the lock held): a
 * request whose point set is busy does not block the requests behind it; a
 * request whose staging does not fit in the free arena stops admission until
 * memory is released. Merged mode puts everything admitted into one pass,
 * per-request mode makes one pass per request. */
static void select_admissions(lupp_server *s, std::vector<Pass *> &out)
{
    Pass *cur = nullptr;
    for (auto it = s->pending.begin(); it != s->pending.end();) {
        if (s->inflight >= s->cfg.max_inflight) break;
        Req *q = *it;
        if (q->r.kind == LUPP_REQ_UPDATE && s->sets[q->r.set_id].busy) {
            ++it;
            continue;
        }
        size_t off = 0;
        if (!s->arena->alloc(q->sg.bytes, &off)) break;
        q->off = off;
        if (q->r.kind == LUPP_REQ_UPDATE) {
            PointSet &ps = s->sets[q->r.set_id];
            ps.busy = true;
            q->set_state = ps.state;
        }
        ++s->inflight;
        s->peak_inflight = std::max(s->peak_inflight, s->inflight);
        s->peak_bytes = std::max(s->peak_bytes, s->arena->used());
        it = s->pending.erase(it);
        if (cur == nullptr || s->cfg.mode != LUPP_SERVE_MERGED) {
            cur = new Pass;
            cur->srv = s;
            cur->stream = s->next_stream;
            s->next_stream = (s->next_stream + 1) % (int)s->streams.size();
            out.push_back(cur);
        }
        cur->reqs.push_back(q);
    }
}

static void finish(lupp_server *s, Req *q, Clock::time_point now)
{
    q->t_done = now;
    s->arena->release(q->off, q->sg.bytes);
    if (q->r.kind == LUPP_REQ_UPDATE) s->sets[q->r.set_id].busy = false;
    --s->inflight;
    q->done = true;
    const double ms = std::chrono::duration<double, std::milli>(q->t_done - q->t_submit).count();
    if (q->status == 0) {
        s->lat_ms.push_back(ms);
        ++s->completed;
    } else {
        ++s->failed;
    }
    s->t_last_done = q->t_done;
}

static void scheduler_loop(lupp_server *s)
{
    hipSetDevice(s->device);
    std::vector<Pass *> batch;
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        while (!s->completed_q.empty()) {
            Pass *ps = s->completed_q.front();
            s->completed_q.pop_front();
            const Clock::time_point now = Clock::now();
            for (Req *q : ps->reqs) finish(s, q, now);
            delete ps;
            s->cv_done.notify_all();
        }
        batch.clear();
        select_admissions(s, batch);
        if (!batch.empty()) {
            s->passes += (int64_t)batch.size();
            lk.unlock();
            int launches = 0;
            for (Pass *ps : batch) launches += run_pass(s, ps);
            lk.lock();
            s->launches += launches;
            continue;
        }
        if (s->stopping && s->pending.empty() && s->inflight == 0 && s->completed_q.empty()) break;
        if (!s->completed_q.empty()) continue;
        s->cv_sched.wait(lk);
    }
}

}  // namespace lupp

extern "C" {

int lupp_server_create(lupp_ctx *ctx, const lupp_server_config *cfg, lupp_server **out)
{
    if (out == nullptr) return -3;
    *out = nullptr;
    if (ctx == nullptr) return -1;
    if (cfg == nullptr || cfg->max_inflight < 1 || cfg->streams < 1 || cfg->streams > 64 ||
        cfg->hbm_budget_bytes < 0 ||
        (cfg->mode != LUPP_SERVE_MERGED && cfg->mode != LUPP_SERVE_PER_REQUEST))
        return -2;
    int dev = 0;
    lupp_get_device(ctx, &dev);
    int cur = 0;
    hipGetDevice(&cur);
    hipSetDevice(dev);
    lupp_server *s = new (std::nothrow) lupp_server;
    if (s == nullptr) return LUPP_E_NOMEM;
    /* the scheduler thread uses a context of its own on the same device,
     * with the caller's settings */
    const int crc = lupp_create(&s->ctx, dev);
    if (crc != 0) {
        delete s;
        hipSetDevice(cur);
        return crc;
    }
    ctx_copy_settings(s->ctx, ctx);
    s->device = dev;
    s->cfg = *cfg;
    size_t budget = (size_t)cfg->hbm_budget_bytes;
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        hipMemGetInfo(&fr, &tot);
        budget = fr / 4;
    }
    hipError_t e = hipMalloc(&s->dev_base, budget);
    if (e != hipSuccess) {
        lupp_destroy(s->ctx);
        delete s;
        hipSetDevice(cur);
        return e == hipErrorOutOfMemory ? LUPP_E_NOMEM : hip_err(e);
    }
    s->arena = new Arena(budget);
    s->cfg.hbm_budget_bytes = (int64_t)budget;
    for (int i = 0; i < cfg->streams; ++i) {
        hipStream_t st;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e != hipSuccess) break;
        s->streams.push_back(st);
    }
    if (e != hipSuccess) {
        for (auto st : s->streams) hipStreamDestroy(st);
        hipFree(s->dev_base);
        delete s->arena;
        lupp_destroy(s->ctx);
        delete s;
        hipSetDevice(cur);
        return hip_err(e);
    }
    s->sched = std::thread(scheduler_loop, s);
    hipSetDevice(cur);
    *out = s;
    return 0;
}

void lupp_server_destroy(lupp_server *s)
{
    if (s == nullptr) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stopping = true;
        s->cv_sched.notify_all();
    }
    s->sched.join();
    int cur = 0;
    hipGetDevice(&cur);
    hipSetDevice(s->device);
    for (auto st : s->streams) {
        hipStreamSynchronize(st);
        hipStreamDestroy(st);
    }
    for (auto &kv : s->sets) hipFree(kv.second.state);
    for (auto &kv : s->by_ticket) delete kv.second;
    hipFree(s->dev_base);
    delete s->arena;
    lupp_destroy(s->ctx);
    hipSetDevice(cur);
    delete s;
}

int lupp_server_add_points(lupp_server *s, int kind, int64_t count, const double *state,
                           int64_t *set_id)
{
    if (s == nullptr) return -1;
    if (kind != LUPP_LAW_NORTON7 && kind != LUPP_LAW_NORTON_AF13) return -2;
    if (count < 1) return -3;
    if (set_id == nullptr) return -5;
    int cur = 0;
    hipGetDevice(&cur);
    hipSetDevice(s->device);
    PointSet ps;
    ps.kind = kind;
    ps.count = count;
    const size_t bytes = (size_t)count * kind * 8;
    hipError_t e = hipMalloc(&ps.state, bytes);
    if (e == hipSuccess) {
        if (state != nullptr) e = hipMemcpy(ps.state, state, bytes, dir(true, is_device(state)));
        else e = hipMemset(ps.state, 0, bytes);
    }
    hipSetDevice(cur);
    if (e != hipSuccess) {
        hipFree(ps.state);
        return e == hipErrorOutOfMemory ? LUPP_E_NOMEM : hip_err(e);
    }
    std::lock_guard<std::mutex> g(s->mu);
    *set_id = s->next_set++;
    s->sets[*set_id] = ps;
    return 0;
}

int lupp_server_read_points(lupp_server *s, int64_t set_id, double *state)
{
    if (s == nullptr) return -1;
    if (state == nullptr) return -3;
    PointSet ps;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        auto it = s->sets.find(set_id);
        if (it == s->sets.end()) return -2;
        /* wait until no request of this set is queued or running */
        for (;;) {
            bool busy = it->second.busy;
            for (Req *q : s->pending)
                if (q->r.kind == LUPP_REQ_UPDATE && q->r.set_id == set_id) busy = true;
            if (!busy) break;
            s->cv_done.wait(lk);
            it = s->sets.find(set_id);
        }
        ps = it->second;
    }
    int cur = 0;
    hipGetDevice(&cur);
    hipSetDevice(s->device);
    const hipError_t e =
        hipMemcpy(state, ps.state, (size_t)ps.count * ps.kind * 8, dir(is_device(state), true));
    hipSetDevice(cur);
    return hip_err(e);
}

int64_t lupp_server_submit(lupp_server *s, const lupp_request *r)
{
    if (s == nullptr) return -1;
    if (r == nullptr) return -2;
    if (r->kind == LUPP_REQ_SOLVE) {
        if (r->n < 1 || r->n > 32 || r->batch < 1 || r->batch > 0x7fffffff || r->A == nullptr ||
            r->b == nullptr || r->x == nullptr)
            return -2;
    } else if (r->kind == LUPP_REQ_UPDATE) {
        if (r->law == nullptr || r->deps == nullptr || r->maxit < 0 || r->maxit > LUPP_MAXIT_LIMIT ||
            !(r->tol >= 0.0))
            return -2;
    } else {
        return -2;
    }
    Req *q = new (std::nothrow) Req;
    if (q == nullptr) return LUPP_E_NOMEM;
    q->r = *r;
    /* where the buffers live decides what is staged (outside the lock: the
     * runtime queries may take a while) */
    if (r->kind == LUPP_REQ_SOLVE) {
        q->dev_A = is_device(r->A);
        q->dev_x = is_device(r->x);
        q->dev_lu = is_device(r->lu);
        q->dev_ipiv = is_device(r->ipiv);
        q->dev_info = is_device(r->info);
    } else {
        q->dev_deps = is_device(r->deps);
        q->dev_sig = is_device(r->sig);
        q->dev_it = is_device(r->iters);
        q->dev_st = is_device(r->status);
        q->dev_tan = is_device(r->tangent);
    }
    std::lock_guard<std::mutex> g(s->mu);
    if (r->kind == LUPP_REQ_UPDATE) {
        auto it = s->sets.find(r->set_id);
        if (it == s->sets.end() || it->second.count != r->count || it->second.kind != r->law->kind) {
            delete q;
            return -2;
        }
        q->law = *r->law;
        q->r.law = &q->law;
    }
    plan_staging(*q);
    if (q->sg.bytes > s->arena->size()) {
        ++s->rejected;
        delete q;
        return LUPP_E_NOMEM;
    }
    q->ticket = s->next_ticket++;
    q->t_submit = Clock::now();
    if (!s->any) {
        s->any = true;
        s->t_first_submit = q->t_submit;
    }
    ++s->submitted;
    s->by_ticket[q->ticket] = q;
    s->pending.push_back(q);
    s->cv_sched.notify_all();
    return q->ticket;
}

int lupp_server_poll(lupp_server *s, int64_t ticket)
{
    if (s == nullptr) return -1;
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->by_ticket.find(ticket);
    if (it == s->by_ticket.end()) return -2;
    return it->second->done ? 1 : 0;
}

int lupp_server_wait(lupp_server *s, int64_t ticket, double *latency_ms)
{
    if (s == nullptr) return -1;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->by_ticket.find(ticket);
    if (it == s->by_ticket.end()) return -2;
    Req *q = it->second;
    s->cv_done.wait(lk, [&] { return q->done; });
    if (latency_ms)
        *latency_ms = std::chrono::duration<double, std::milli>(q->t_done - q->t_submit).count();
    const int st = q->status;
    s->by_ticket.erase(it);
    delete q;
    return st;
}

int lupp_server_get_stats(lupp_server *s, lupp_server_stats *o)
{
    if (s == nullptr) return -1;
    if (o == nullptr) return -2;
    std::lock_guard<std::mutex> g(s->mu);
    std::memset(o, 0, sizeof(*o));
    o->submitted = s->submitted;
    o->completed = s->completed;
    o->rejected = s->rejected;
    o->failed = s->failed;
    o->inflight = s->inflight;
    o->queued = (int64_t)s->pending.size();
    o->peak_bytes = (int64_t)s->peak_bytes;
    o->peak_inflight = s->peak_inflight;
    o->budget_bytes = s->cfg.hbm_budget_bytes;
    o->passes = s->passes;
    o->launches = s->launches;
    if (!s->lat_ms.empty()) {
        std::vector<double> v = s->lat_ms;
        std::sort(v.begin(), v.end());
        auto pct = [&](double p) {
            const size_t i = (size_t)std::min<double>((double)v.size() - 1, p * (double)(v.size() - 1) + 0.5);
            return v[i];
        };
        o->p50_ms = pct(0.50);
        o->p99_ms = pct(0.99);
        double sum = 0;
        for (double x : v) sum += x;
        o->mean_ms = sum / (double)v.size();
        o->max_ms = v.back();
    }
    if (s->any && s->completed > 0)
        o->elapsed_s = std::chrono::duration<double>(s->t_last_done - s->t_first_submit).count();
    return 0;
}

int lupp_server_reset_stats(lupp_server *s)
{
    if (s == nullptr) return -1;
    std::lock_guard<std::mutex> g(s->mu);
    s->lat_ms.clear();
    s->submitted = s->completed = s->rejected = s->failed = s->passes = s->launches = 0;
    s->peak_bytes = s->arena->used();
    s->peak_inflight = s->inflight;
    s->any = false;
    return 0;
}

}  // extern "C"
