/* Serving loop: continuous batching of standalone-solve and constitutive-
 * update requests under an HBM budget.
 *
 * A request names its inputs and outputs by pointer (host or device). The
 * server owns a device arena the size of its HBM budget; a request is
 * admitted when its footprint fits in the arena and an in-flight slot is
 * free, its inputs are copied into arena buffers, its kernels run on one of
 * the server's streams (so admitted requests overlap on the GPU), its results
 * are copied out, and its arena range is released, which admits the next
 * waiting requests. Integration-point state lives on the device in
 * registered point sets that update requests advance; requests on the same
 * set run in submission order. Latency is measured from submit to the
 * completion of the request's last copy.
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

#include "internal.h"

namespace lupp {

using Clock = std::chrono::steady_clock;

/* first-fit allocator over [0, size) with 256-byte granules */
class Arena {
  public:
    explicit Arena(size_t size) : size_(size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = (bytes + 255) & ~(size_t)255;
        if (bytes == 0) bytes = 256;
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
        if (bytes == 0) bytes = 256;
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
    double *state = nullptr;  /* [kind][count] device, owned */
    bool busy = false;        /* a request on this set is in flight */
};

struct Req {
    int64_t ticket = 0;
    lupp_request r{};
    lupp_law law{};
    size_t bytes = 0, off = 0;
    int stream = 0;
    Clock::time_point t_submit, t_admit, t_done;
    int status = 0;  /* 0 ok or a lupp error */
    bool done = false;
    struct lupp_server *srv = nullptr;
};

static size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

/* device bytes a request needs in the arena */
static size_t footprint(const lupp_request &r)
{
    if (r.kind == LUPP_REQ_SOLVE) {
        const size_t n = (size_t)r.n, B = (size_t)r.batch;
        return round256(B * n * n * 8) + round256(B * n * 8) + round256(B * n * 4) +
               round256(B * 4);
    }
    const size_t P = (size_t)r.count;
    return round256(P * 6 * 8) * 2 + round256(P * 4) * 2 + (r.tangent ? round256(P * 36 * 8) : 0);
}

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
    std::deque<Req *> completed_q;
    std::unordered_map<int64_t, Req *> by_ticket;
    std::unordered_map<int64_t, PointSet> sets;
    int64_t next_ticket = 1, next_set = 1;
    int inflight = 0;
    bool stopping = false;
    std::thread sched;

    /* statistics */
    std::vector<double> lat_ms;
    int64_t submitted = 0, completed = 0, rejected = 0, failed = 0;
    size_t peak_bytes = 0;
    int peak_inflight = 0;
    Clock::time_point t_first_submit, t_last_done;
    bool any = false;
    double busy_bytes = 0;
};

namespace lupp {

static void host_done(void *p)
{
    Req *q = static_cast<Req *>(p);
    lupp_server *s = q->srv;
    std::lock_guard<std::mutex> g(s->mu);
    s->completed_q.push_back(q);
    s->cv_sched.notify_all();
}

static hipMemcpyKind kind_of(const void *p)
{
    hipPointerAttribute_t a;
    std::memset(&a, 0, sizeof(a));
    if (hipPointerGetAttributes(&a, p) == hipSuccess && a.type == hipMemoryTypeDevice)
        return hipMemcpyDeviceToDevice;
    (void)hipGetLastError();
    return hipMemcpyHostToDevice;
}

static hipMemcpyKind kind_out(const void *p)
{
    return kind_of(p) == hipMemcpyDeviceToDevice ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
}

/* Enqueue one admitted request on its stream. Called WITHOUT the server lock:
 * a copy from pageable host memory may wait for earlier work on the stream,
 * whose completion callbacks take the lock. Point-set state pointers are
 * stable while the set has a request in flight. */
static int launch_req(lupp_server *s, Req *q, double *set_state)
{
    hipStream_t st = s->streams[q->stream];
    char *base = static_cast<char *>(s->dev_base) + q->off;
    const lupp_request &r = q->r;
    hipError_t e = hipSuccess;
    int rc = 0;
    if (r.kind == LUPP_REQ_SOLVE) {
        const size_t n = (size_t)r.n, B = (size_t)r.batch;
        const size_t oA = 0, ob = round256(B * n * n * 8), op = ob + round256(B * n * 8),
                     oi = op + round256(B * n * 4);
        double *dA = reinterpret_cast<double *>(base + oA);
        double *db = reinterpret_cast<double *>(base + ob);
        int32_t *dp = reinterpret_cast<int32_t *>(base + op);
        int32_t *di = reinterpret_cast<int32_t *>(base + oi);
        e = hipMemcpyAsync(dA, r.A, B * n * n * 8, kind_of(r.A), st);
        if (e == hipSuccess) e = hipMemcpyAsync(db, r.b, B * n * 8, kind_of(r.b), st);
        if (e != hipSuccess) return hip_err(e);
        rc = lupp_batched_solve(s->ctx, r.n, r.batch, LUPP_AOS, dA, r.n, r.n * r.n, db, r.n, dp, di,
                                r.lu == nullptr ? LUPP_KEEP_A : 0u, st);
        if (rc != 0) return rc;
        e = hipMemcpyAsync(r.x, db, B * n * 8, kind_out(r.x), st);
        if (e == hipSuccess && r.ipiv) e = hipMemcpyAsync(r.ipiv, dp, B * n * 4, kind_out(r.ipiv), st);
        if (e == hipSuccess && r.info) e = hipMemcpyAsync(r.info, di, B * 4, kind_out(r.info), st);
        if (e == hipSuccess && r.lu) e = hipMemcpyAsync(r.lu, dA, B * n * n * 8, kind_out(r.lu), st);
    } else {
        const size_t P = (size_t)r.count;
        double *dd = reinterpret_cast<double *>(base);
        double *dsig = reinterpret_cast<double *>(base + round256(P * 48));
        int32_t *dit = reinterpret_cast<int32_t *>(base + 2 * round256(P * 48));
        int32_t *dst = reinterpret_cast<int32_t *>(base + 2 * round256(P * 48) + round256(P * 4));
        double *dtan = r.tangent ? reinterpret_cast<double *>(base + 2 * round256(P * 48) +
                                                              2 * round256(P * 4))
                                 : nullptr;
        e = hipMemcpyAsync(dd, r.deps, P * 48, kind_of(r.deps), st);
        if (e != hipSuccess) return hip_err(e);
        lupp_points pts{(int64_t)P, (int64_t)P, dd, set_state, dsig, dit, dst, dtan};
        rc = constitutive_update(s->ctx, &pts, &q->law, r.tol, r.maxit, st);
        if (rc != 0) return rc;
        if (r.sig) e = hipMemcpyAsync(r.sig, dsig, P * 48, kind_out(r.sig), st);
        if (e == hipSuccess && r.iters) e = hipMemcpyAsync(r.iters, dit, P * 4, kind_out(r.iters), st);
        if (e == hipSuccess && r.status)
            e = hipMemcpyAsync(r.status, dst, P * 4, kind_out(r.status), st);
        if (e == hipSuccess && r.tangent)
            e = hipMemcpyAsync(r.tangent, dtan, P * 36 * 8, kind_out(r.tangent), st);
    }
    return hip_err(e);
}

/* Choose what to admit, in submission order (called with the lock held): a
 * request whose point set is busy does not block the requests behind it; a
 * request that does not fit in the free arena stops admission until memory
 * is released. */
static void select_admissions(lupp_server *s, std::vector<std::pair<Req *, double *>> &out)
{
    for (auto it = s->pending.begin(); it != s->pending.end();) {
        if (s->inflight >= s->cfg.max_inflight) break;
        Req *q = *it;
        if (q->r.kind == LUPP_REQ_UPDATE && s->sets[q->r.set_id].busy) {
            ++it;
            continue;
        }
        size_t off = 0;
        if (!s->arena->alloc(q->bytes, &off)) break;
        q->off = off;
        q->stream = s->next_stream;
        s->next_stream = (s->next_stream + 1) % (int)s->streams.size();
        q->t_admit = Clock::now();
        double *state = nullptr;
        if (q->r.kind == LUPP_REQ_UPDATE) {
            PointSet &ps = s->sets[q->r.set_id];
            ps.busy = true;
            state = ps.state;
        }
        ++s->inflight;
        s->peak_inflight = std::max(s->peak_inflight, s->inflight);
        s->peak_bytes = std::max(s->peak_bytes, s->arena->used());
        it = s->pending.erase(it);
        out.emplace_back(q, state);
    }
}

static void finish(lupp_server *s, Req *q)
{
    q->t_done = Clock::now();
    s->arena->release(q->off, q->bytes);
    if (q->r.kind == LUPP_REQ_UPDATE) s->sets[q->r.set_id].busy = false;
    --s->inflight;
    q->done = true;
    const double ms = std::chrono::duration<double, std::milli>(q->t_done - q->t_submit).count();
    if (q->status == 0) {
        s->lat_ms.push_back(ms);
        ++s->completed;
        s->busy_bytes += (double)q->bytes;
    } else {
        ++s->failed;
    }
    s->t_last_done = q->t_done;
}

static void scheduler_loop(lupp_server *s)
{
    hipSetDevice(s->device);
    std::vector<std::pair<Req *, double *>> batch;
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        while (!s->completed_q.empty()) {
            Req *q = s->completed_q.front();
            s->completed_q.pop_front();
            finish(s, q);
            s->cv_done.notify_all();
        }
        batch.clear();
        select_admissions(s, batch);
        if (!batch.empty()) {
            lk.unlock();
            for (auto &qs : batch) {
                Req *q = qs.first;
                q->status = launch_req(s, q, qs.second);
                /* completion always flows through the stream, after the work
                 * already enqueued for the request */
                hipError_t e = hipLaunchHostFunc(s->streams[q->stream], host_done, q);
                if (e != hipSuccess) {
                    hipStreamSynchronize(s->streams[q->stream]);
                    if (q->status == 0) q->status = hip_err(e);
                    std::lock_guard<std::mutex> g(s->mu);
                    s->completed_q.push_back(q);
                }
            }
            lk.lock();
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
        cfg->hbm_budget_bytes < 0)
        return -2;
    int dev = 0;
    lupp_get_device(ctx, &dev);
    int cur = 0;
    hipGetDevice(&cur);
    hipSetDevice(dev);
    lupp_server *s = new (std::nothrow) lupp_server;
    if (s == nullptr) return LUPP_E_NOMEM;
    /* the scheduler thread uses a context of its own on the same device */
    const int crc = lupp_create(&s->ctx, dev);
    if (crc != 0) {
        delete s;
        hipSetDevice(cur);
        return crc;
    }
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
        if (state != nullptr) e = hipMemcpy(ps.state, state, bytes, kind_of(state));
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
    const hipError_t e = hipMemcpy(state, ps.state, (size_t)ps.count * ps.kind * 8, kind_out(state));
    hipSetDevice(cur);
    return hip_err(e);
}

int64_t lupp_server_submit(lupp_server *s, const lupp_request *r)
{
    if (s == nullptr) return -1;
    if (r == nullptr) return -2;
    if (r->kind == LUPP_REQ_SOLVE) {
        if (r->n < 1 || r->n > 32 || r->batch < 1 || r->A == nullptr || r->b == nullptr ||
            r->x == nullptr)
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
    q->srv = s;
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
    q->bytes = footprint(q->r);
    if (q->bytes > s->arena->size()) {
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
    s->submitted = s->completed = s->rejected = s->failed = 0;
    s->peak_bytes = s->arena->used();
    s->peak_inflight = s->inflight;
    s->any = false;
    return 0;
}

}  // extern "C"
