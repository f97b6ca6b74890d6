// Serving loop: continuous batching of independent interpolation requests
// of mixed size and tolerance on one GPU.
//
// A scheduler thread owns every device object.  Each pass it (1) retires
// requests whose completion event has fired, returning their plan to the
// cache and their slot to the free list, and (2) admits queued requests in
// arrival order while a slot is free and the request's device footprint
// fits the HBM budget (evicting idle cached plans, least recently used
// first, when that makes it fit).  An admitted request is enqueued on its
// slot's stream: host-to-device copies, setpts, exec, device-to-host copy,
// completion event.  Slots run concurrently, so requests that arrive while
// others are on the GPU overlap with them.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "nufft2.h"
#include "nufft2_internal.hpp"
#include "plan_state.hpp"

#define NUFFT2_API extern "C" __attribute__((visibility("default")))

namespace {

constexpr uint64_t kDefaultBudget = 16ull << 30;
constexpr int kDefaultInflight = 8;
constexpr int kMaxInflight = 64;
constexpr size_t kPlanTableSlack = 1u << 20;  // tables, counters, bins

struct PlanKey {
    int prec, F;
    int64_t Kt, Kp;
    double eps;
    bool operator==(const PlanKey &o) const
    {
        return prec == o.prec && F == o.F && Kt == o.Kt && Kp == o.Kp && eps == o.eps;
    }
};

struct CachedPlan {
    PlanKey key;
    nufft2_handle h = nullptr;
    bool busy = false;
    uint64_t last_use = 0;
    size_t bytes = 0;  // reserved for it: the plan's own workspace count
};

struct Request {
    uint64_t id = 0;
    nufft2_request r{};
    PlanKey key{};
    size_t plan_bytes = 0;  // estimated footprint of a new plan for it
    size_t buf_bytes = 0;   // its input and output buffers
    nufft2_status status = NUFFT2_OK;
    double latency = 0;
    double t_admit = 0;     // server clock when its work was enqueued
    bool done = false;
};

struct Slot {
    hipStream_t stream = nullptr;
    // recorded before the host-to-device copies, after them, after the
    // kernels, and after the device-to-host copy (completion)
    hipEvent_t start = nullptr, h2d = nullptr, kern = nullptr, done = nullptr;
    void *d_buf = nullptr;  // coeffs | phi | theta | out
    size_t cap = 0;
    void *h_stage = nullptr;  // pinned; outputs of requests without out_host
    size_t stage_cap = 0;
    Request *req = nullptr;
    CachedPlan *plan = nullptr;
};

size_t csize(int prec) { return prec == NUFFT2_FP32 ? 2 * sizeof(float) : 2 * sizeof(double); }

int64_t fine_size(int64_t K, int w)
{
    int64_t n = 2 * K;
    if (n < 2 * w) n = 2 * w;
    if (n < 32) n = 32;
    int64_t p = 1;
    while (p < n) p <<= 1;
    return p;
}

// Device bytes a plan for this request will hold (fine grid, theta-pass
// buffer, point records), as nufft2_plan and nufft2_setpts size them.
size_t plan_estimate(const nufft2_request &r)
{
    int32_t w = 0;
    double beta = 0;
    if (nufft2_kernel_params((nufft2_prec)r.prec, r.eps, &w, &beta) != NUFFT2_OK) return 0;
    const int64_t nft = fine_size(r.n_modes_theta, w), nfp = fine_size(r.n_modes_phi, w);
    const size_t cs = csize(r.prec), rs = cs / 2;
    return cs * (size_t)r.n_fields * nft * (size_t)(nfp + r.n_modes_phi) +
           (size_t)r.n_pts * (sizeof(int2) + 2 * rs + 8 + sizeof(int32_t)) + kPlanTableSlack;
}

size_t buffer_bytes(const nufft2_request &r)
{
    const size_t cs = csize(r.prec);
    return cs * (size_t)r.n_fields * r.n_modes_theta * r.n_modes_phi + 2 * sizeof(double) * (size_t)r.n_pts +
           cs * (size_t)r.n_fields * r.n_pts;
}

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Device bytes per point of a plan's point workspaces (as nufft2_setpts
// grows them): keyrank, record, permutation.
size_t point_bytes(int prec)
{
    const size_t rs = csize(prec) / 2;
    return sizeof(int2) + 2 * rs + 8 + sizeof(int32_t);
}

}  // namespace

struct nufft2_server_s {
    uint64_t budget = 0;
    int max_inflight = 0;
    int device = 0;
    std::chrono::steady_clock::time_point t0;

    // shared with the API threads, under mu
    std::mutex mu;
    std::condition_variable cv_work;  // new submissions, stop
    std::condition_variable cv_done;  // a request completed
    std::deque<Request *> queue;
    std::vector<Request *> all;       // every request ever submitted (owned)
    uint64_t next_id = 1;
    int inflight = 0, max_inflight_seen = 0;
    bool stop = false;
    int64_t completed = 0, failed = 0, pf = 0, created = 0, evicted = 0;
    std::vector<double> latencies;
    // per completed request: queue wait (arrival to admission), host-to-
    // device copies, kernels, device-to-host copy (seconds)
    std::vector<double> t_queue, t_h2d, t_kern, t_d2h;
    double first_arrival = 1e300, last_completion = 0;
    size_t high_water = 0;

    // the scheduler thread's own state (no lock)
    std::vector<Slot> slots;
    std::vector<CachedPlan *> plans;
    std::vector<std::pair<void *, size_t>> retired;  // buffers to free once the device is idle
    uint64_t tick = 0;
    size_t reserved = 0;
    int busy = 0;  // slots with a request
    std::thread worker;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    void reserve(size_t b)
    {
        reserved += b;
        if (reserved > high_water) {
            std::lock_guard<std::mutex> lk(mu);
            high_water = std::max(high_water, reserved);
        }
    }
};

namespace {

// ---- the scheduler thread's side ------------------------------------------

void evict_plan(nufft2_server_s *s, CachedPlan *cp)
{
    (void)nufft2_destroy(cp->h);
    s->reserved -= cp->bytes;
    s->plans.erase(std::find(s->plans.begin(), s->plans.end(), cp));
    delete cp;
    std::lock_guard<std::mutex> lk(s->mu);
    s->evicted += 1;
}

void free_retired(nufft2_server_s *s)
{
    for (auto &b : s->retired) {
        (void)hipFree(b.first);
        s->reserved -= b.second;
    }
    s->retired.clear();
}

// Make `need` bytes fit under the budget: free retired buffers, destroy
// idle plans (least recently used first), then free the buffers of idle
// slots other than `keep`.  These frees synchronise the device, so they only
// happen under memory pressure.  Returns whether it fits.  (A request that
// passed the submit check and needs a new plan always fits once nothing else
// is in flight; start() falls back to that when a cached plan's growth does
// not fit beside the plan.)
bool make_room(nufft2_server_s *s, size_t need, const Slot *keep)
{
    if (s->reserved + need > s->budget) free_retired(s);
    while (s->reserved + need > s->budget) {
        CachedPlan *lru = nullptr;
        for (CachedPlan *cp : s->plans)
            if (!cp->busy && (!lru || cp->last_use < lru->last_use)) lru = cp;
        if (lru) {
            evict_plan(s, lru);
            continue;
        }
        Slot *idle = nullptr;
        for (Slot &sl : s->slots)
            if (&sl != keep && !sl.req && sl.cap > 0) {
                idle = &sl;
                break;
            }
        if (!idle) return false;
        (void)hipFree(idle->d_buf);
        s->reserved -= idle->cap;
        idle->d_buf = nullptr;
        idle->cap = 0;
    }
    return true;
}

enum class Start { kWait, kStarted, kFailed };

// Start request q on free slot sl.  kWait: no room yet (nothing changed);
// kFailed: *st holds the request's error.
Start start(nufft2_server_s *s, Slot &sl, Request *q, nufft2_status *st)
{
    const nufft2_request &r = q->r;
    CachedPlan *cp = nullptr;
    for (CachedPlan *c : s->plans)
        if (!c->busy && c->key == q->key) {
            cp = c;
            break;
        }
    const size_t need_buf = round_up(q->buf_bytes, 1u << 20);
    const size_t grow = need_buf > sl.cap ? need_buf : 0;  // a new buffer
    if (grow && sl.d_buf) {
        // the slot's old buffer is idle (its request has completed): it
        // retires now, reserved until make_room or an idle device frees it
        s->retired.push_back({sl.d_buf, sl.cap});
        sl.d_buf = nullptr;
        sl.cap = 0;
    }
    // a cached plan grows its point workspaces in setpts when this request
    // has more points than it held before
    const size_t pts_grow =
        cp && r.n_pts > cp->h->pts_cap ? (size_t)(r.n_pts - cp->h->pts_cap) * point_bytes(r.prec) : 0;
    size_t need = grow + (cp ? pts_grow : q->plan_bytes);
    if (cp) cp->busy = true;  // not a candidate for eviction while making room
    if (!make_room(s, need, &sl)) {
        if (cp) cp->busy = false;
        if (s->busy > 0) return Start::kWait;  // room comes back as in-flight work completes
        // nothing in flight, so nothing else will free memory: drop the
        // cached plan and fall back to a new one, which the submit check
        // guarantees fits an otherwise empty budget
        if (cp) {
            evict_plan(s, cp);
            cp = nullptr;
            need = grow + q->plan_bytes;
        }
        if (!make_room(s, need, &sl)) {
            *st = NUFFT2_ERR_ALLOC;
            return Start::kFailed;
        }
    }
    auto fail = [&](nufft2_status e) {
        if (cp) cp->busy = false;
        *st = e;
        return Start::kFailed;
    };
    if (grow) {
        void *nb = nullptr;
        if (hipMalloc(&nb, need_buf) != hipSuccess) {
            (void)hipGetLastError();
            return fail(NUFFT2_ERR_ALLOC);
        }
        sl.d_buf = nb;
        sl.cap = need_buf;
        s->reserve(need_buf);
    }
    const size_t cs = csize(r.prec);
    const size_t out_bytes = cs * (size_t)r.n_fields * r.n_pts;
    if (!r.out_host && out_bytes > sl.stage_cap) {
        // pinned host memory: not part of the device budget
        if (sl.h_stage) (void)hipHostFree(sl.h_stage);
        sl.h_stage = nullptr;
        sl.stage_cap = 0;
        if (hipHostMalloc(&sl.h_stage, out_bytes, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return fail(NUFFT2_ERR_ALLOC);
        }
        sl.stage_cap = out_bytes;
    }
    if (!cp) {
        cp = new (std::nothrow) CachedPlan();
        if (!cp) return fail(NUFFT2_ERR_ALLOC);
        cp->key = q->key;
        nufft2_status e = nufft2_plan((nufft2_prec)r.prec, r.n_modes_theta, r.n_modes_phi, r.n_fields, r.eps,
                                      nullptr, sl.stream, &cp->h);
        if (e != NUFFT2_OK) {
            delete cp;
            cp = nullptr;
            return fail(e);
        }
        // reserved: the estimate, which also covers the point workspaces
        // setpts will add; corrected to the plan's own count after setpts
        cp->bytes = q->plan_bytes;
        cp->busy = true;
        s->reserve(cp->bytes);
        s->plans.push_back(cp);
        std::lock_guard<std::mutex> lk(s->mu);
        s->created += 1;
    }
    cp->h->stream = sl.stream;  // the plan is idle: its earlier work has completed
    const size_t c_bytes = cs * (size_t)r.n_fields * r.n_modes_theta * r.n_modes_phi;
    const size_t p_bytes = sizeof(double) * (size_t)r.n_pts;
    char *base = (char *)sl.d_buf;
    void *d_coeffs = base, *d_phi = base + c_bytes, *d_theta = base + c_bytes + p_bytes,
         *d_out = base + c_bytes + 2 * p_bytes;
    nufft2_status e = NUFFT2_OK;
    q->t_admit = s->now();
    if (hipEventRecord(sl.start, sl.stream) != hipSuccess ||
        hipMemcpyAsync(d_coeffs, r.coeffs_host, c_bytes, hipMemcpyHostToDevice, sl.stream) != hipSuccess ||
        hipMemcpyAsync(d_phi, r.phi_host, p_bytes, hipMemcpyHostToDevice, sl.stream) != hipSuccess ||
        hipMemcpyAsync(d_theta, r.theta_host, p_bytes, hipMemcpyHostToDevice, sl.stream) != hipSuccess ||
        hipEventRecord(sl.h2d, sl.stream) != hipSuccess)
        e = NUFFT2_ERR_HIP;
    if (e == NUFFT2_OK) e = nufft2_setpts(cp->h, r.n_pts, (const double *)d_phi, (const double *)d_theta);
    if (e == NUFFT2_OK) {
        // the plan's own count from now on (setpts may have grown it)
        const size_t own = cp->h->ws_bytes;
        if (own > cp->bytes) s->reserve(own - cp->bytes);
        else s->reserved -= cp->bytes - own;
        cp->bytes = own;
    }
    if (e == NUFFT2_OK) e = nufft2_exec(cp->h, d_coeffs, d_out);
    if (e == NUFFT2_OK && (hipEventRecord(sl.kern, sl.stream) != hipSuccess ||
                           hipMemcpyAsync(r.out_host ? r.out_host : sl.h_stage, d_out, out_bytes,
                                          hipMemcpyDeviceToHost, sl.stream) != hipSuccess ||
                           hipEventRecord(sl.done, sl.stream) != hipSuccess))
        e = NUFFT2_ERR_HIP;
    if (e != NUFFT2_OK) {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(sl.stream);
        evict_plan(s, cp);  // its state is unknown
        *st = e;
        return Start::kFailed;
    }
    sl.req = q;
    sl.plan = cp;
    s->busy += 1;
    return Start::kStarted;
}

// Stage durations of a request whose completion event has fired (seconds;
// -1 where an interval cannot be read).
struct StageTimes {
    double h2d = -1, kern = -1, d2h = -1;
};
StageTimes stage_times(const Slot &sl)
{
    StageTimes t;
    float ms = 0;
    if (hipEventElapsedTime(&ms, sl.start, sl.h2d) == hipSuccess) t.h2d = 1e-3 * ms;
    if (hipEventElapsedTime(&ms, sl.h2d, sl.kern) == hipSuccess) t.kern = 1e-3 * ms;
    if (hipEventElapsedTime(&ms, sl.kern, sl.done) == hipSuccess) t.d2h = 1e-3 * ms;
    (void)hipGetLastError();
    return t;
}

// Record a finished request (lock held).
void record(nufft2_server_s *s, Request *q, nufft2_status st, double t_done, const StageTimes *tm = nullptr)
{
    q->status = st;
    q->latency = t_done - q->r.t_arrival;
    q->done = true;
    if (st == NUFFT2_OK) {
        s->completed += 1;
        s->pf += (int64_t)q->r.n_fields * q->r.n_pts;
        s->latencies.push_back(q->latency);
        s->t_queue.push_back(q->t_admit - q->r.t_arrival);
        if (tm && tm->h2d >= 0 && tm->kern >= 0 && tm->d2h >= 0) {
            s->t_h2d.push_back(tm->h2d);
            s->t_kern.push_back(tm->kern);
            s->t_d2h.push_back(tm->d2h);
        }
        s->first_arrival = std::min(s->first_arrival, q->r.t_arrival);
        s->last_completion = std::max(s->last_completion, t_done);
    } else {
        s->failed += 1;
    }
}

void worker_loop(nufft2_server_s *s)
{
    (void)hipSetDevice(s->device);
    struct Done {
        Request *q;
        nufft2_status st;
        StageTimes tm;
    };
    std::vector<Done> done;
    for (;;) {
        bool progress = false;
        // 1. retire completed requests
        done.clear();
        for (Slot &sl : s->slots) {
            if (!sl.req) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipErrorNotReady) continue;
            const nufft2_status st = q == hipSuccess ? NUFFT2_OK : NUFFT2_ERR_HIP;
            if (q != hipSuccess) (void)hipGetLastError();
            done.push_back({sl.req, st, st == NUFFT2_OK ? stage_times(sl) : StageTimes{}});
            CachedPlan *cp = sl.plan;
            cp->busy = false;
            cp->last_use = ++s->tick;
            if (st != NUFFT2_OK) evict_plan(s, cp);
            sl.req = nullptr;
            sl.plan = nullptr;
            s->busy -= 1;
        }
        if (!done.empty()) {
            const double t = s->now();
            {
                std::lock_guard<std::mutex> lk(s->mu);
                for (auto &d : done) record(s, d.q, d.st, t, &d.tm);
                s->inflight -= (int)done.size();
            }
            s->cv_done.notify_all();
            progress = true;
        }
        if (s->busy == 0 && !s->retired.empty()) free_retired(s);
        // 2. admit queued requests in arrival order
        for (;;) {
            Slot *slot = nullptr;
            for (Slot &sl : s->slots)
                if (!sl.req) {
                    slot = &sl;
                    break;
                }
            if (!slot) break;
            Request *q = nullptr;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                if (!s->queue.empty()) q = s->queue.front();
            }
            if (!q) break;
            nufft2_status st = NUFFT2_OK;
            const Start r = start(s, *slot, q, &st);
            if (r == Start::kWait) break;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                s->queue.pop_front();
                if (r == Start::kStarted) {
                    s->inflight += 1;
                    s->max_inflight_seen = std::max(s->max_inflight_seen, s->inflight);
                } else {
                    record(s, q, st, s->now());
                }
            }
            if (r == Start::kFailed) s->cv_done.notify_all();
            progress = true;
        }
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->stop && s->queue.empty() && s->inflight == 0) break;
        if (!progress) {
            if (s->inflight > 0) {
                // poll the in-flight work about every 20 microseconds
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
            } else {
                s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty(); });
            }
        }
    }
    free_retired(s);
}

}  // namespace

NUFFT2_API nufft2_status nufft2_server_create(const nufft2_server_opts *opts, nufft2_server *out)
{
    if (!out) return NUFFT2_ERR_ARG;
    nufft2_server_opts o{};
    if (opts) o = *opts;
    if (o.max_inflight < 0 || o.max_inflight > kMaxInflight || o.reserved != 0) return NUFFT2_ERR_ARG;
    nufft2_server_s *s = new (std::nothrow) nufft2_server_s();
    if (!s) return NUFFT2_ERR_ALLOC;
    s->budget = o.hbm_budget ? o.hbm_budget : kDefaultBudget;
    s->max_inflight = o.max_inflight ? o.max_inflight : kDefaultInflight;
    s->t0 = std::chrono::steady_clock::now();
    if (hipGetDevice(&s->device) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return NUFFT2_ERR_HIP;
    }
    s->slots.resize(s->max_inflight);
    auto release = [&]() {
        for (Slot &x : s->slots) {
            for (hipEvent_t ev : {x.start, x.h2d, x.kern, x.done})
                if (ev) (void)hipEventDestroy(ev);
            if (x.stream) (void)hipStreamDestroy(x.stream);
        }
    };
    for (Slot &sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreate(&sl.start) != hipSuccess || hipEventCreate(&sl.h2d) != hipSuccess ||
            hipEventCreate(&sl.kern) != hipSuccess || hipEventCreate(&sl.done) != hipSuccess) {
            (void)hipGetLastError();
            release();
            delete s;
            return NUFFT2_ERR_HIP;
        }
    }
    try {
        s->worker = std::thread(worker_loop, s);
    } catch (...) {
        release();
        delete s;
        return NUFFT2_ERR_ALLOC;
    }
    *out = s;
    return NUFFT2_OK;
}

NUFFT2_API double nufft2_server_clock(nufft2_server s) { return s ? s->now() : 0.0; }

NUFFT2_API nufft2_status nufft2_server_submit(nufft2_server s, const nufft2_request *req, uint64_t *ticket)
{
    if (!s || !req || !ticket) return NUFFT2_ERR_ARG;
    const nufft2_request &r = *req;
    if ((r.prec != NUFFT2_FP32 && r.prec != NUFFT2_FP64) || r.n_fields < 1 || r.n_modes_theta < 1 ||
        r.n_modes_phi < 1 || r.n_modes_theta > 2048 || r.n_modes_phi > 2048 || r.n_pts < 1 ||
        r.n_pts > (int64_t)0x7fffffff || !r.coeffs_host || !r.phi_host || !r.theta_host || !isfinite(r.t_arrival))
        return NUFFT2_ERR_ARG;
    int32_t w;
    double beta;
    nufft2_status st = nufft2_kernel_params((nufft2_prec)r.prec, r.eps, &w, &beta);
    if (st != NUFFT2_OK) return st;
    Request *q = new (std::nothrow) Request();
    if (!q) return NUFFT2_ERR_ALLOC;
    q->r = r;
    q->key = PlanKey{r.prec, r.n_fields, r.n_modes_theta, r.n_modes_phi, r.eps};
    q->plan_bytes = plan_estimate(r);
    q->buf_bytes = buffer_bytes(r);
    if (q->plan_bytes + round_up(q->buf_bytes, 1u << 20) > s->budget) {
        delete q;
        return NUFFT2_ERR_ARG;
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        q->id = s->next_id++;
        s->all.push_back(q);
        s->queue.push_back(q);
        *ticket = q->id;
    }
    s->cv_work.notify_one();
    return NUFFT2_OK;
}

NUFFT2_API nufft2_status nufft2_server_wait(nufft2_server s, uint64_t ticket, nufft2_status *req_status,
                                           double *latency)
{
    if (!s || ticket == 0) return NUFFT2_ERR_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    if (ticket >= s->next_id) return NUFFT2_ERR_ARG;
    Request *q = s->all[ticket - 1];
    s->cv_done.wait(lk, [&] { return q->done; });
    if (req_status) *req_status = q->status;
    if (latency) *latency = q->latency;
    return NUFFT2_OK;
}

NUFFT2_API nufft2_status nufft2_server_drain(nufft2_server s)
{
    if (!s) return NUFFT2_ERR_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->queue.empty() && s->inflight == 0; });
    return NUFFT2_OK;
}

NUFFT2_API nufft2_status nufft2_server_stats(nufft2_server s, nufft2_server_stats_t *st)
{
    if (!s || !st) return NUFFT2_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    memset(st, 0, sizeof(*st));
    st->submitted = (int64_t)s->all.size();
    st->completed = s->completed;
    st->failed = s->failed;
    st->points_fields = s->pf;
    std::vector<double> lat(s->latencies);
    std::sort(lat.begin(), lat.end());
    if (!lat.empty()) {
        auto pct = [&](double p) { return lat[std::min(lat.size() - 1, (size_t)(p * (double)lat.size()))]; };
        st->latency_p50 = pct(0.50);
        st->latency_p99 = pct(0.99);
        st->latency_max = lat.back();
        st->first_arrival = s->first_arrival;
        st->last_completion = s->last_completion;
    }
    auto pcts = [](std::vector<double> v, double &p50, double &p99) {
        std::sort(v.begin(), v.end());
        if (v.empty()) return;
        p50 = v[std::min(v.size() - 1, (size_t)(0.50 * (double)v.size()))];
        p99 = v[std::min(v.size() - 1, (size_t)(0.99 * (double)v.size()))];
    };
    pcts(s->t_queue, st->queue_p50, st->queue_p99);
    pcts(s->t_h2d, st->h2d_p50, st->h2d_p99);
    pcts(s->t_kern, st->kernel_p50, st->kernel_p99);
    pcts(s->t_d2h, st->d2h_p50, st->d2h_p99);
    st->plans_created = s->created;
    st->plans_evicted = s->evicted;
    st->hbm_high_water = s->high_water;
    st->max_inflight_seen = s->max_inflight_seen;
    return NUFFT2_OK;
}

NUFFT2_API nufft2_status nufft2_server_destroy(nufft2_server s)
{
    if (!s) return NUFFT2_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (CachedPlan *cp : s->plans) {
        (void)nufft2_destroy(cp->h);
        delete cp;
    }
    for (Slot &sl : s->slots) {
        (void)hipStreamSynchronize(sl.stream);
        if (sl.d_buf) (void)hipFree(sl.d_buf);
        if (sl.h_stage) (void)hipHostFree(sl.h_stage);
        for (hipEvent_t ev : {sl.start, sl.h2d, sl.kern, sl.done}) (void)hipEventDestroy(ev);
        (void)hipStreamDestroy(sl.stream);
    }
    for (Request *q : s->all) delete q;
    delete s;
    return NUFFT2_OK;
}
