// Definitions behind hip/hip_runtime.h of this directory, and a stand-in
// for the four plan calls the serving loop makes (nufft2_plan, _setpts,
// _exec, _destroy) plus nufft2_kernel_params.  The stand-in plan allocates
// workspaces of the sizes the library would report, through the stub
// hipMalloc, so that the serving loop's memory accounting can be checked
// against what is really allocated; its exec writes a value that depends
// on the request's inputs only:
//   out[f][j] = c[f][0][0] + (f + 1) phi[j] + i theta[j]
// Test infrastructure only.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <map>
#include <vector>
#include <mutex>
#include <thread>

#include "hip/hip_runtime.h"
#include "nufft2.h"
#include "plan_state.hpp"
#include "stub_control.h"

namespace {

using Clock = std::chrono::steady_clock;

std::mutex g_mu;                       // guards the allocation table
std::map<void *, size_t> g_live;       // "device" allocations
size_t g_bytes = 0, g_peak = 0;
std::atomic<int64_t> g_fail_at{-1};     // fail the allocation of at least this size
std::atomic<int64_t> g_mallocs{0};

double now_s() { return std::chrono::duration<double>(Clock::now().time_since_epoch()).count(); }

}  // namespace

struct StubStream {
    double busy_until = 0;  // simulated completion time of the enqueued work
};
struct StubEvent {
    double t = -1;          // completion time; < 0: never recorded
};

namespace {

// Work enqueued on s takes `sec` seconds of simulated device time.
void advance(hipStream_t s, double sec)
{
    if (!s) return;
    s->busy_until = std::max(s->busy_until, now_s()) + sec;
}

}  // namespace

void stub_fail_allocations_of_at_least(int64_t bytes) { g_fail_at.store(bytes); }
size_t stub_device_bytes()
{
    std::lock_guard<std::mutex> lk(g_mu);
    return g_bytes;
}
size_t stub_device_peak()
{
    std::lock_guard<std::mutex> lk(g_mu);
    return g_peak;
}
void stub_reset_peak()
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_peak = g_bytes;
}

hipError_t hipMalloc(void **ptr, size_t bytes)
{
    g_mallocs.fetch_add(1);
    const int64_t f = g_fail_at.load();
    if (f >= 0 && (int64_t)bytes >= f) {
        *ptr = nullptr;
        return hipErrorOutOfMemory;
    }
    void *p = malloc(bytes ? bytes : 1);
    if (!p) return hipErrorOutOfMemory;
    std::lock_guard<std::mutex> lk(g_mu);
    g_live[p] = bytes;
    g_bytes += bytes;
    g_peak = std::max(g_peak, g_bytes);
    *ptr = p;
    return hipSuccess;
}

hipError_t hipFree(void *ptr)
{
    if (!ptr) return hipSuccess;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_live.find(ptr);
    if (it == g_live.end()) return hipErrorInvalidValue;
    g_bytes -= it->second;
    g_live.erase(it);
    free(ptr);
    return hipSuccess;
}

hipError_t hipHostMalloc(void **ptr, size_t bytes, unsigned)
{
    *ptr = malloc(bytes ? bytes : 1);
    return *ptr ? hipSuccess : hipErrorOutOfMemory;
}

hipError_t hipHostFree(void *ptr)
{
    free(ptr);
    return hipSuccess;
}

hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind, hipStream_t s)
{
    if (bytes && (!dst || !src)) return hipErrorInvalidValue;
    memcpy(dst, src, bytes);
    advance(s, 2e-6 + bytes / 20e9);
    return hipSuccess;
}

hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned)
{
    *s = new StubStream();
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s)
{
    delete s;
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s)
{
    if (s) {
        const double wait = s->busy_until - now_s();
        if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(wait));
    }
    return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t *e)
{
    *e = new StubEvent();
    return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e)
{
    delete e;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s)
{
    if (!e) return hipErrorInvalidValue;
    e->t = s ? std::max(s->busy_until, now_s()) : now_s();
    return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e)
{
    if (!e || e->t < 0) return hipErrorInvalidValue;
    return now_s() >= e->t ? hipSuccess : hipErrorNotReady;
}
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b)
{
    if (!a || !b || a->t < 0 || b->t < 0) return hipErrorInvalidValue;
    *ms = (float)((b->t - a->t) * 1e3);
    return hipSuccess;
}
hipError_t hipGetDevice(int *d)
{
    *d = 0;
    return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetLastError(void) { return hipSuccess; }

// ---- the plan calls ----------------------------------------------------

namespace {

int64_t fine(int64_t K, int w)
{
    int64_t n = std::max<int64_t>({2 * K, 2 * (int64_t)w, 32});
    int64_t f = 1;
    while (f < n) f <<= 1;
    return f;
}

// per point: key/rank, record, permutation (as the library's setpts grows them)
size_t point_bytes(int prec) { return sizeof(int2) + 2 * (prec == NUFFT2_FP32 ? 4 : 8) + 8 + sizeof(int32_t); }

struct StubPlan {
    std::vector<void *> bufs;
    const double *phi = nullptr, *theta = nullptr;  // the last setpts' points
};
std::mutex g_plan_mu;
std::map<nufft2_plan_s *, StubPlan> g_plans;

}  // namespace

extern "C" nufft2_status nufft2_kernel_params(nufft2_prec prec, double eps, int32_t *w, double *beta)
{
    if (!w || !beta || !(eps > 0.0) || !isfinite(eps)) return NUFFT2_ERR_ARG;
    if (prec != NUFFT2_FP32 && prec != NUFFT2_FP64) return NUFFT2_ERR_ARG;
    if (eps < (prec == NUFFT2_FP32 ? 1e-7 : 1e-15) * (1.0 - 1e-12)) return NUFFT2_ERR_EPS_RANGE;
    *w = std::max(2, std::min(16, (int)ceil(-log10(eps) - 1e-9) + 1));
    *beta = 2.30 * *w;
    return NUFFT2_OK;
}

extern "C" nufft2_status nufft2_plan(nufft2_prec prec, int64_t Kt, int64_t Kp, int32_t F, double eps,
                                     const nufft2_opts *, void *stream, nufft2_handle *out)
{
    int32_t w;
    double beta;
    nufft2_status st = nufft2_kernel_params(prec, eps, &w, &beta);
    if (st != NUFFT2_OK) return st;
    nufft2_plan_s *p = new nufft2_plan_s();
    p->prec = prec;
    p->Kt = Kt;
    p->Kp = Kp;
    p->F = F;
    p->w = w;
    p->nft = (int)fine(Kt, w);
    p->nfp = (int)fine(Kp, w);
    p->stream = (hipStream_t)stream;
    p->n_pts = -1;
    const size_t cs = prec == NUFFT2_FP32 ? 8 : 16;
    // the fine grids and the theta-pass buffer, as the library allocates them
    const size_t bytes = cs * (size_t)F * p->nft * (size_t)(p->nfp + Kp) + (64u << 10);
    void *b = nullptr;
    if (hipMalloc(&b, bytes) != hipSuccess) {
        delete p;
        return NUFFT2_ERR_ALLOC;
    }
    p->ws_bytes = bytes;
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        g_plans[p].bufs.push_back(b);
    }
    advance(p->stream, 20e-6);
    *out = p;
    return NUFFT2_OK;
}

extern "C" nufft2_status nufft2_setpts(nufft2_handle p, int64_t n, const double *phi, const double *theta)
{
    if (!p || n < 0 || (n > 0 && (!phi || !theta))) return NUFFT2_ERR_ARG;
    if (n > p->pts_cap) {
        const size_t grow = (size_t)(n - p->pts_cap) * point_bytes(p->prec);
        void *b = nullptr;
        if (hipMalloc(&b, grow) != hipSuccess) return NUFFT2_ERR_ALLOC;
        std::lock_guard<std::mutex> lk(g_plan_mu);
        g_plans[p].bufs.push_back(b);
        p->ws_bytes += grow;
        p->pts_cap = n;
    }
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        g_plans[p].phi = phi;
        g_plans[p].theta = theta;
    }
    p->n_pts = n;
    advance(p->stream, 5e-6 + n * 2e-10);
    return NUFFT2_OK;
}

extern "C" nufft2_status nufft2_exec(nufft2_handle p, const void *coeffs, void *out)
{
    if (!p || !coeffs || !out) return NUFFT2_ERR_ARG;
    if (p->n_pts < 0) return NUFFT2_ERR_NO_POINTS;
    const double *phi, *theta;
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        phi = g_plans[p].phi;
        theta = g_plans[p].theta;
    }
    for (int f = 0; f < p->F; ++f) {
        const size_t c0 = (size_t)f * p->Kt * p->Kp;
        for (int64_t j = 0; j < p->n_pts; ++j) {
            const size_t o = (size_t)f * p->n_pts + j;
            if (p->prec == NUFFT2_FP32) {
                const float2 c = ((const float2 *)coeffs)[c0];
                ((float2 *)out)[o] = float2{c.x + (float)((f + 1) * phi[j]), c.y + (float)theta[j]};
            } else {
                const double2 c = ((const double2 *)coeffs)[c0];
                ((double2 *)out)[o] = double2{c.x + (f + 1) * phi[j], c.y + theta[j]};
            }
        }
    }
    advance(p->stream, 10e-6 + p->n_pts * p->F * 1e-9);
    return NUFFT2_OK;
}

extern "C" nufft2_status nufft2_destroy(nufft2_handle p)
{
    if (!p) return NUFFT2_OK;
    std::vector<void *> bufs;
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        bufs = g_plans[p].bufs;
        g_plans.erase(p);
    }
    for (void *b : bufs) (void)hipFree(b);
    delete p;
    return NUFFT2_OK;
}
