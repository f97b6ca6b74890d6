// Autotuner: kernel width by measured accuracy, gather tiles by measured
// time, with a JSON cache.  Host code over the public C ABI (it plans,
// runs and destroys ordinary plans).
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "nufft2.h"
#include "nufft2_internal.hpp"

#define NUFFT2_API extern "C" __attribute__((visibility("default")))

namespace {

constexpr int kMaxW = 16;
constexpr int64_t kProbePoints = 16384;
constexpr int kTimedReps = 3;
constexpr int32_t kMaxTuneMembers = 4096;  // members of a timed group
// Gather tile shapes tried (rows, columns of first-tap cells per bin).
constexpr int kTileCandidates[][2] = {{8, 32}, {16, 32}, {32, 16}, {16, 64}, {32, 32}, {8, 64}, {32, 64}, {8, 128}};

struct CacheEntry {
    std::string key;
    int w = 0, tt = 0, tp = 0;
    double err = 0, ms = 0;
};

// One entry per line: {"key": "...", "w": 7, "tile_theta": 16, "tile_phi": 32, "err": ..., "ms": ...}
std::vector<CacheEntry> read_cache(const char *path)
{
    std::vector<CacheEntry> out;
    FILE *f = path ? fopen(path, "r") : nullptr;
    if (!f) return out;
    char line[1024];
    while (fgets(line, sizeof line, f)) {
        const char *k = strstr(line, "{\"key\": \"");
        if (!k) continue;
        k += 9;
        const char *e = strchr(k, '"');
        if (!e) continue;
        CacheEntry c;
        c.key.assign(k, e - k);
        if (sscanf(e, "\", \"w\": %d, \"tile_theta\": %d, \"tile_phi\": %d, \"err\": %lf, \"ms\": %lf", &c.w, &c.tt,
                   &c.tp, &c.err, &c.ms) == 5)
            out.push_back(c);
    }
    fclose(f);
    return out;
}

bool write_cache(const char *path, const std::vector<CacheEntry> &entries)
{
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return false;
    fprintf(f, "{\"nufft2_autotune\": [\n");
    for (size_t i = 0; i < entries.size(); ++i) {
        const CacheEntry &c = entries[i];
        fprintf(f, "{\"key\": \"%s\", \"w\": %d, \"tile_theta\": %d, \"tile_phi\": %d, \"err\": %.6e, \"ms\": %.6f}%s\n",
                c.key.c_str(), c.w, c.tt, c.tp, c.err, c.ms, i + 1 < entries.size() ? "," : "");
    }
    fprintf(f, "]}\n");
    const bool ok = fclose(f) == 0;
    return ok && rename(tmp.c_str(), path) == 0;
}

// splitmix64: a small counter-based generator for the probe coefficients
uint64_t splitmix64(uint64_t &state)
{
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double uniform_pm1(uint64_t &state) { return (double)(splitmix64(state) >> 11) * (2.0 / 9007199254740992.0) - 1.0; }

// RAII for device buffers and plans of one tuning run.
struct Scratch {
    std::vector<void *> bufs;
    std::vector<nufft2_handle> plans;
    ~Scratch()
    {
        for (nufft2_handle p : plans) (void)nufft2_destroy(p);
        for (void *b : bufs) (void)hipFree(b);
    }
    void *alloc(size_t bytes)
    {
        void *p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        bufs.push_back(p);
        return p;
    }
};

// One field of flat-spectrum coefficients (complex FP64, then optionally FP32).
void probe_coeffs(int64_t Kt, int64_t Kp, std::vector<double> &c64, std::vector<float> &c32)
{
    uint64_t st = 0x5EEDull;
    c64.resize((size_t)(2 * Kt * Kp));
    for (double &x : c64) x = uniform_pm1(st);
    c32.assign(c64.begin(), c64.end());
}

double rel_l2(const std::vector<double> &got, const std::vector<double> &ref)
{
    long double num = 0, den = 0;
    for (size_t i = 0; i < ref.size(); ++i) {
        const long double d = (long double)got[i] - ref[i];
        num += d * d;
        den += (long double)ref[i] * ref[i];
    }
    return den > 0 ? (double)sqrtl(num / den) : 0.0;
}

}  // namespace

namespace {

// members == 1: tiles timed on one plan; members > 1: on a group of that
// many plans, every member with the caller's points.
nufft2_status autotune_impl(nufft2_prec prec, int64_t Kt, int64_t Kp, int32_t n_fields, double eps, int64_t n_pts,
                            const double *phi_dev, const double *theta_dev, void *stream, const char *cache_path,
                            nufft2_opts *opts_out, nufft2_tune_result *result, int32_t members)
{
    if (!opts_out || n_pts < 1 || n_pts > (int64_t)0x7fffffff || !phi_dev || !theta_dev || n_fields < 1)
        return NUFFT2_ERR_ARG;
    if (members < 1 || members > kMaxTuneMembers || (int64_t)members * n_pts > (int64_t)0x7fffffff)
        return NUFFT2_ERR_ARG;
    // opts_out->hermitian on input: time the tiles on real-field plans
    const int herm = opts_out->hermitian;
    if (herm != 0 && herm != 1) return NUFFT2_ERR_ARG;
    if (herm && (Kt % 2 == 0 || Kp % 2 == 0)) return NUFFT2_ERR_ARG;
    int32_t w0;
    double beta0;
    nufft2_status st = nufft2_kernel_params(prec, eps, &w0, &beta0);
    if (st != NUFFT2_OK) return st;
    if (Kt <= 0 || Kp <= 0 || Kt > 2048 || Kp > 2048) return NUFFT2_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;

    char key[256];
    {
        int dev = 0;
        hipDeviceProp_t prop{};
        if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
            (void)hipGetLastError();
            return NUFFT2_ERR_HIP;
        }
        char arch[64];
        snprintf(arch, sizeof arch, "%s", prop.gcnArchName);
        for (char *c = arch; *c; ++c)
            if (*c == '"' || *c == '\\' || *c == ':') *c = '_';
        int64_t nb = 1;
        while (nb < n_pts) nb <<= 1;
        char grp[24] = "";
        if (members > 1) snprintf(grp, sizeof grp, "_m%d", (int)members);
        snprintf(key, sizeof key, "prec%d_K%lldx%lld_F%d_eps%.3e_n%lld_h%d%s_%s", (int)prec, (long long)Kt,
                 (long long)Kp, n_fields, eps, (long long)nb, herm, grp, arch);
    }
    std::vector<CacheEntry> cache = read_cache(cache_path);
    for (const CacheEntry &c : cache)
        if (c.key == key) {
            memset(opts_out, 0, sizeof(*opts_out));
            opts_out->w = c.w;
            opts_out->tile_theta = c.tt;
            opts_out->tile_phi = c.tp;
            opts_out->hermitian = herm;
            if (result) {
                memset(result, 0, sizeof(*result));
                result->w = c.w;
                result->tile_theta = c.tt;
                result->tile_phi = c.tp;
                result->err = c.err;
                result->ms = c.ms;
                result->from_cache = 1;
            }
            return NUFFT2_OK;
        }

    Scratch sc;
    const size_t cs = prec == NUFFT2_FP32 ? 2 * sizeof(float) : 2 * sizeof(double);
    const int64_t np = std::min(n_pts, kProbePoints);
    std::vector<double> c64;
    std::vector<float> c32;
    probe_coeffs(Kt, Kp, c64, c32);
    void *d_c64 = sc.alloc(c64.size() * sizeof(double));
    void *d_cin = prec == NUFFT2_FP32 ? sc.alloc(c32.size() * sizeof(float)) : d_c64;
    void *d_ref = sc.alloc((size_t)np * 2 * sizeof(double));
    // one output per member (the members of a timed group write side by side)
    void *d_out = sc.alloc((size_t)members * n_pts * n_fields * cs);
    void *d_cf = sc.alloc((size_t)n_fields * Kt * Kp * cs);
    if (!d_c64 || !d_cin || !d_ref || !d_out || !d_cf) return NUFFT2_ERR_ALLOC;
    hipError_t e;
    if ((e = hipMemcpy(d_c64, c64.data(), c64.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess ||
        (prec == NUFFT2_FP32 &&
         (e = hipMemcpy(d_cin, c32.data(), c32.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess))
        return NUFFT2_ERR_HIP;
    for (int f = 0; f < n_fields; ++f)
        if ((e = hipMemcpy((char *)d_cf + (size_t)f * Kt * Kp * cs, d_cin, (size_t)Kt * Kp * cs,
                           hipMemcpyDeviceToDevice)) != hipSuccess)
            return NUFFT2_ERR_HIP;

    auto make_plan = [&](nufft2_prec pr, int32_t F, int32_t w, int tt, int tp, nufft2_handle *h, int hm = 0) {
        nufft2_opts o{};
        o.w = w;
        o.tile_theta = tt;
        o.tile_phi = tp;
        o.hermitian = hm;
        const double pe = pr == NUFFT2_FP64 ? std::max(eps, 1e-15) : eps;
        nufft2_status r = nufft2_plan(pr, Kt, Kp, F, pe, &o, stream, h);
        if (r == NUFFT2_OK) sc.plans.push_back(*h);
        return r;
    };

    // reference: FP64, three widths above the rule
    std::vector<double> ref((size_t)np * 2);
    {
        nufft2_handle h;
        if ((st = make_plan(NUFFT2_FP64, 1, std::min(kMaxW, w0 + 3), 0, 0, &h)) != NUFFT2_OK) return st;
        if ((st = nufft2_setpts(h, np, phi_dev, theta_dev)) != NUFFT2_OK ||
            (st = nufft2_exec(h, d_c64, d_ref)) != NUFFT2_OK)
            return st;
        if ((e = hipStreamSynchronize(s)) != hipSuccess ||
            (e = hipMemcpy(ref.data(), d_ref, ref.size() * sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess)
            return NUFFT2_ERR_HIP;
    }
    // width: smallest candidate within eps on the probe, widening up to the
    // reference's width (beyond it the reference cannot judge)
    int w_best = -1;
    double err_best = 0;
    const int w_ref = std::min(kMaxW, w0 + 3);
    // (at the widest width the reference is the only judge there is)
    for (int w = std::max(2, w0 - 1); w < w_ref || (w == w_ref && w == kMaxW); ++w) {
        nufft2_handle h;
        if ((st = make_plan(prec, 1, w, 0, 0, &h)) != NUFFT2_OK) return st;
        if ((st = nufft2_setpts(h, np, phi_dev, theta_dev)) != NUFFT2_OK || (st = nufft2_exec(h, d_cin, d_out)) != NUFFT2_OK)
            return st;
        std::vector<double> got((size_t)np * 2);
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return NUFFT2_ERR_HIP;
        if (prec == NUFFT2_FP32) {
            std::vector<float> g32(got.size());
            if ((e = hipMemcpy(g32.data(), d_out, g32.size() * sizeof(float), hipMemcpyDeviceToHost)) != hipSuccess)
                return NUFFT2_ERR_HIP;
            got.assign(g32.begin(), g32.end());
        } else if ((e = hipMemcpy(got.data(), d_out, got.size() * sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess) {
            return NUFFT2_ERR_HIP;
        }
        const double err = rel_l2(got, ref);
        w_best = w;
        err_best = err;
        if (err <= eps) break;
    }
    if (!(err_best <= eps)) {
        // no width reaches eps on the probe (the precision's floor): report
        // the closest, write nothing to the cache
        if (result) {
            memset(result, 0, sizeof(*result));
            result->w = w_best;
            result->err = err_best;
        }
        return NUFFT2_ERR_EPS_RANGE;
    }
    // tiles: fastest candidate for that width
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (hipEventCreate(&ev0) != hipSuccess || hipEventCreate(&ev1) != hipSuccess) {
        (void)hipGetLastError();
        if (ev0) (void)hipEventDestroy(ev0);
        return NUFFT2_ERR_HIP;
    }
    int tt_best = 0, tp_best = 0, timed = 0;
    double ms_best = 1e300;
    const std::vector<int64_t> g_n(members, n_pts);
    const std::vector<const double *> g_phi(members, phi_dev), g_theta(members, theta_dev);
    const std::vector<const void *> g_cf(members, d_cf);
    std::vector<void *> g_out(members);
    for (int i = 0; i < members; ++i) g_out[i] = (char *)d_out + (size_t)i * n_pts * n_fields * cs;
    for (const auto &tc : kTileCandidates) {
        std::vector<nufft2_handle> hs;
        bool made = true;
        for (int i = 0; i < members && made; ++i) {
            nufft2_handle h;
            made = make_plan(prec, n_fields, w_best, tc[0], tc[1], &h, herm) == NUFFT2_OK;  // e.g. LDS limit
            if (made) hs.push_back(h);
        }
        nufft2_group g = nullptr;
        if (made && members > 1) made = nufft2_group_create(hs.data(), members, &g) == NUFFT2_OK;
        std::vector<float> ms;
        for (int rep = 0; made && rep <= kTimedReps; ++rep) {
            if (hipEventRecord(ev0, s) != hipSuccess) break;
            if (g) {
                if (nufft2_group_setpts(g, g_n.data(), g_phi.data(), g_theta.data()) != NUFFT2_OK ||
                    nufft2_group_exec(g, g_cf.data(), g_out.data()) != NUFFT2_OK)
                    break;
            } else if (nufft2_setpts(hs[0], n_pts, phi_dev, theta_dev) != NUFFT2_OK ||
                       nufft2_exec(hs[0], d_cf, d_out) != NUFFT2_OK) {
                break;
            }
            float t = 0;
            if (hipEventRecord(ev1, s) != hipSuccess || hipEventSynchronize(ev1) != hipSuccess ||
                hipEventElapsedTime(&t, ev0, ev1) != hipSuccess)
                break;
            if (rep > 0) ms.push_back(t);  // rep 0 warms up
        }
        (void)hipGetLastError();
        // release this candidate's workspaces before the next one
        if (g) (void)nufft2_group_destroy(g);
        for (nufft2_handle h : hs) {
            (void)nufft2_destroy(h);
            sc.plans.erase(std::find(sc.plans.begin(), sc.plans.end(), h));
        }
        if ((int)ms.size() != kTimedReps) continue;
        std::sort(ms.begin(), ms.end());
        ++timed;
        if (ms[kTimedReps / 2] < ms_best) {
            ms_best = ms[kTimedReps / 2];
            tt_best = tc[0];
            tp_best = tc[1];
        }
    }
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    if (timed == 0) return NUFFT2_ERR_HIP;

    memset(opts_out, 0, sizeof(*opts_out));
    opts_out->w = w_best;
    opts_out->tile_theta = tt_best;
    opts_out->tile_phi = tp_best;
    opts_out->hermitian = herm;
    if (result) {
        memset(result, 0, sizeof(*result));
        result->w = w_best;
        result->tile_theta = tt_best;
        result->tile_phi = tp_best;
        result->err = err_best;
        result->ms = ms_best;
        result->n_timed = timed;
    }
    if (cache_path) {
        CacheEntry c;
        c.key = key;
        c.w = w_best;
        c.tt = tt_best;
        c.tp = tp_best;
        c.err = err_best;
        c.ms = ms_best;
        bool replaced = false;
        for (CacheEntry &x : cache)
            if (x.key == c.key) {
                x = c;
                replaced = true;
            }
        if (!replaced) cache.push_back(c);
        (void)write_cache(cache_path, cache);
    }
    return NUFFT2_OK;
}

}  // namespace

NUFFT2_API nufft2_status nufft2_autotune(nufft2_prec prec, int64_t Kt, int64_t Kp, int32_t n_fields, double eps,
                                         int64_t n_pts, const double *phi_dev, const double *theta_dev, void *stream,
                                         const char *cache_path, nufft2_opts *opts_out, nufft2_tune_result *result)
{
    return autotune_impl(prec, Kt, Kp, n_fields, eps, n_pts, phi_dev, theta_dev, stream, cache_path, opts_out,
                         result, 1);
}

NUFFT2_API nufft2_status nufft2_autotune_group(nufft2_prec prec, int64_t Kt, int64_t Kp, int32_t n_fields,
                                               double eps, int32_t members, int64_t n_pts, const double *phi_dev,
                                               const double *theta_dev, void *stream, const char *cache_path,
                                               nufft2_opts *opts_out, nufft2_tune_result *result)
{
    return autotune_impl(prec, Kt, Kp, n_fields, eps, n_pts, phi_dev, theta_dev, stream, cache_path, opts_out,
                         result, members);
}
