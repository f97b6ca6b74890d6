// Host side of the C ABI: plan construction, kernel parameters and
// deconvolution factors, workspace ownership, and the launch sequence of
// setpts / exec.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "nufft2.h"
#include "nufft2_internal.hpp"
#include "plan_state.hpp"

#define NUFFT2_API extern "C" __attribute__((visibility("default")))

using namespace nufft2;

namespace {

constexpr int kMaxNf = 4096;
constexpr int kMaxW = 16;
constexpr double kDefaultBetaOverW = 2.30;
constexpr int kDefaultTileTheta = 16;
constexpr int kDefaultTilePhi = 32;
// Real-field plans: a real patch takes half the LDS of a complex one, so
// the tiles are wider.  Measured at 1024 x 2048 (setpts + exec, 3 fields):
// FP32 16 x 64 (compile-time patch geometry) ahead of 16 x 32, 32 x 32,
// 8 x 64, 32 x 64 and 16 x 128, and level with 8 x 128 even with that
// geometry compiled too; FP64 8 x 64 ahead of 16 x 32 (about 1% per step),
// 32 x 16, 32 x 32, 16 x 64, 8 x 32 and 16 x 16.  Complex plans keep
// 16 x 32 (FP64 complex: ahead of 8 x 32, 16 x 16, 32 x 16 and 8 x 64).
constexpr int kDefaultTileThetaReal32 = 16;
constexpr int kDefaultTilePhiReal32 = 64;
constexpr int kDefaultTileThetaReal64 = 8;
constexpr int kDefaultTilePhiReal64 = 64;
constexpr size_t kGatherLdsLimit = 65536;  // per staged field group
constexpr size_t kFftLdsLimit = 155648;    // 152 KiB of the 160 KiB per workgroup
constexpr size_t kCuLds = 163840;          // LDS per CU
constexpr int kGatherMaxFieldsPerPass = 4;
// an FFT pass with fewer waves than this at 16 elements per thread (8 per
// SIMD of the 256 CUs) runs with 8 elements per thread
constexpr int64_t kSmallLaunchWaves = 8 * 256;

}  // namespace

namespace {

int ilog2(int64_t x)
{
    int l = 0;
    while ((int64_t(1) << l) < x) ++l;
    return l;
}

bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

// w = ceil(log10(1/eps)) + 1 at upsampling 2 (13 for 1e-12, 7 for 1e-6).
nufft2_status kernel_params(int prec, double eps, int32_t *w_out, double *beta_out)
{
    if (!(eps > 0.0) || !isfinite(eps)) return NUFFT2_ERR_ARG;
    if (prec != NUFFT2_FP32 && prec != NUFFT2_FP64) return NUFFT2_ERR_ARG;
    const double floor_eps = prec == NUFFT2_FP32 ? 1e-7 : 1e-15;
    if (eps < floor_eps * (1.0 - 1e-12)) return NUFFT2_ERR_EPS_RANGE;
    int w = (int)ceil(-log10(eps) - 1e-9) + 1;
    if (w < 2) w = 2;
    if (w > kMaxW) w = kMaxW;
    *w_out = w;
    *beta_out = kDefaultBetaOverW * w;
    return NUFFT2_OK;
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_n, long double).
void gauss_legendre(int n, std::vector<long double> &x, std::vector<long double> &wt)
{
    x.assign(n, 0.0L);
    wt.assign(n, 0.0L);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < (n + 1) / 2; ++i) {
        long double z = cosl(pi * (i + 0.75L) / (n + 0.5L)), pp = 1.0L;
        for (int it = 0; it < 100; ++it) {
            long double p1 = 1.0L, p2 = 0.0L;
            for (int j = 1; j <= n; ++j) {
                const long double p3 = p2;
                p2 = p1;
                p1 = ((2.0L * j - 1.0L) * z * p2 - (j - 1.0L) * p3) / j;
            }
            pp = n * (z * p1 - p2) / (z * z - 1.0L);
            const long double z1 = z;
            z = z1 - p1 / pp;
            if (fabsl(z - z1) < 1e-19L) break;
        }
        x[i] = -z;
        x[n - 1 - i] = z;
        wt[i] = wt[n - 1 - i] = 2.0L / ((1.0L - z * z) * pp * pp);
    }
}

// Phi(xi) = int_{-1}^{1} exp(beta (sqrt(1 - z^2) - 1)) cos(xi z) dz, by the
// substitution z = sin s (which removes the square-root edge of the kernel)
// and Gauss-Legendre in s on [-pi/2, pi/2].
long double kernel_ft(long double xi, long double beta, const std::vector<long double> &x,
                      const std::vector<long double> &wt)
{
    const long double half_pi = 1.570796326794896619231321691639751442L;
    long double acc = 0.0L;
    for (size_t q = 0; q < x.size(); ++q) {
        const long double s = half_pi * x[q];
        const long double cs = cosl(s);
        acc += wt[q] * expl(beta * (cs - 1.0L)) * cosl(xi * sinl(s)) * cs;
    }
    return acc * half_pi;
}

nufft2_status kernel_correction(int64_t K, int64_t nf, int w, double beta, double *corr)
{
    if (K <= 0 || nf <= 0 || w < 2 || w > kMaxW || !(beta > 0) || !corr) return NUFFT2_ERR_ARG;
    const long double pi = 3.141592653589793238462643383279502884L;
    std::vector<long double> prev(K), cur(K), x, wt;
    // Double the node count until no factor moves by more than 1e-16 relative.
    for (int n = 32;; n *= 2) {
        gauss_legendre(n, x, wt);
        long double change = 0.0L;
        for (int64_t a = 0; a < K; ++a) {
            const long double k = (long double)(a - K / 2);
            cur[a] = kernel_ft(pi * w * k / (long double)nf, beta, x, wt);
            if (n > 32) {
                const long double d = fabsl(cur[a] - prev[a]) / fabsl(cur[a]);
                if (d > change) change = d;
            }
        }
        prev.swap(cur);
        if ((n > 32 && change < 1e-17L) || n >= 2048) break;
    }
    for (int64_t a = 0; a < K; ++a) corr[a] = (double)(2.0L / ((long double)w * prev[a]));
    return NUFFT2_OK;
}

// Twiddle tables of an N-point transform in the kernels' layout:
// lo[u] = e^{2 pi i u / N} for u < 64, then hi[v] = e^{2 pi i 64 v / N} for
// v < max(N / 64, 1); the kernels form e^{2 pi i t / N} = lo[t % 64] hi[t / 64].
template <typename T> void fill_twiddle_tables(std::vector<T> &buf, int N)
{
    const long double two_pi = 6.283185307179586476925286766559005768L;
    const int lo = 64, hi = N > 64 ? N / 64 : 1;
    buf.clear();
    for (int u = 0; u < lo; ++u) {
        const long double ang = two_pi * (long double)u / (long double)N;
        buf.push_back((T)cosl(ang));
        buf.push_back((T)sinl(ang));
    }
    for (int v = 0; v < hi; ++v) {
        const long double ang = two_pi * (long double)(64 * v) / (long double)N;
        buf.push_back((T)cosl(ang));
        buf.push_back((T)sinl(ang));
    }
}

// ES kernel exp(beta (sqrt(1 - z^2) - 1)) in long double, z^2 clamped to 1.
long double es_kernel_ld(long double z, long double beta)
{
    long double z2 = z * z;
    if (z2 > 1.0L) z2 = 1.0L;
    return expl(-beta * z2 / (1.0L + sqrtl(1.0L - z2)));
}

// Tap weights as polynomials.  A point's offset v (first tap i0 = ceil(t -
// w/2), v = t - i0 - floor(w/2)) lies in [vlo, vlo + 1], vlo = w/2 - 1 -
// floor(w/2); tap b has weight phi((b - floor(w/2) - v) / (w/2)), a smooth
// function of v except for the square-root edge of the kernel at the end of
// the support, which lies in the intervals of taps 0 and w - 1.  Tap b's
// weight (taps first .. last - 1) is interpolated in long double by a
// polynomial of degree D - 1 in u = v - (vlo + 1/2) at the Chebyshev points
// of [-1/2, 1/2] (coefficients lowest degree first, rounded to C, row b of
// out; other rows zero).  False when a rounded polynomial misses the kernel
// by more than tol on a fine grid of u.
template <int D, typename C>
static bool fit_tap_polynomials(int w, double beta, long double tol, int first, int last, std::vector<C> &out)
{
    const long double pi = 3.141592653589793238462643383279502884L;
    const int H = w / 2;
    const long double hw = (long double)w / 2.0L;
    const long double c = ((long double)w / 2.0L - 1.0L - (long double)H) + 0.5L;
    out.assign((size_t)w * D, (C)0);
    std::vector<long double> u(D);
    for (int i = 0; i < D; ++i) u[i] = 0.5L * cosl(pi * (2.0L * i + 1.0L) / (2.0L * D));
    for (int b = first; b < last; ++b) {
        // Vandermonde system at the nodes, Gaussian elimination with pivoting
        long double A[D][D + 1];
        for (int i = 0; i < D; ++i) {
            long double pw = 1.0L;
            for (int j = 0; j < D; ++j) {
                A[i][j] = pw;
                pw *= u[i];
            }
            A[i][D] = es_kernel_ld(((long double)(b - H) - (u[i] + c)) / hw, beta);
        }
        for (int col = 0; col < D; ++col) {
            int piv = col;
            for (int r = col + 1; r < D; ++r)
                if (fabsl(A[r][col]) > fabsl(A[piv][col])) piv = r;
            for (int k = 0; k <= D; ++k) std::swap(A[col][k], A[piv][k]);
            for (int r = 0; r < D; ++r) {
                if (r == col) continue;
                const long double f = A[r][col] / A[col][col];
                for (int k = col; k <= D; ++k) A[r][k] -= f * A[col][k];
            }
        }
        for (int j = 0; j < D; ++j) out[(size_t)b * D + j] = (C)(A[j][D] / A[j][j]);
        // check the rounded polynomial against the kernel
        for (int q = 0; q <= 1024; ++q) {
            const long double uu = -0.5L + (long double)q / 1024.0L;
            long double acc = 0.0L;
            for (int j = D - 1; j >= 0; --j) acc = acc * uu + (long double)out[(size_t)b * D + j];
            const long double ex = es_kernel_ld(((long double)(b - H) - (uu + c)) / hw, beta);
            if (fabsl(acc - ex) > tol) return false;
        }
    }
    return true;
}

// FP32 plans: every tap, degree kPolyCoefs - 1, within 1e-7 (false for w < 7
// at beta = 2.30 w, where the edge taps' square-root term is too large).
// FP64 plans: the interior taps 1 .. w - 2, degree kPolyCoefs64 - 1, within
// 2e-15 (at beta = 2.30 w and w >= 7 they reach 1e-15); the edge taps are
// evaluated directly.  The table is raw device storage: FP64 coefficients
// occupy two floats each.
bool weight_polynomials(int prec, int w, double beta, std::vector<float> &out)
{
    if (prec == NUFFT2_FP32) return fit_tap_polynomials<kPolyCoefs>(w, beta, 1e-7L, 0, w, out);
    std::vector<double> c;
    if (!fit_tap_polynomials<kPolyCoefs64>(w, beta, 2e-15L, 1, w - 1, c)) return false;
    out.resize(2 * c.size());
    memcpy(out.data(), c.data(), sizeof(double) * c.size());
    return true;
}

// Floats of a plan's polynomial table (0: direct evaluation).
size_t poly_table_floats(int prec, int w)
{
    if (prec == NUFFT2_FP32) return w >= kPolyMinW ? (size_t)w * kPolyCoefs : 0;
    return w >= kPolyMinW64 ? 2 * (size_t)w * kPolyCoefs64 : 0;
}

void free_all(nufft2_plan_s *p)
{
    void *ptrs[] = {p->corr_t, p->corr_p, p->tw_t,  p->tw_p,  p->twist_t,   p->S,     p->grid,
                    p->bincount, p->binstart, p->binlist, p->rowmark, p->rowtouched, p->flags, p->keyrank,
                    p->rec,    p->perm,   p->stage, p->passtot, p->lstart, p->c2r, p->wpoly, p->pq};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    p->c2r = nullptr;
    p->wpoly = nullptr;
    p->corr_t = p->corr_p = p->tw_t = p->tw_p = p->twist_t = p->S = p->grid = nullptr;
    p->bincount = p->binstart = p->binlist = p->flags = p->perm = nullptr;
    p->rowmark = p->rowtouched = nullptr;
    p->keyrank = nullptr;
    p->rec = nullptr;
    p->stage = nullptr;
    p->passtot = nullptr;
    p->lstart = nullptr;
    p->pq = nullptr;
    p->pq_cap = 0;
    p->rot_u = p->rot_v = -1;
}

bool dev_alloc(nufft2_plan_s *p, void **ptr, size_t bytes)
{
    if (bytes == 0) bytes = 16;
    if (hipMalloc(ptr, bytes) != hipSuccess) {
        *ptr = nullptr;
        (void)hipGetLastError();
        return false;
    }
    p->ws_bytes += bytes;
    return true;
}

nufft2_status fail_hip(nufft2_plan_s *p, hipError_t e)
{
    p->last_err = e;
    return NUFFT2_ERR_HIP;
}

// Deconvolution factors are a pure function of (K, nf, w, beta); plans of
// the same shape (a serving loop creates many) share one computation.
nufft2_status cached_correction(int64_t K, int64_t nf, int w, double beta, std::vector<double> &out)
{
    struct Entry {
        int64_t K, nf;
        int w;
        double beta;
        std::vector<double> corr;
    };
    static std::mutex mu;
    static std::vector<Entry> cache;
    {
        std::lock_guard<std::mutex> lk(mu);
        for (const Entry &e : cache)
            if (e.K == K && e.nf == nf && e.w == w && e.beta == beta) {
                out = e.corr;
                return NUFFT2_OK;
            }
    }
    out.assign(K, 0.0);
    nufft2_status st = kernel_correction(K, nf, w, beta, out.data());
    if (st != NUFFT2_OK) return st;
    std::lock_guard<std::mutex> lk(mu);
    if (cache.size() < 256) cache.push_back(Entry{K, nf, w, beta, out});
    return NUFFT2_OK;
}

template <typename T> nufft2_status upload_tables(nufft2_plan_s *p)
{
    std::vector<double> ct, cp;
    nufft2_status st = cached_correction(p->Kt, p->nft, p->w, p->beta, ct);
    if (st != NUFFT2_OK) return st;
    st = cached_correction(p->Kp, p->nfp, p->w, p->beta, cp);
    if (st != NUFFT2_OK) return st;
    std::vector<T> ctT(ct.begin(), ct.end()), cpT(cp.begin(), cp.end());
    std::vector<T> twt, twp, twist(4 * (size_t)p->Kt);
    fill_twiddle_tables<T>(twt, p->nft / 2);
    fill_twiddle_tables<T>(twp, 1 << p->fp.log_phi_len);
    {
        const long double two_pi = 6.283185307179586476925286766559005768L;
        for (int64_t a = 0; a < p->Kt; ++a) {
            const long double ang = two_pi * (long double)(a - p->Kt / 2) / (long double)p->nft;
            twist[2 * a] = (T)ct[a];
            twist[2 * a + 1] = (T)0;
            twist[2 * (p->Kt + a)] = (T)((long double)ct[a] * cosl(ang));
            twist[2 * (p->Kt + a) + 1] = (T)((long double)ct[a] * sinl(ang));
        }
    }
    hipError_t e;
    if ((e = hipMemcpy(p->corr_t, ctT.data(), sizeof(T) * ctT.size(), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(p->corr_p, cpT.data(), sizeof(T) * cpT.size(), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(p->tw_t, twt.data(), sizeof(T) * twt.size(), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(p->tw_p, twp.data(), sizeof(T) * twp.size(), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(p->twist_t, twist.data(), sizeof(T) * twist.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return fail_hip(p, e);
    if (p->c2r) {
        std::vector<T> tab(2 * (size_t)p->ncols);
        const long double two_pi = 6.283185307179586476925286766559005768L;
        for (int64_t k = 0; k < p->ncols; ++k) {
            const long double ang = two_pi * (long double)k / (long double)p->nfp;
            tab[2 * k] = (T)cosl(ang);
            tab[2 * k + 1] = (T)sinl(ang);
        }
        if ((e = hipMemcpy(p->c2r, tab.data(), sizeof(T) * tab.size(), hipMemcpyHostToDevice)) != hipSuccess)
            return fail_hip(p, e);
    }
    return NUFFT2_OK;
}

hipEvent_t prof_event(nufft2_plan_s *p)
{
    if (!p->prof_pool.empty()) {
        hipEvent_t e = p->prof_pool.back();
        p->prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

// Open a bracket for `stage` if it is being timed; returns its slot or -1.
int prof_begin(nufft2_plan_s *p, int stage)
{
    if (!(p->prof_mask & (1u << stage))) return -1;
    hipEvent_t a = prof_event(p), b = prof_event(p);
    if (!a || !b || hipEventRecord(a, p->stream) != hipSuccess) {
        if (a) p->prof_pool.push_back(a);
        if (b) p->prof_pool.push_back(b);
        (void)hipGetLastError();
        return -1;
    }
    p->prof_pending.push_back({stage, a, b});
    return (int)p->prof_pending.size() - 1;
}

void prof_end(nufft2_plan_s *p, int slot)
{
    if (slot < 0) return;
    if (hipEventRecord(p->prof_pending[slot].b, p->stream) != hipSuccess) {
        (void)hipGetLastError();
        p->prof_pool.push_back(p->prof_pending[slot].a);
        p->prof_pool.push_back(p->prof_pending[slot].b);
        p->prof_pending.erase(p->prof_pending.begin() + slot);
    }
}

void prof_release_all(nufft2_plan_s *p)
{
    for (auto &br : p->prof_pending) {
        (void)hipEventDestroy(br.a);
        (void)hipEventDestroy(br.b);
    }
    for (hipEvent_t e : p->prof_pool) (void)hipEventDestroy(e);
    p->prof_pending.clear();
    p->prof_pool.clear();
}

int choose_tile(int32_t requested, int dflt, int nf, bool *bad)
{
    int t = requested > 0 ? requested : dflt;
    if (requested > 0 && (!is_pow2(requested) || requested < 4 || requested > 128)) *bad = true;
    if (t > nf) t = nf;
    return t;
}

}  // namespace

// Elements per thread of the FFT passes and the phi pass's rows per
// workgroup, for a launch of `members` plans of p's shape at once: a pass
// that would launch fewer than kSmallLaunchWaves waves with 16 elements per
// thread runs with 8, so that it has about twice the waves to hide LDS and
// memory latency (theta pass: twice the threads per workgroup; phi pass:
// 2048 instead of 4096 elements per workgroup).
void nufft2::fft_launch_shape(const nufft2_plan_s *p, int64_t members, FFTParams &fp)
{
    const int64_t L = p->nft / 2;
    const int64_t max_threads = p->prec == NUFFT2_FP32 ? 1024 : 512;
    const int64_t b = fp.theta_batch;
    const int64_t theta_waves16 = members * 2 * ((p->ncols + b - 1) / b) * (int64_t)p->F * L * b / 16 / 64;
    fp.theta_ept = (theta_waves16 < kSmallLaunchWaves && L * b / 8 <= max_threads && L >= 64) ? 8 : 16;
    const int64_t N = int64_t(1) << fp.log_phi_len;  // phi transform length
    const int64_t phi_waves16 = members * (int64_t)p->F * (p->nft / 2) * N / 16 / 64;
    fp.phi_ept = (phi_waves16 < kSmallLaunchWaves && N >= 64) ? 8 : 16;
    int64_t pb = (fp.phi_ept == 8 ? 2048 : 4096) / N;
    if (pb < 1) pb = 1;
    if (pb > p->nft) pb = p->nft;
    fp.phi_batch = (int)pb;
    fp.log_phi_batch = ilog2(pb);
}

NUFFT2_API const char *nufft2_strerror(nufft2_status s)
{
    switch (s) {
    case NUFFT2_OK: return "ok";
    case NUFFT2_ERR_ARG: return "invalid argument";
    case NUFFT2_ERR_EPS_RANGE: return "tolerance below what the precision can reach";
    case NUFFT2_ERR_ALLOC: return "device allocation failed";
    case NUFFT2_ERR_NO_POINTS: return "exec before setpts";
    case NUFFT2_ERR_NONFINITE: return "non-finite point coordinate";
    case NUFFT2_ERR_HIP: return "HIP runtime or launch error";
    }
    return "unknown status";
}

NUFFT2_API nufft2_status nufft2_kernel_params(nufft2_prec prec, double eps, int32_t *w, double *beta)
{
    if (!w || !beta) return NUFFT2_ERR_ARG;
    return kernel_params(prec, eps, w, beta);
}

NUFFT2_API nufft2_status nufft2_kernel_correction(int64_t K, int64_t nf, int32_t w, double beta,
                                                  double *corr)
{
    return kernel_correction(K, nf, w, beta, corr);
}

namespace {

// Validate the arguments of a plan and fill every parameter of *p (no
// device memory is touched; p's workspace pointers stay null).
nufft2_status plan_configure(nufft2_plan_s *p, int prec, int64_t n_modes_theta, int64_t n_modes_phi,
                             int32_t n_fields, double eps, const nufft2_opts *opts, void *stream)
{
    if (prec != NUFFT2_FP32 && prec != NUFFT2_FP64) return NUFFT2_ERR_ARG;
    if (n_modes_theta <= 0 || n_modes_phi <= 0 || n_fields <= 0) return NUFFT2_ERR_ARG;
    if (n_modes_theta > kMaxNf / 2 || n_modes_phi > kMaxNf / 2) return NUFFT2_ERR_ARG;
    nufft2_opts o{};
    if (opts) o = *opts;
    if ((o.hermitian != 0 && o.hermitian != 1) || (o.m_major != 0 && o.m_major != 1) || o.reserved != 0 ||
        o.w < 0 || o.w > kMaxW || o.w == 1 || o.beta_over_w < 0 ||
        !isfinite(o.beta_over_w) || (o.real_output != 0 && o.real_output != 1))
        return NUFFT2_ERR_ARG;
    // a real field's modes are symmetric about zero: odd counts
    if (o.hermitian && (n_modes_theta % 2 == 0 || n_modes_phi % 2 == 0)) return NUFFT2_ERR_ARG;

    int32_t w;
    double beta;
    nufft2_status st = kernel_params(prec, eps, &w, &beta);
    if (st != NUFFT2_OK) return st;
    if (o.w > 0) w = o.w;
    beta = (o.beta_over_w > 0 ? o.beta_over_w : kDefaultBetaOverW) * w;

    auto fine = [&](int64_t K) {
        int64_t n = 2 * K;
        if (n < 2 * w) n = 2 * w;
        if (n < 32) n = 32;
        return int64_t(1) << ilog2(n);
    };
    const int64_t nft = fine(n_modes_theta), nfp = fine(n_modes_phi);
    if (nft > kMaxNf || nfp > kMaxNf) return NUFFT2_ERR_ARG;
    if ((int64_t)n_fields * nft * nfp > (int64_t(1) << 34)) return NUFFT2_ERR_ARG;

    bool bad_tile = false;
    const int tt = choose_tile(o.tile_theta,
                               o.hermitian ? (prec == NUFFT2_FP32 ? kDefaultTileThetaReal32 : kDefaultTileThetaReal64)
                                           : kDefaultTileTheta,
                               (int)nft, &bad_tile);
    const int tp = choose_tile(o.tile_phi,
                               o.hermitian ? (prec == NUFFT2_FP32 ? kDefaultTilePhiReal32 : kDefaultTilePhiReal64)
                                           : kDefaultTilePhi,
                               (int)nfp, &bad_tile);
    if (bad_tile) return NUFFT2_ERR_ARG;
    {
        // the gather stages a (tile + w - 1)^2 patch of one field in LDS
        const size_t cs = prec == NUFFT2_FP32 ? sizeof(float2) : sizeof(double2);
        const size_t es = o.hermitian ? cs / 2 : cs;
        const size_t v = 16 / es;  // elements per 16-byte staging chunk
        if (es * (size_t)(tt + w - 1) * ((tp + w - 1 + v - 1) / v * v) > kGatherLdsLimit) return NUFFT2_ERR_ARG;
    }

    p->prec = prec;
    p->Kt = n_modes_theta;
    p->Kp = n_modes_phi;
    p->F = n_fields;
    p->w = w;
    p->beta = beta;
    p->nft = (int)nft;
    p->nfp = (int)nfp;
    p->tile_t = tt;
    p->tile_p = tp;
    p->nbins_t = (int)(nft / tt);
    p->nbins_p = (int)(nfp / tp);
    p->nbins = (int64_t)p->nbins_t * p->nbins_p;
    p->hermitian = o.hermitian;
    p->real_output = o.real_output || o.hermitian;
    p->ncols = o.hermitian ? n_modes_phi / 2 + 1 : n_modes_phi;
    p->stream = (hipStream_t)stream;
    p->csize = prec == NUFFT2_FP32 ? sizeof(float2) : sizeof(double2);
    p->rsize = prec == NUFFT2_FP32 ? sizeof(float) : sizeof(double);
    p->gsize = o.hermitian ? p->rsize : p->csize;
    if (hipGetDevice(&p->device) != hipSuccess) {
        (void)hipGetLastError();
        return NUFFT2_ERR_HIP;
    }

    FFTParams &fp = p->fp;
    fp.Kt = (int)p->Kt;
    fp.Kp = (int)p->Kp;
    fp.nft = p->nft;
    fp.nfp = p->nfp;
    fp.log_nft = ilog2(p->nft);
    fp.log_nfp = ilog2(p->nfp);
    fp.n_fields = p->F;
    fp.col0 = o.hermitian ? (int)(p->Kp / 2) : 0;
    fp.ncols = (int)p->ncols;
    fp.m_major = o.m_major;
    fp.c2r = o.hermitian;
    fp.log_phi_len = fp.log_nfp - (o.hermitian ? 1 : 0);
    {
        // theta pass: columns per workgroup so that a row segment is >= 64 bytes
        // where possible, at least 64 threads, at most 1024 (FP32) or 512 (FP64)
        // threads, and within the per-workgroup LDS limit (data, twiddle
        // tables, row flags).  Fewer, larger workgroups measured faster than
        // smaller ones that share a CU, except where one workgroup would take
        // more than half of the CU's LDS: there two workgroups of half the
        // columns (32-byte segments), one loading while the other transforms,
        // measured 5-7% faster (length 4096 transforms).
        const int64_t L = p->nft / 2;
        const int64_t max_threads = prec == NUFFT2_FP32 ? 1024 : 512;
        auto lds_bytes = [&](int64_t b) {
            return (int64_t)p->csize * ((L + L / 32) * b + 64 + (L > 64 ? L / 64 : 1)) + ((L + 15) & ~15);
        };
        int64_t b = prec == NUFFT2_FP32 ? 8 : 4;
        while (L * b < 1024) b *= 2;
        while (b > 1 && (L * b / 16 > max_threads || lds_bytes(b) > (int64_t)kFftLdsLimit)) b /= 2;
        while (lds_bytes(b) > (int64_t)kCuLds / 2 && b * (int64_t)p->csize > 32) b /= 2;
        if (lds_bytes(b) > (int64_t)kFftLdsLimit || L * b / 16 > max_threads) return NUFFT2_ERR_ARG;
        fp.theta_batch = (int)b;
        fp.log_theta_batch = ilog2(b);
    }
    fft_launch_shape(p, 1, fp);
    {
        // Patch rows of 16-byte elements (complex FP64) are padded to a
        // multiple of 16 elements: the LDS serves 16-byte reads 16 lanes at a
        // time over 64 banks, and with such a pitch the bank slot of a tap
        // depends on its column only, which the gather's lane dealing keeps
        // distinct (a CPU model of the 2048^2 wind workload that reproduces
        // the measured FP64 conflict rate, 0.79 per access, puts it at
        // 0.25).  Only where the padded patch of one field stays within the
        // LDS limit.
        // Other rows hold whole 16-byte staging chunks.
        const int tc = tp + w - 1;
        const int padded = (tc + 15) & ~15;
        const int v = (int)(16 / p->gsize);
        p->tile_pitch = p->gsize == 16 ? (p->gsize * (size_t)(tt + w - 1) * (size_t)padded <= kGatherLdsLimit ? padded : tc)
                                       : (tc + v - 1) / v * v;
        const size_t tile = p->gsize * (size_t)(tt + w - 1) * (size_t)p->tile_pitch;
        int g = (int)(kGatherLdsLimit / tile);
        if (g > kGatherMaxFieldsPerPass) g = kGatherMaxFieldsPerPass;
        if (g > p->F) g = p->F;
        if (g < 1) g = 1;
        p->fields_per_pass = g;
    }
    return NUFFT2_OK;
}

// The plan's device workspaces (not the point workspaces), each from
// get(&ptr, bytes): the allocating plan passes dev_alloc, the allocation-
// free entry point a carve-out of its static scratch.  False if get fails.
template <class Get> bool plan_workspaces(nufft2_plan_s *p, size_t n_poly, Get get)
{
    const size_t rs = p->rsize, cs = p->csize, gs = p->gsize;
    // the tables first: their offsets then depend on the table parameters only
    return get((void **)&p->corr_t, rs * p->Kt) && get((void **)&p->corr_p, rs * p->Kp) &&
           get((void **)&p->tw_t, cs * (64 + p->nft)) && get((void **)&p->tw_p, cs * (64 + p->nfp)) &&
           get((void **)&p->twist_t, 2 * cs * p->Kt) &&
           (!p->hermitian || get((void **)&p->c2r, cs * (size_t)p->ncols)) &&
           (n_poly == 0 || get((void **)&p->wpoly, sizeof(float) * n_poly)) &&
           get((void **)&p->S, cs * (size_t)p->F * p->nft * p->ncols) &&
           get((void **)&p->grid, gs * (size_t)p->F * p->nft * p->nfp) &&
           get((void **)&p->bincount, sizeof(int32_t) * (size_t)p->nbins) &&
           get((void **)&p->binstart, sizeof(int32_t) * (size_t)(p->nbins + 1)) &&
           get((void **)&p->binlist, binlist_bytes(p->nbins)) && get((void **)&p->rowmark, (size_t)p->nft) &&
           get((void **)&p->rowtouched, (size_t)p->nft) && get((void **)&p->flags, sizeof(int32_t) * 4) &&
           (p->nbins <= kDealtMaxBins ||
            (get((void **)&p->stage, sizeof(int4) * (size_t)p->nbins) &&
             get((void **)&p->lstart, sizeof(int32_t) * (size_t)p->nbins) &&
             get((void **)&p->passtot, sizeof(int2) * (size_t)scan_passes(p->nbins))));
}

// Device work of a new plan's set-up on its stream: tables, polynomial
// coefficients, and the counters, flags and buffers that must start at
// zero (S and the grid: so that reads of rows no point reaches are defined).
nufft2_status plan_initialise(nufft2_plan_s *p, const std::vector<float> &wpoly, bool clear_grids)
{
    nufft2_status st = p->prec == NUFFT2_FP32 ? upload_tables<float>(p) : upload_tables<double>(p);
    if (st == NUFFT2_OK && p->wpoly) {
        const hipError_t e = hipMemcpy(p->wpoly, wpoly.data(), sizeof(float) * wpoly.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) st = fail_hip(p, e);
    }
    if (st != NUFFT2_OK) return st;
    hipError_t e;
    hipStream_t ps = p->stream;
    if ((clear_grids &&
         ((e = hipMemsetAsync(p->S, 0, p->csize * (size_t)p->F * p->nft * p->ncols, ps)) != hipSuccess ||
          (e = hipMemsetAsync(p->grid, 0, p->gsize * (size_t)p->F * p->nft * p->nfp, ps)) != hipSuccess)) ||
        (e = hipMemsetAsync(p->rowtouched, 0, (size_t)p->nft, ps)) != hipSuccess ||
        (e = hipMemsetAsync(p->rowmark, 0, (size_t)p->nft, ps)) != hipSuccess ||
        (e = hipMemsetAsync(p->bincount, 0, sizeof(int32_t) * (size_t)p->nbins, ps)) != hipSuccess ||
        (e = hipMemsetAsync(p->binstart, 0, sizeof(int32_t) * (size_t)(p->nbins + 1), ps)) != hipSuccess ||
        (e = hipMemsetAsync(p->binlist, 0, binlist_bytes(p->nbins), ps)) != hipSuccess ||
        (e = hipMemsetAsync(p->flags, 0, sizeof(int32_t) * 4, ps)) != hipSuccess)
        return fail_hip(p, e);
    return NUFFT2_OK;
}

}  // namespace

NUFFT2_API nufft2_status nufft2_plan(nufft2_prec prec, int64_t n_modes_theta, int64_t n_modes_phi,
                                     int32_t n_fields, double eps, const nufft2_opts *opts,
                                     void *stream, nufft2_handle *out)
{
    if (!out) return NUFFT2_ERR_ARG;
    nufft2_plan_s *p = new (std::nothrow) nufft2_plan_s();
    if (!p) return NUFFT2_ERR_ALLOC;
    nufft2_status st = plan_configure(p, prec, n_modes_theta, n_modes_phi, n_fields, eps, opts, stream);
    if (st != NUFFT2_OK) {
        delete p;
        return st;
    }
    std::vector<float> wpoly;
    const bool use_poly = poly_table_floats(prec, p->w) > 0 && weight_polynomials(prec, p->w, p->beta, wpoly);
    if (!plan_workspaces(p, use_poly ? wpoly.size() : 0, [&](void **q, size_t n) { return dev_alloc(p, q, n); })) {
        free_all(p);
        delete p;
        return NUFFT2_ERR_ALLOC;
    }
    // cleared on the plan's stream, which is then synchronised: work on
    // other streams (other plans) keeps running meanwhile
    st = plan_initialise(p, wpoly, true);
    if (st == NUFFT2_OK) {
        const hipError_t e = hipStreamSynchronize(p->stream);
        if (e != hipSuccess) st = fail_hip(p, e);
    }
    if (st != NUFFT2_OK) {
        free_all(p);
        delete p;
        return st;
    }
    *out = p;
    return NUFFT2_OK;
}

nufft2_status nufft2::plan_reserve_points(nufft2_plan_s *p, int64_t n_pts)
{
    if (n_pts <= p->pts_cap) return NUFFT2_OK;
    // grow the point workspaces; wait for work that may still use them
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return fail_hip(p, e);
    void *ptrs[] = {p->keyrank, p->rec, p->perm};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    p->ws_bytes -= (size_t)p->pts_cap * (sizeof(int2) + 2 * p->rsize + 8 + sizeof(int32_t));
    p->keyrank = nullptr;
    p->rec = nullptr;
    p->perm = nullptr;
    p->pts_cap = 0;
    p->n_pts = -1;
    const size_t recsz = p->prec == NUFFT2_FP32 ? sizeof(PointRec<float>) : sizeof(PointRec<double>);
    const size_t before = p->ws_bytes;
    if (!dev_alloc(p, (void **)&p->keyrank, sizeof(int2) * (size_t)n_pts) ||
        !dev_alloc(p, &p->rec, recsz * (size_t)n_pts) ||
        !dev_alloc(p, (void **)&p->perm, sizeof(int32_t) * (size_t)n_pts)) {
        void *q2[] = {p->keyrank, p->rec, p->perm};
        for (void *q : q2)
            if (q) (void)hipFree(q);
        p->keyrank = nullptr;
        p->rec = nullptr;
        p->perm = nullptr;
        p->ws_bytes = before;
        return NUFFT2_ERR_ALLOC;
    }
    p->ws_bytes = before + (size_t)n_pts * (sizeof(int2) + 2 * p->rsize + 8 + sizeof(int32_t));
    p->pts_cap = n_pts;
    return NUFFT2_OK;
}

SetptsParams nufft2::plan_setpts_params(const nufft2_plan_s *p, int64_t n_pts)
{
    SetptsParams sp{};
    const double inv_two_pi = 0.15915494309189533576888376337251436;
    sp.th.to_grid = (double)p->nft * inv_two_pi;
    sp.th.inv_nf = 1.0 / (double)p->nft;
    sp.th.nf = p->nft;
    sp.th.tile = p->tile_t;
    sp.ph.to_grid = (double)p->nfp * inv_two_pi;
    sp.ph.inv_nf = 1.0 / (double)p->nfp;
    sp.ph.nf = p->nfp;
    sp.ph.tile = p->tile_p;
    sp.w = p->w;
    sp.nbins_phi = p->nbins_p;
    sp.n = n_pts;
    return sp;
}

GatherParams nufft2::plan_gather_params(const nufft2_plan_s *p)
{
    GatherParams gp{};
    gp.nft = p->nft;
    gp.nfp = p->nfp;
    gp.tile_t = p->tile_t;
    gp.tile_p = p->tile_p;
    gp.nbins_phi = p->nbins_p;
    gp.nbins = p->nbins;
    gp.w = p->w;
    gp.beta = p->beta;
    gp.n_fields = p->F;
    gp.fields_per_pass = p->fields_per_pass;
    gp.tile_pitch = p->tile_pitch;
    gp.n_pts = p->n_pts;
    gp.real_output = p->real_output;
    gp.real_grid = p->hermitian;
    gp.wpoly = p->wpoly;
    gp.pq = p->rot_u >= 0 ? p->pq : nullptr;
    gp.rot_u = p->rot_u;
    gp.rot_v = p->rot_v;
    return gp;
}

namespace {

// Set-up of the points, with the vector rotation's (p, q) pairs when
// phi_a != nullptr (pq then has room for n_pts pairs).
nufft2_status setpts_impl(nufft2_plan_s *p, int64_t n_pts, const double *phi_dev, const double *theta_dev,
                          const double *phi_a, const double *theta_a)
{
    nufft2_status st = plan_reserve_points(p, n_pts);
    if (st != NUFFT2_OK) return st;
    SetptsParams sp = plan_setpts_params(p, n_pts);
    if (phi_a) {
        sp.phi_a = phi_a;
        sp.theta_a = theta_a;
        sp.pq = p->pq;
    }
    const int slot = prof_begin(p, 0);
    hipError_t e = launch_setpts(p->prec, sp, phi_dev, theta_dev, p->bincount, p->binstart, p->binlist, p->nbins,
                                 p->keyrank, p->rowmark, p->rowtouched, p->rec, p->perm, p->flags, p->stage,
                                 p->passtot, p->lstart, p->stream);
    prof_end(p, slot);
    if (e != hipSuccess) return fail_hip(p, e);
    p->n_pts = n_pts;
    return NUFFT2_OK;
}

}  // namespace

NUFFT2_API nufft2_status nufft2_setpts(nufft2_handle p, int64_t n_pts, const double *phi_dev,
                                       const double *theta_dev)
{
    if (!p || n_pts < 0 || n_pts > (int64_t)0x7fffffff) return NUFFT2_ERR_ARG;
    if (n_pts > 0 && (!phi_dev || !theta_dev)) return NUFFT2_ERR_ARG;
    p->rot_u = p->rot_v = -1;
    return setpts_impl(p, n_pts, phi_dev, theta_dev, nullptr, nullptr);
}

NUFFT2_API nufft2_status nufft2_setpts_vector(nufft2_handle p, int64_t n_pts, const double *phi_dev,
                                              const double *theta_dev, const double *phi_a_dev,
                                              const double *theta_a_dev, int32_t field_u, int32_t field_v)
{
    if (!p || n_pts < 0 || n_pts > (int64_t)0x7fffffff) return NUFFT2_ERR_ARG;
    if (n_pts > 0 && (!phi_dev || !theta_dev || !phi_a_dev || !theta_a_dev)) return NUFFT2_ERR_ARG;
    if (field_u < 0 || field_u >= p->F || field_v < 0 || field_v >= p->F || field_u == field_v) return NUFFT2_ERR_ARG;
    // the gather rotates the pair in its epilogue: both fields in one pass
    if (field_u / p->fields_per_pass != field_v / p->fields_per_pass) return NUFFT2_ERR_ARG;
    p->rot_u = p->rot_v = -1;
    if (n_pts > p->pq_cap) {
        hipError_t e = hipStreamSynchronize(p->stream);
        if (e != hipSuccess) return fail_hip(p, e);
        if (p->pq) (void)hipFree(p->pq);
        p->ws_bytes -= 2 * p->rsize * (size_t)p->pq_cap;
        p->pq = nullptr;
        p->pq_cap = 0;
        if (!dev_alloc(p, &p->pq, 2 * p->rsize * (size_t)n_pts)) return NUFFT2_ERR_ALLOC;
        p->pq_cap = n_pts;
    }
    nufft2_status st = setpts_impl(p, n_pts, phi_dev, theta_dev, n_pts > 0 ? phi_a_dev : nullptr, theta_a_dev);
    if (st != NUFFT2_OK) return st;
    p->rot_u = field_u;
    p->rot_v = field_v;
    return NUFFT2_OK;
}

NUFFT2_API nufft2_status nufft2_exec(nufft2_handle p, const void *coeffs_dev, void *out_dev)
{
    if (!p) return NUFFT2_ERR_ARG;
    if (p->n_pts < 0) return NUFFT2_ERR_NO_POINTS;
    if (p->n_pts == 0) return NUFFT2_OK;
    if (!coeffs_dev || !out_dev) return NUFFT2_ERR_ARG;
    int slot = prof_begin(p, 1);
    hipError_t e = launch_theta_pass(p->prec, p->fp, coeffs_dev, p->twist_t, p->corr_p, p->tw_t,
                                     p->rowtouched, p->S, p->stream);
    prof_end(p, slot);
    if (e != hipSuccess) return fail_hip(p, e);
    slot = prof_begin(p, 2);
    e = launch_phi_pass(p->prec, p->fp, p->S, p->tw_p, p->c2r, p->rowtouched, p->grid, p->stream);
    prof_end(p, slot);
    if (e != hipSuccess) return fail_hip(p, e);
    const GatherParams gp = plan_gather_params(p);
    slot = prof_begin(p, 3);
    e = launch_gather(p->prec, gp, p->grid, p->rec, p->perm, p->binlist, out_dev,
                      p->stream);
    prof_end(p, slot);
    if (e != hipSuccess) return fail_hip(p, e);
    return NUFFT2_OK;
}

NUFFT2_API nufft2_status nufft2_rotate_uv(nufft2_handle p, void *out_dev, int32_t field_u, int32_t field_v,
                                          const double *phi_a_dev, const double *theta_a_dev,
                                          const double *phi_d_dev, const double *theta_d_dev)
{
    if (!p) return NUFFT2_ERR_ARG;
    if (p->n_pts < 0) return NUFFT2_ERR_NO_POINTS;
    if (field_u < 0 || field_u >= p->F || field_v < 0 || field_v >= p->F || field_u == field_v)
        return NUFFT2_ERR_ARG;
    if (p->n_pts == 0) return NUFFT2_OK;
    if (!out_dev || !phi_a_dev || !theta_a_dev || !phi_d_dev || !theta_d_dev) return NUFFT2_ERR_ARG;
    const int comps = p->real_output ? 1 : 2;
    const size_t field_bytes = p->rsize * comps * (size_t)p->n_pts;
    char *base = (char *)out_dev;
    const hipError_t e = launch_rotate_uv(p->prec, base + field_bytes * field_u, base + field_bytes * field_v, comps,
                                          p->n_pts, phi_a_dev, theta_a_dev, phi_d_dev, theta_d_dev, p->stream);
    if (e != hipSuccess) return fail_hip(p, e);
    return NUFFT2_OK;
}

NUFFT2_API nufft2_status nufft2_check(nufft2_handle p)
{
    if (!p) return NUFFT2_ERR_ARG;
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return fail_hip(p, e);
    if (p->last_err != hipSuccess) return NUFFT2_ERR_HIP;
    int32_t flags = 0;  // flags[1]: published by the last setpts
    e = hipMemcpy(&flags, p->flags + 1, sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail_hip(p, e);
    if (p->n_pts > 0 && (flags & 1)) return NUFFT2_ERR_NONFINITE;
    return NUFFT2_OK;
}

NUFFT2_API nufft2_status nufft2_set_stream(nufft2_handle p, void *stream)
{
    if (!p) return NUFFT2_ERR_ARG;
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return fail_hip(p, e);
    p->stream = (hipStream_t)stream;
    return NUFFT2_OK;
}

NUFFT2_API nufft2_status nufft2_destroy(nufft2_handle p)
{
    if (!p) return NUFFT2_OK;
    (void)hipStreamSynchronize(p->stream);
    prof_release_all(p);
    free_all(p);
    delete p;
    return NUFFT2_OK;
}

NUFFT2_API nufft2_status nufft2_profile_enable(nufft2_handle p, uint32_t stage_mask)
{
    if (!p || (stage_mask >> NUFFT2_N_STAGES) != 0) return NUFFT2_ERR_ARG;
    p->prof_mask = stage_mask;
    return NUFFT2_OK;
}

NUFFT2_API nufft2_status nufft2_profile_read(nufft2_handle p, double *total_ms, int64_t *count)
{
    if (!p || !total_ms || !count) return NUFFT2_ERR_ARG;
    for (int i = 0; i < NUFFT2_N_STAGES; ++i) {
        total_ms[i] = 0.0;
        count[i] = 0;
    }
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return fail_hip(p, e);
    for (auto &br : p->prof_pending) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, br.a, br.b) == hipSuccess) {
            total_ms[br.stage] += ms;
            count[br.stage] += 1;
        } else {
            (void)hipGetLastError();
        }
        p->prof_pool.push_back(br.a);
        p->prof_pool.push_back(br.b);
    }
    p->prof_pending.clear();
    return NUFFT2_OK;
}

NUFFT2_API nufft2_status nufft2_get_info(nufft2_handle p, nufft2_info *info)
{
    if (!p || !info) return NUFFT2_ERR_ARG;
    memset(info, 0, sizeof(*info));
    info->prec = p->prec;
    info->w = p->w;
    info->beta = p->beta;
    info->n_modes_theta = p->Kt;
    info->n_modes_phi = p->Kp;
    info->nf_theta = p->nft;
    info->nf_phi = p->nfp;
    info->n_fields = p->F;
    info->real_output = p->real_output;
    info->tile_theta = p->tile_t;
    info->tile_phi = p->tile_p;
    info->n_bins = p->nbins;
    info->n_pts = p->n_pts;
    info->workspace_bytes = p->ws_bytes;
    info->last_hip_error = (int32_t)p->last_err;
    info->device = p->device;
    info->hermitian = p->hermitian;
    info->fields_per_pass = p->fields_per_pass;
    info->m_major = p->fp.m_major;
    return NUFFT2_OK;
}

NUFFT2_API nufft2_status nufft2_debug_buffer(nufft2_handle p, int32_t which, void **dev_ptr,
                                             uint64_t *bytes)
{
    if (!p || !dev_ptr || !bytes) return NUFFT2_ERR_ARG;
    const bool needs_pts = (which >= 1 && which <= 4) || which == 6;
    if (needs_pts && p->n_pts < 0) return NUFFT2_ERR_NO_POINTS;
    const size_t recsz = p->prec == NUFFT2_FP32 ? sizeof(PointRec<float>) : sizeof(PointRec<double>);
    switch (which) {
    case 0: *dev_ptr = p->grid; *bytes = p->gsize * (size_t)p->F * p->nft * p->nfp; break;
    case 1: *dev_ptr = p->rec; *bytes = recsz * (size_t)p->n_pts; break;
    case 2: *dev_ptr = p->perm; *bytes = sizeof(int32_t) * (size_t)p->n_pts; break;
    case 3: *dev_ptr = p->binstart; *bytes = sizeof(int32_t) * (size_t)(p->nbins + 1); break;
    case 4: *dev_ptr = p->rowtouched; *bytes = (size_t)p->nft; break;
    case 5: *dev_ptr = p->S; *bytes = p->csize * (size_t)p->F * p->nft * p->ncols; break;
    case 6: *dev_ptr = p->binlist; *bytes = sizeof(int32_t) * (size_t)(p->nbins + 1); break;
    default: return NUFFT2_ERR_ARG;
    }
    return NUFFT2_OK;
}

// ---- evaluation without device allocation ---------------------------------

namespace {

// Device memory of nufft2_exec_noalloc: every workspace of one evaluation
// (tables, sorted points, bins, theta-pass output, fine grid) is carved
// from this array.  Each GPU the library runs on holds its own copy until
// the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns for that device.
constexpr size_t kNoAllocScratchBytes = size_t(128) << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kNoAllocMaxDevices = 64;

// What the tables at the start of a device's scratch describe.
struct TableKey {
    int prec = 0, w = 0, hermitian = 0, nft = 0, nfp = 0;
    int64_t Kt = 0, Kp = 0;
    double beta = 0;
    bool operator==(const TableKey &o) const
    {
        return prec == o.prec && w == o.w && hermitian == o.hermitian && nft == o.nft && nfp == o.nfp &&
               Kt == o.Kt && Kp == o.Kp && beta == o.beta;
    }
};

struct ScratchDevice {
    unsigned char *ptr = nullptr;  // this device's copy of scratch
    bool tables_valid = false;
    bool poly = false;             // the tables include tap-weight polynomials
    TableKey tables;
};

std::mutex g_scratch_mu;
ScratchDevice g_scratch[kNoAllocMaxDevices];

}  // namespace

NUFFT2_API nufft2_status nufft2_exec_noalloc(nufft2_prec prec, int64_t n_modes_theta, int64_t n_modes_phi,
                                             int32_t n_fields, double eps, const nufft2_opts *opts, int64_t n_pts,
                                             const double *phi_dev, const double *theta_dev, const void *coeffs_dev,
                                             void *out_dev, void *stream)
{
    if (n_pts < 0 || n_pts > (int64_t)0x7fffffff) return NUFFT2_ERR_ARG;
    if (n_pts > 0 && (!phi_dev || !theta_dev || !coeffs_dev || !out_dev)) return NUFFT2_ERR_ARG;
    nufft2_plan_s p;  // parameters only; its pointers are set into the scratch below
    nufft2_status st = plan_configure(&p, prec, n_modes_theta, n_modes_phi, n_fields, eps, opts, stream);
    if (st != NUFFT2_OK) return st;
    if (n_pts == 0) return NUFFT2_OK;
    if (p.device < 0 || p.device >= kNoAllocMaxDevices) return NUFFT2_ERR_ARG;

    std::lock_guard<std::mutex> lk(g_scratch_mu);
    ScratchDevice &dev = g_scratch[p.device];
    if (!dev.ptr) {
        // once per device, with that device current
        void *q = nullptr;
        const hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !q) {
            (void)hipGetLastError();
            return NUFFT2_ERR_HIP;
        }
        dev.ptr = (unsigned char *)q;
    }
    // carve the workspaces (256-byte aligned) in a fixed order: tables,
    // plan buffers, then the point buffers
    size_t used = 0;
    auto carve = [&](void **q, size_t n) {
        const size_t at = (used + 255) & ~(size_t)255;
        if (n > kNoAllocScratchBytes || at > kNoAllocScratchBytes - n) return false;
        *q = dev.ptr + at;
        used = at + n;
        return true;
    };
    const size_t n_poly = poly_table_floats(p.prec, p.w);
    const size_t recsz = p.prec == NUFFT2_FP32 ? sizeof(PointRec<float>) : sizeof(PointRec<double>);
    if (!plan_workspaces(&p, n_poly, carve) || !carve((void **)&p.keyrank, sizeof(int2) * (size_t)n_pts) ||
        !carve(&p.rec, recsz * (size_t)n_pts) || !carve((void **)&p.perm, sizeof(int32_t) * (size_t)n_pts))
        return NUFFT2_ERR_ARG;  // the evaluation does not fit in kNoAllocScratchBytes
    p.pts_cap = n_pts;
    p.n_pts = n_pts;

    // tables: uploaded only when they differ from the last call's on this
    // device (host-side work and the blocking copies happen then only)
    TableKey key;
    key.prec = p.prec;
    key.w = p.w;
    key.hermitian = p.hermitian;
    key.nft = p.nft;
    key.nfp = p.nfp;
    key.Kt = p.Kt;
    key.Kp = p.Kp;
    key.beta = p.beta;
    hipError_t e;
    if (!dev.tables_valid || !(dev.tables == key)) {
        dev.tables_valid = false;
        std::vector<float> wpoly;
        if (n_poly && !weight_polynomials(p.prec, p.w, p.beta, wpoly)) p.wpoly = nullptr;
        // earlier work on this stream may still read the old tables
        if ((e = hipStreamSynchronize(p.stream)) != hipSuccess) {
            (void)hipGetLastError();
            return NUFFT2_ERR_HIP;
        }
        st = p.prec == NUFFT2_FP32 ? upload_tables<float>(&p) : upload_tables<double>(&p);
        if (st == NUFFT2_OK && p.wpoly &&
            (e = hipMemcpy(p.wpoly, wpoly.data(), sizeof(float) * wpoly.size(), hipMemcpyHostToDevice)) != hipSuccess)
            st = NUFFT2_ERR_HIP;
        if (st != NUFFT2_OK) {
            (void)hipGetLastError();
            return st;
        }
        dev.tables = key;
        dev.poly = p.wpoly != nullptr;
        dev.tables_valid = true;
    } else if (!dev.poly) {
        p.wpoly = nullptr;
    }
    // The scratch keeps the last call's contents: the counters, row marks,
    // bin lists and flags that the sort expects at zero are cleared here.
    if ((e = hipMemsetAsync(p.rowtouched, 0, (size_t)p.nft, p.stream)) != hipSuccess ||
        (e = hipMemsetAsync(p.rowmark, 0, (size_t)p.nft, p.stream)) != hipSuccess ||
        (e = hipMemsetAsync(p.bincount, 0, sizeof(int32_t) * (size_t)p.nbins, p.stream)) != hipSuccess ||
        (e = hipMemsetAsync(p.binstart, 0, sizeof(int32_t) * (size_t)(p.nbins + 1), p.stream)) != hipSuccess ||
        (e = hipMemsetAsync(p.binlist, 0, binlist_bytes(p.nbins), p.stream)) != hipSuccess ||
        (e = hipMemsetAsync(p.flags, 0, sizeof(int32_t) * 4, p.stream)) != hipSuccess) {
        (void)hipGetLastError();
        return NUFFT2_ERR_HIP;
    }
    const SetptsParams sp = plan_setpts_params(&p, n_pts);
    e = launch_setpts(p.prec, sp, phi_dev, theta_dev, p.bincount, p.binstart, p.binlist, p.nbins, p.keyrank,
                      p.rowmark, p.rowtouched, p.rec, p.perm, p.flags, p.stage, p.passtot, p.lstart, p.stream);
    if (e == hipSuccess)
        e = launch_theta_pass(p.prec, p.fp, coeffs_dev, p.twist_t, p.corr_p, p.tw_t, p.rowtouched, p.S, p.stream);
    if (e == hipSuccess) e = launch_phi_pass(p.prec, p.fp, p.S, p.tw_p, p.c2r, p.rowtouched, p.grid, p.stream);
    if (e == hipSuccess) {
        const GatherParams gp = plan_gather_params(&p);
        e = launch_gather(p.prec, gp, p.grid, p.rec, p.perm, p.binlist, out_dev, p.stream);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return NUFFT2_ERR_HIP;
    }
    return NUFFT2_OK;
}

NUFFT2_API nufft2_status nufft2_noalloc_capacity(uint64_t *bytes)
{
    if (!bytes) return NUFFT2_ERR_ARG;
    *bytes = kNoAllocScratchBytes;
    return NUFFT2_OK;
}

// ---- DFS analysis plans ------------------------------------------------------

struct nufft2_analysis_s {
    int prec = 0;
    int J = 0, F = 0;
    hipStream_t stream = nullptr;
    void *tws = nullptr, *phase = nullptr, *A = nullptr;
    int32_t *cut = nullptr;  // zonal filter: kept |m| per row
    bool zonal = false;
    int m_major = 0;         // output layout
};

namespace {

void analysis_free(nufft2_analysis_s *a)
{
    if (a->tws) (void)hipFree(a->tws);
    if (a->phase) (void)hipFree(a->phase);
    if (a->A) (void)hipFree(a->A);
    if (a->cut) (void)hipFree(a->cut);
    delete a;
}

template <typename T> hipError_t analysis_tables(nufft2_analysis_s *a)
{
    const int L = 2 * a->J, K = 2 * a->J - 1;
    std::vector<T> tw, ph(2 * (size_t)K);
    fill_twiddle_tables<T>(tw, L);
    const long double pi = 3.141592653589793238462643383279502884L;
    const long double norm = 1.0L / ((long double)L * (long double)L);
    for (int q = 0; q < K; ++q) {
        const long double ang = -(long double)(q - (a->J - 1)) * pi / (long double)L;
        ph[2 * q] = (T)(cosl(ang) * norm);
        ph[2 * q + 1] = (T)(sinl(ang) * norm);
    }
    hipError_t e = hipMemcpy(a->tws, tw.data(), sizeof(T) * tw.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(a->phase, ph.data(), sizeof(T) * ph.size(), hipMemcpyHostToDevice);
    return e;
}

}  // namespace

NUFFT2_API nufft2_status nufft2_analysis_plan(nufft2_prec prec, int64_t J, int32_t n_fields, void *stream,
                                              nufft2_analysis *out)
{
    if (!out || (prec != NUFFT2_FP32 && prec != NUFFT2_FP64) || n_fields < 1 || J < 16 || J > 2048 ||
        !is_pow2(J))
        return NUFFT2_ERR_ARG;
    nufft2_analysis_s *a = new (std::nothrow) nufft2_analysis_s();
    if (!a) return NUFFT2_ERR_ALLOC;
    a->prec = prec;
    a->J = (int)J;
    a->F = n_fields;
    a->stream = (hipStream_t)stream;
    const size_t cs = prec == NUFFT2_FP32 ? sizeof(float2) : sizeof(double2);
    const size_t K = 2 * (size_t)J - 1;
    if (hipMalloc(&a->tws, cs * (64 + 2 * (size_t)J)) != hipSuccess || hipMalloc(&a->phase, cs * K) != hipSuccess ||
        hipMalloc(&a->A, cs * (size_t)n_fields * J * (2 * (size_t)J)) != hipSuccess ||  // 2J x J: blocked layout
        hipMalloc(&a->cut, sizeof(int32_t) * (size_t)J) != hipSuccess) {
        (void)hipGetLastError();
        analysis_free(a);
        return NUFFT2_ERR_ALLOC;
    }
    const hipError_t e = prec == NUFFT2_FP32 ? analysis_tables<float>(a) : analysis_tables<double>(a);
    if (e != hipSuccess) {
        analysis_free(a);
        return NUFFT2_ERR_HIP;
    }
    *out = a;
    return NUFFT2_OK;
}

NUFFT2_API nufft2_status nufft2_analysis_exec(nufft2_analysis a, const void *values_dev, void *coeffs_dev)
{
    if (!a || !values_dev || !coeffs_dev) return NUFFT2_ERR_ARG;
    AnalysisParams ap{};
    ap.J = a->J;
    ap.log_len = ilog2(2 * (int64_t)a->J);
    ap.n_fields = a->F;
    ap.zonal_cut = a->zonal ? a->cut : nullptr;
    ap.m_major = a->m_major;
    const hipError_t e = launch_analysis(a->prec, ap, values_dev, a->tws, a->phase, a->A, coeffs_dev, a->stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return NUFFT2_ERR_HIP;
    }
    return NUFFT2_OK;
}

// Zonal filter (section 4): M_zf(theta_i) = min(M, M0 + M sin theta_i) with
// M = J - 1 at the Grid [0] colatitudes; row i keeps |m| <= floor(M_zf).
NUFFT2_API nufft2_status nufft2_analysis_set_zonal_filter(nufft2_analysis a, int32_t M0)
{
    if (!a) return NUFFT2_ERR_ARG;
    if (M0 < 0) {
        a->zonal = false;
        return NUFFT2_OK;
    }
    const double pi = 3.14159265358979323846;
    const int M = a->J - 1;
    std::vector<int32_t> cut(a->J);
    for (int i = 0; i < a->J; ++i) {
        const double theta = ((double)i + 0.5) * pi / (double)a->J;
        double lim = (double)M0 + (double)M * sin(theta);
        if (lim > (double)M) lim = (double)M;
        cut[i] = (int32_t)floor(lim);
    }
    // ordered after earlier work on the plan's stream that reads the table
    if (hipStreamSynchronize(a->stream) != hipSuccess ||
        hipMemcpy(a->cut, cut.data(), sizeof(int32_t) * cut.size(), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        return NUFFT2_ERR_HIP;
    }
    a->zonal = true;
    return NUFFT2_OK;
}

NUFFT2_API nufft2_status nufft2_analysis_set_layout(nufft2_analysis a, int32_t m_major)
{
    if (!a || (m_major != 0 && m_major != 1)) return NUFFT2_ERR_ARG;
    a->m_major = m_major;
    return NUFFT2_OK;
}

NUFFT2_API nufft2_status nufft2_analysis_destroy(nufft2_analysis a)
{
    if (!a) return NUFFT2_OK;
    (void)hipStreamSynchronize(a->stream);
    analysis_free(a);
    return NUFFT2_OK;
}

// ---- Gauss-Legendre DFS analysis ----------------------------------------------

namespace {

// Roots of the degree-J Legendre polynomial (Newton from cos(pi (k + 3/4) /
// (J + 1/2)), long double), as colatitudes in increasing order.
void gl_colatitudes(int J, std::vector<long double> &theta)
{
    const long double pi = 3.141592653589793238462643383279502884L;
    theta.resize(J);
    for (int k = 0; k < J; ++k) {
        long double z = cosl(pi * ((long double)k + 0.75L) / ((long double)J + 0.5L));
        for (int it = 0; it < 100; ++it) {
            long double p0 = 1.0L, p1 = z;
            for (int n = 2; n <= J; ++n) {
                const long double p2 = ((2.0L * n - 1.0L) * z * p1 - (n - 1.0L) * p0) / (long double)n;
                p0 = p1;
                p1 = p2;
            }
            const long double dp = (long double)J * (z * p1 - p0) / (z * z - 1.0L);
            const long double dz = p1 / dp;
            z -= dz;
            if (fabsl(dz) < 1e-19L * fabsl(z) + 1e-30L) break;
        }
        theta[k] = acosl(z);  // z decreases with k: theta increases
    }
}

// Inverse of the J x J matrix M (row-major) by LU with partial pivoting
// (Gauss-Jordan on [M | I]), long double; false if singular.
bool invert_ld(int J, std::vector<long double> &M, std::vector<long double> &inv)
{
    inv.assign((size_t)J * J, 0.0L);
    for (int i = 0; i < J; ++i) inv[(size_t)i * J + i] = 1.0L;
    for (int c = 0; c < J; ++c) {
        int piv = c;
        for (int r = c + 1; r < J; ++r)
            if (fabsl(M[(size_t)r * J + c]) > fabsl(M[(size_t)piv * J + c])) piv = r;
        if (M[(size_t)piv * J + c] == 0.0L) return false;
        if (piv != c)
            for (int k = 0; k < J; ++k) {
                std::swap(M[(size_t)c * J + k], M[(size_t)piv * J + k]);
                std::swap(inv[(size_t)c * J + k], inv[(size_t)piv * J + k]);
            }
        const long double d = 1.0L / M[(size_t)c * J + c];
        for (int k = 0; k < J; ++k) {
            M[(size_t)c * J + k] *= d;
            inv[(size_t)c * J + k] *= d;
        }
        for (int r = 0; r < J; ++r) {
            if (r == c) continue;
            const long double f = M[(size_t)r * J + c];
            if (f == 0.0L) continue;
            long double *mr = &M[(size_t)r * J], *ir = &inv[(size_t)r * J];
            const long double *mc = &M[(size_t)c * J], *ic = &inv[(size_t)c * J];
            for (int k = c; k < J; ++k) mr[k] -= f * mc[k];
            for (int k = 0; k < J; ++k) ir[k] -= f * ic[k];
        }
    }
    return true;
}

}  // namespace

struct nufft2_gl_s {
    int prec = 0;
    int J = 0, F = 0;
    hipStream_t stream = nullptr;
    void *tws = nullptr, *inv = nullptr, *A = nullptr;
};

static void gl_free(nufft2_gl_s *g)
{
    if (g->tws) (void)hipFree(g->tws);
    if (g->inv) (void)hipFree(g->inv);
    if (g->A) (void)hipFree(g->A);
    delete g;
}

template <typename T> static hipError_t gl_tables(nufft2_gl_s *g)
{
    const int J = g->J;
    std::vector<long double> th;
    gl_colatitudes(J, th);
    std::vector<T> out(2 * (size_t)J * J);
    for (int p = 0; p < 2; ++p) {
        // rows: samples j; columns: basis n (cos(n theta), n < J; sin((n + 1) theta))
        std::vector<long double> M((size_t)J * J), inv;
        for (int j = 0; j < J; ++j)
            for (int n = 0; n < J; ++n)
                M[(size_t)j * J + n] = p == 0 ? cosl((long double)n * th[j]) : sinl((long double)(n + 1) * th[j]);
        if (!invert_ld(J, M, inv)) return hipErrorInvalidValue;
        for (size_t e = 0; e < inv.size(); ++e) out[(size_t)p * J * J + e] = (T)inv[e];
    }
    std::vector<T> tw;
    fill_twiddle_tables<T>(tw, 2 * J);
    hipError_t e = hipMemcpy(g->inv, out.data(), sizeof(T) * out.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(g->tws, tw.data(), sizeof(T) * tw.size(), hipMemcpyHostToDevice);
    return e;
}

NUFFT2_API nufft2_status nufft2_gl_nodes(int64_t J, double *theta)
{
    if (!theta || J < 1 || J > 4096) return NUFFT2_ERR_ARG;
    std::vector<long double> th;
    gl_colatitudes((int)J, th);
    for (int64_t j = 0; j < J; ++j) theta[j] = (double)th[j];
    return NUFFT2_OK;
}

NUFFT2_API nufft2_status nufft2_gl_plan(nufft2_prec prec, int64_t J, int32_t n_fields, void *stream, nufft2_gl *out)
{
    if (!out || (prec != NUFFT2_FP32 && prec != NUFFT2_FP64) || n_fields < 1 || J < 16 || J > 1024 ||
        !is_pow2(J))
        return NUFFT2_ERR_ARG;
    nufft2_gl_s *g = new (std::nothrow) nufft2_gl_s();
    if (!g) return NUFFT2_ERR_ALLOC;
    g->prec = prec;
    g->J = (int)J;
    g->F = n_fields;
    g->stream = (hipStream_t)stream;
    const size_t rs = prec == NUFFT2_FP32 ? sizeof(float) : sizeof(double);
    const size_t K = 2 * (size_t)J - 1;
    if (hipMalloc(&g->tws, 2 * rs * (64 + 2 * (size_t)J)) != hipSuccess ||
        hipMalloc(&g->inv, rs * 2 * (size_t)J * J) != hipSuccess ||
        hipMalloc(&g->A, 2 * rs * (size_t)n_fields * J * K) != hipSuccess) {
        (void)hipGetLastError();
        gl_free(g);
        return NUFFT2_ERR_ALLOC;
    }
    const hipError_t e = prec == NUFFT2_FP32 ? gl_tables<float>(g) : gl_tables<double>(g);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        gl_free(g);
        return NUFFT2_ERR_HIP;
    }
    *out = g;
    return NUFFT2_OK;
}

NUFFT2_API nufft2_status nufft2_gl_exec(nufft2_gl g, const void *values_dev, void *coeffs_dev)
{
    if (!g || !values_dev || !coeffs_dev) return NUFFT2_ERR_ARG;
    AnalysisParams ap{};
    ap.J = g->J;
    ap.log_len = ilog2(2 * (int64_t)g->J);
    ap.n_fields = g->F;
    ap.zonal_cut = nullptr;
    hipError_t e = launch_analysis_rows(g->prec, ap, values_dev, g->tws, g->A, g->stream);
    if (e == hipSuccess) e = launch_gl_latitude(g->prec, g->J, g->F, g->inv, g->A, coeffs_dev, g->stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return NUFFT2_ERR_HIP;
    }
    return NUFFT2_OK;
}

NUFFT2_API nufft2_status nufft2_gl_destroy(nufft2_gl g)
{
    if (!g) return NUFFT2_OK;
    (void)hipStreamSynchronize(g->stream);
    gl_free(g);
    return NUFFT2_OK;
}
