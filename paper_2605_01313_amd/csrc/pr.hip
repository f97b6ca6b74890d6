// Partial-regularity DFS expansion (section 4, eq. pr_dfs): least-squares
// projection of exp-form coefficients onto the partial-regularity basis, and
// the conversion back to exp form.
//
// Column m of the basis multiplies cos(m phi) and sin(m phi) by
//   class 0 (m = 0):       cos(n theta)                n = 0 .. N
//   class 1 (m = 1):       sin(theta) cos(n theta)     n = 0 .. N-1
//   class 2 (even m >= 2): sin(theta) sin(n theta)     n = 1 .. N-1
//   class 3 (odd m >= 3):  sin^2(theta) sin(n theta)   n = 1 .. N-2
// By the product-to-sum identities each basis function is a combination of
// at most three standard factors (cos(n theta) for even m, sin(n theta) for
// odd m), which is the conversion printed after eq. std_dfs (for even m the
// constant term of sin(theta) sin(theta) is 1/2, so the standard n = 0
// coefficient is f_{1,m} / 2).
//
// The projection solves, per column, the normal equations G x = A^T W b of
// the section 4 orthogonality conditions (A: basis -> standard factors, W:
// the integrals of the squared standard factors).  Basis function j couples
// only with j - 4 .. j + 4 in steps of 2, so each column splits into two
// independent chains (even and odd j) with a tridiagonal (classes 1, 2) or
// pentadiagonal (class 3) matrix.  The host factors the four class matrices
// once per plan (G = L D L^T, long double); a thread then runs one chain of
// one column for both the cos and sin parts: a forward and a backward sweep.
// Everything is computed in FP64 whatever the plan precision: the odd-m
// matrices have condition numbers up to ~5e9 at N = 1023.
#include <math.h>
#include <stdint.h>

#include <new>
#include <vector>

#include "nufft2.h"
#include "nufft2_internal.hpp"

#define NUFFT2_API extern "C" __attribute__((visibility("default")))

namespace nufft2 {
namespace {

constexpr int kPrPad = 5;  // zero entries past j = N in the factor tables

__host__ __device__ inline int pr_class(int m) { return m == 0 ? 0 : (m == 1 ? 1 : 2 + (m & 1)); }

// Standard-factor weights divided by pi/2: 2 for the constant cosine, 0 for
// sin(0 theta), 1 otherwise.
__host__ __device__ inline double std_weight(int cls, int i)
{
    if (i > 0) return 1.0;
    return (cls == 0 || cls == 2) ? 2.0 : 0.0;
}

// Entries of column j of A (standard coefficients of basis function j of a
// class): up to three (row, value) pairs; returns their number.  Rows past
// N are dropped by the caller.
__host__ __device__ inline int basis_terms(int cls, int j, int *row, double *val)
{
    switch (cls) {
    case 0: row[0] = j; val[0] = 1.0; return 1;
    case 1:  // sin th cos j th = (sin (j+1) th - sin (j-1) th) / 2
        row[0] = j + 1; val[0] = j == 0 ? 1.0 : 0.5;
        if (j >= 2) { row[1] = j - 1; val[1] = -0.5; return 2; }
        return 1;
    case 2:  // sin th sin j th = (cos (j-1) th - cos (j+1) th) / 2
        row[0] = j - 1; val[0] = 0.5;
        row[1] = j + 1; val[1] = -0.5;
        return 2;
    default:  // sin^2 th sin j th = sin j th / 2 - (sin (j+2) th + sin (j-2) th) / 4
        row[0] = j; val[0] = j == 1 ? 0.75 : 0.5;
        row[1] = j + 2; val[1] = -0.25;
        if (j >= 3) { row[2] = j - 2; val[2] = -0.25; return 3; }
        return 2;
    }
}

__host__ __device__ inline void pr_range(int cls, int N, int &lo, int &hi)
{
    lo = (cls == 0 || cls == 1) ? 0 : 1;
    hi = cls == 0 ? N : (cls == 3 ? N - 2 : N - 1);
}

struct PrParams {
    int N, M, F;
};

template <typename T> struct C2 { T x, y; };

// Standard coefficients (c, s) at (n, m), n, m >= 0, read from exp-form
// entries e(+-n, +-m) as the least-squares inverse of eq. dfs_fourier_coeffs.
template <typename T>
__device__ inline void exp_to_std(const C2<T> *__restrict__ e, const PrParams &p, int n, int m, double &c,
                                  double &s)
{
    const int W = 2 * p.M + 1;
    auto at = [&](int nn, int mm) {
        const C2<T> v = e[(int64_t)(nn + p.N) * W + (mm + p.M)];
        return C2<double>{(double)v.x, (double)v.y};
    };
    if (m == 0) {
        const C2<double> a = at(n, 0);
        c = n == 0 ? a.x : a.x + at(-n, 0).x;
        s = 0.0;
    } else if ((m & 1) == 0) {
        if (n == 0) {
            const C2<double> a = at(0, m), b = at(0, -m);
            c = a.x + b.x;
            s = b.y - a.y;
        } else {
            const C2<double> a = at(n, m), b = at(-n, m), d = at(n, -m), g = at(-n, -m);
            c = a.x + b.x + d.x + g.x;
            s = d.y + g.y - a.y - b.y;
        }
    } else {
        if (n == 0) {
            c = s = 0.0;
        } else {
            const C2<double> a = at(n, m), b = at(-n, m), d = at(n, -m), g = at(-n, -m);
            c = -(a.y - b.y + d.y - g.y);
            s = d.x - g.x - a.x + b.x;
        }
    }
}

// rhs[f][cs][j][m] = sum_i A[i][j] w_i b_i (zero outside the column's range).
template <typename T>
__global__ __launch_bounds__(256) void k_pr_rhs(const C2<T> *__restrict__ e, double *__restrict__ rhs, PrParams p)
{
    const int64_t W = p.M + 1, H = p.N + 1;
    const int64_t total = (int64_t)p.F * H * W;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int m = (int)(t % W);
    const int j = (int)((t / W) % H);
    const int f = (int)(t / (W * H));
    const int cls = pr_class(m);
    int lo, hi;
    pr_range(cls, p.N, lo, hi);
    double rc = 0.0, rs = 0.0;
    if (j >= lo && j <= hi) {
        const C2<T> *ef = e + (int64_t)f * (2 * p.N + 1) * (2 * p.M + 1);
        int row[3];
        double val[3];
        const int nt = basis_terms(cls, j, row, val);
        for (int q = 0; q < nt; ++q) {
            if (row[q] > p.N) continue;
            double c, s;
            exp_to_std(ef, p, row[q], m, c, s);
            const double a = val[q] * std_weight(cls, row[q]);
            rc += a * c;
            rs += a * s;
        }
    }
    double *r = rhs + (int64_t)f * 2 * H * W;
    r[(int64_t)j * W + m] = rc;
    r[H * W + (int64_t)j * W + m] = rs;
}

// One thread per (field, chain parity, column m): forward and backward
// sweeps of L D L^T x = rhs along j = parity, parity + 2, ... for the cos and
// sin parts.  fac = [4 classes][3][N + 1 + kPrPad]: L(j, j-2), L(j, j-4),
// 1 / D(j), zero outside the class range (so the chain runs over all j of
// its parity and writes zeros there).  z is kept in rhs between the sweeps.
// The loads do not depend on the recurrence, so each sweep reads a group of
// kPrUnroll steps ahead of the group it computes.
constexpr int kPrUnroll = 8;

template <typename T>
__global__ __launch_bounds__(64) void k_pr_solve(double *__restrict__ rhs, const double *__restrict__ fac,
                                                 T *__restrict__ out, PrParams p)
{
    const int64_t W = p.M + 1, H = p.N + 1;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= p.F * 2 * (int)W) return;
    const int m = t % (int)W;
    const int par = (t / (int)W) & 1;
    const int f = t / (2 * (int)W);
    const int cls = pr_class(m);
    const int FL = p.N + 1 + kPrPad;
    const double *L1 = fac + (int64_t)cls * 3 * FL;
    const double *L2 = L1 + FL;
    const double *DI = L2 + FL;
    double *rc = rhs + (int64_t)f * 2 * H * W + m;
    double *rs = rc + H * W;
    const int nsteps = (p.N - par) / 2 + 1;  // j = par + 2 k, k < nsteps
    constexpr int U = kPrUnroll;

    // forward: y_j = r_j - L(j, j-2) y_{j-2} - L(j, j-4) y_{j-4};  z_j = y_j / D(j)
    double yc1 = 0, yc2 = 0, ys1 = 0, ys2 = 0;
    double ac[U], as[U], a1[U], a2[U], ad[U];
    auto load_fwd = [&](int k0) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + u < nsteps ? k0 + u : nsteps - 1;
            const int j = par + 2 * k;
            ac[u] = rc[(int64_t)j * W];
            as[u] = rs[(int64_t)j * W];
            a1[u] = L1[j];
            a2[u] = L2[j];
            ad[u] = DI[j];
        }
    };
    load_fwd(0);
    for (int k0 = 0; k0 < nsteps; k0 += U) {
        double bc[U], bs[U], b1[U], b2[U], bd[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            bc[u] = ac[u];
            bs[u] = as[u];
            b1[u] = a1[u];
            b2[u] = a2[u];
            bd[u] = ad[u];
        }
        if (k0 + U < nsteps) load_fwd(k0 + U);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (k0 + u < nsteps) {
                const int j = par + 2 * (k0 + u);
                const double yc = bc[u] - b1[u] * yc1 - b2[u] * yc2;
                const double ys = bs[u] - b1[u] * ys1 - b2[u] * ys2;
                rc[(int64_t)j * W] = yc * bd[u];
                rs[(int64_t)j * W] = ys * bd[u];
                yc2 = yc1;
                yc1 = yc;
                ys2 = ys1;
                ys1 = ys;
            }
        }
    }
    // the forward stores and the backward loads are the same thread's
    // addresses, so program order makes them visible

    // backward: x_j = z_j - L(j+2, j) x_{j+2} - L(j+4, j) x_{j+4}
    T *oc = out + (int64_t)f * 2 * H * W + m;
    T *os = oc + H * W;
    double xc1 = 0, xc2 = 0, xs1 = 0, xs2 = 0;
    auto load_bwd = [&](int k0) {  // steps k0, k0 - 1, ...
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 - u >= 0 ? k0 - u : 0;
            const int j = par + 2 * k;
            ac[u] = rc[(int64_t)j * W];
            as[u] = rs[(int64_t)j * W];
            a1[u] = L1[j + 2];
            a2[u] = L2[j + 4];
        }
    };
    load_bwd(nsteps - 1);
    for (int k0 = nsteps - 1; k0 >= 0; k0 -= U) {
        double bc[U], bs[U], b1[U], b2[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            bc[u] = ac[u];
            bs[u] = as[u];
            b1[u] = a1[u];
            b2[u] = a2[u];
        }
        if (k0 - U >= 0) load_bwd(k0 - U);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (k0 - u >= 0) {
                const int j = par + 2 * (k0 - u);
                const double xc = bc[u] - b1[u] * xc1 - b2[u] * xc2;
                const double xs = bs[u] - b1[u] * xs1 - b2[u] * xs2;
                oc[(int64_t)j * W] = (T)xc;
                os[(int64_t)j * W] = (T)(m == 0 ? 0.0 : xs);
                xc2 = xc1;
                xc1 = xc;
                xs2 = xs1;
                xs1 = xs;
            }
        }
    }
}

// Standard coefficient at (n, m) of a pr column (the conversion after
// eq. std_dfs), from col[k * stride], k in the class range.
template <typename T>
__device__ inline double pr_to_std_entry(const T *__restrict__ col, int64_t stride, int cls, int n, int N)
{
    int lo, hi;
    pr_range(cls, N, lo, hi);
    auto F = [&](int k) { return (k >= lo && k <= hi) ? (double)col[(int64_t)k * stride] : 0.0; };
    switch (cls) {
    case 0: return F(n);
    case 1: return n == 0 ? 0.0 : 0.5 * F(n - 1) - 0.5 * F(n + 1) + (n == 1 ? 0.5 * F(0) : 0.0);
    case 2: return 0.5 * F(n + 1) - 0.5 * F(n - 1);
    default: return n == 0 ? 0.0 : 0.5 * F(n) - 0.25 * F(n - 2) - 0.25 * F(n + 2) + (n == 1 ? 0.25 * F(1) : 0.0);
    }
}

// Exp-form entry (n, m) of the pr expansion: standard coefficients of column
// |m| at |n|, then the map of eq. dfs_fourier_coeffs.
template <typename T>
__global__ __launch_bounds__(256) void k_pr_synth(const T *__restrict__ pr, C2<T> *__restrict__ e, PrParams p)
{
    const int64_t Wd = 2 * p.M + 1, Hd = 2 * p.N + 1;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)p.F * Hd * Wd) return;
    const int b = (int)(t % Wd);
    const int a = (int)((t / Wd) % Hd);
    const int f = (int)(t / (Wd * Hd));
    const int n = a - p.N, m = b - p.M;
    const int an = n < 0 ? -n : n, am = m < 0 ? -m : m;
    const int64_t W = p.M + 1, H = p.N + 1;
    const T *pc = pr + (int64_t)f * 2 * H * W + am;
    const T *ps = pc + H * W;
    const int cls = pr_class(am);
    const double c = pr_to_std_entry(pc, W, cls, an, p.N);
    const double s = am == 0 ? 0.0 : pr_to_std_entry(ps, W, cls, an, p.N);
    double re, im;
    if (am == 0) {
        re = n == 0 ? c : 0.5 * c;
        im = 0.0;
    } else if ((am & 1) == 0) {
        const double k = n == 0 ? 0.5 : 0.25;
        re = k * c;
        im = m > 0 ? -k * s : k * s;
    } else if (n == 0) {
        re = im = 0.0;
    } else {
        // (+n, +m): -(i c + s)/4; (-n, +m): +(i c + s)/4;
        // (+n, -m): -(i c - s)/4; (-n, -m): +(i c - s)/4
        const double sg = n > 0 ? -0.25 : 0.25;
        re = m > 0 ? sg * s : -sg * s;
        im = sg * c;
    }
    e[t] = C2<T>{(T)re, (T)im};
}

template <typename T> hipError_t launch_rhs(const void *e, double *rhs, const PrParams &p, hipStream_t s)
{
    const int64_t total = (int64_t)p.F * (p.N + 1) * (p.M + 1);
    hipLaunchKernelGGL(k_pr_rhs<T>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, (const C2<T> *)e, rhs,
                       p);
    return hipGetLastError();
}

template <typename T> hipError_t launch_solve(double *rhs, const double *fac, void *out, const PrParams &p,
                                              hipStream_t s)
{
    const int threads = p.F * 2 * (p.M + 1);
    hipLaunchKernelGGL(k_pr_solve<T>, dim3((threads + 63) / 64), dim3(64), 0, s, rhs, fac, (T *)out, p);
    return hipGetLastError();
}

template <typename T> hipError_t launch_synth(const void *pr, void *e, const PrParams &p, hipStream_t s)
{
    const int64_t total = (int64_t)p.F * (2 * p.N + 1) * (2 * p.M + 1);
    hipLaunchKernelGGL(k_pr_synth<T>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, (const T *)pr,
                       (C2<T> *)e, p);
    return hipGetLastError();
}

// G = A^T W A of one class restricted to its range, factored along each
// parity chain as L D L^T (long double); tables as k_pr_solve reads them.
void factor_class(int cls, int N, double *L1, double *L2, double *DI)
{
    const int FL = N + 1 + kPrPad;
    for (int j = 0; j < FL; ++j) L1[j] = L2[j] = DI[j] = 0.0;
    int lo, hi;
    pr_range(cls, N, lo, hi);
    // columns of A as dense vectors over rows 0..N
    auto gram = [&](int j, int k) -> long double {
        if (j < lo || j > hi || k < lo || k > hi) return 0.0L;
        int rj[3], rk[3];
        double vj[3], vk[3];
        const int nj = basis_terms(cls, j, rj, vj), nk = basis_terms(cls, k, rk, vk);
        long double g = 0.0L;
        for (int a = 0; a < nj; ++a)
            for (int b = 0; b < nk; ++b)
                if (rj[a] == rk[b] && rj[a] <= N) g += (long double)vj[a] * vk[b] * std_weight(cls, rj[a]);
        return g;
    };
    std::vector<long double> D(N + 1, 0.0L), l1(N + 1, 0.0L), l2(N + 1, 0.0L);
    for (int j = lo; j <= hi; ++j) {
        long double a2 = 0.0L, a1 = 0.0L;
        if (j - 4 >= lo) a2 = gram(j, j - 4) / D[j - 4];
        if (j - 2 >= lo) {
            long double g = gram(j, j - 2);
            if (j - 4 >= lo) g -= a2 * D[j - 4] * l1[j - 2];
            a1 = g / D[j - 2];
        }
        long double d = gram(j, j);
        if (j - 2 >= lo) d -= a1 * a1 * D[j - 2];
        if (j - 4 >= lo) d -= a2 * a2 * D[j - 4];
        D[j] = d;
        l1[j] = a1;
        l2[j] = a2;
        L1[j] = (double)a1;
        L2[j] = (double)a2;
        DI[j] = (double)(1.0L / d);
    }
}

}  // namespace
}  // namespace nufft2

using namespace nufft2;

struct nufft2_pr_s {
    int prec = 0;
    int N = 0, M = 0, F = 0;
    hipStream_t stream = nullptr;
    double *fac = nullptr;  // [4][3][N + 1 + kPrPad]
    double *rhs = nullptr;  // [F][2][N + 1][M + 1]
};

static void pr_free(nufft2_pr_s *h)
{
    if (h->fac) (void)hipFree(h->fac);
    if (h->rhs) (void)hipFree(h->rhs);
    delete h;
}

NUFFT2_API nufft2_status nufft2_pr_plan(nufft2_prec prec, int64_t N, int64_t M, int32_t n_fields, void *stream,
                                        nufft2_pr *out)
{
    if (!out || (prec != NUFFT2_FP32 && prec != NUFFT2_FP64) || n_fields < 1 || n_fields > 64 || N < 5 ||
        N > 2047 || M < 5 || M > 2047)
        return NUFFT2_ERR_ARG;
    nufft2_pr_s *h = new (std::nothrow) nufft2_pr_s();
    if (!h) return NUFFT2_ERR_ALLOC;
    h->prec = prec;
    h->N = (int)N;
    h->M = (int)M;
    h->F = n_fields;
    h->stream = (hipStream_t)stream;
    const int FL = h->N + 1 + kPrPad;
    std::vector<double> fac(4 * 3 * (size_t)FL);
    for (int c = 0; c < 4; ++c) {
        double *b = fac.data() + (size_t)c * 3 * FL;
        factor_class(c, h->N, b, b + FL, b + 2 * FL);
    }
    if (hipMalloc(&h->fac, sizeof(double) * fac.size()) != hipSuccess ||
        hipMalloc(&h->rhs, sizeof(double) * 2 * (size_t)n_fields * (N + 1) * (M + 1)) != hipSuccess) {
        (void)hipGetLastError();
        pr_free(h);
        return NUFFT2_ERR_ALLOC;
    }
    if (hipMemcpy(h->fac, fac.data(), sizeof(double) * fac.size(), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        pr_free(h);
        return NUFFT2_ERR_HIP;
    }
    *out = h;
    return NUFFT2_OK;
}

NUFFT2_API nufft2_status nufft2_pr_project(nufft2_pr h, const void *coeffs_dev, void *pr_dev)
{
    if (!h || !coeffs_dev || !pr_dev) return NUFFT2_ERR_ARG;
    const PrParams p{h->N, h->M, h->F};
    hipError_t e = h->prec == NUFFT2_FP32 ? launch_rhs<float>(coeffs_dev, h->rhs, p, h->stream)
                                          : launch_rhs<double>(coeffs_dev, h->rhs, p, h->stream);
    if (e == hipSuccess)
        e = h->prec == NUFFT2_FP32 ? launch_solve<float>(h->rhs, h->fac, pr_dev, p, h->stream)
                                   : launch_solve<double>(h->rhs, h->fac, pr_dev, p, h->stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return NUFFT2_ERR_HIP;
    }
    return NUFFT2_OK;
}

NUFFT2_API nufft2_status nufft2_pr_synthesize(nufft2_pr h, const void *pr_dev, void *coeffs_dev)
{
    if (!h || !coeffs_dev || !pr_dev) return NUFFT2_ERR_ARG;
    const PrParams p{h->N, h->M, h->F};
    const hipError_t e = h->prec == NUFFT2_FP32 ? launch_synth<float>(pr_dev, coeffs_dev, p, h->stream)
                                                : launch_synth<double>(pr_dev, coeffs_dev, p, h->stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return NUFFT2_ERR_HIP;
    }
    return NUFFT2_OK;
}

NUFFT2_API nufft2_status nufft2_pr_destroy(nufft2_pr h)
{
    if (!h) return NUFFT2_OK;
    (void)hipStreamSynchronize(h->stream);
    pr_free(h);
    return NUFFT2_OK;
}
