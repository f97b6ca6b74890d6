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

// The elementwise kernels (k_pr_rhs, k_pr_synth) run kPrThreads-thread
// blocks along one row of their output each.
constexpr int kPrThreads = 256;
__host__ __device__ inline int pr_row_blocks(int width) { return (width + kPrThreads - 1) / kPrThreads; }

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
__global__ __launch_bounds__(kPrThreads) void k_pr_rhs(const C2<T> *__restrict__ e, double *__restrict__ rhs, PrParams p)
{
    const int64_t W = p.M + 1, H = p.N + 1;
    // blocks of one row (f, j) each: the row and field come from one
    // block-uniform division instead of 64-bit divisions per thread
    const int nbx = pr_row_blocks((int)W);
    const int row = (int)blockIdx.x / nbx;
    const int m = ((int)blockIdx.x - row * nbx) * kPrThreads + (int)threadIdx.x;
    if (m >= W) return;
    const int f = row / (int)H;
    const int j = row - f * (int)H;
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

// The solve of L D L^T x = rhs along each chain j = parity, parity + 2, ...
// (cos and sin parts together; fac = [4 classes][3][N + 1 + kPrPad]:
// L(j, j-2), L(j, j-4), 1 / D(j), zero outside the class range, so a chain
// runs over all j of its parity and writes zeros there).  With step k for
// j = parity + 2k the sweeps are linear two-term recurrences:
//   forward   y_k = r_k - L(j, j-2) y_{k-1} - L(j, j-4) y_{k-2},  z_k = y_k / D(j),
//   backward  x_k = z_k - L(j+2, j) x_{k+1} - L(j+4, j) x_{k+2}.
// A chain of N / 2 steps run by one thread leaves the GPU almost idle (one
// wave per 64 columns, parity and field), so each sweep is split into
// segments of kPrSeg steps run side by side: a first kernel runs every
// segment from a zero state and keeps its end state; a second one chains
// the segments' end states through the segments' homogeneous propagators
// (2 x 2 products of the recurrence matrices, the same for every column of a
// class; made on the host in long double) to find the state each segment
// starts from, and runs the segment again from it, writing the results.
// By linearity this is the serial recurrence, up to rounding.
constexpr int kPrSeg = 32;

__host__ __device__ inline int pr_steps(int N, int par) { return (N - par) / 2 + 1; }
__host__ __device__ inline int pr_segments(int N) { return (pr_steps(N, 0) + kPrSeg - 1) / kPrSeg; }

// One workgroup: 64 consecutive columns of one segment, parity and field.
struct PrSegIdx {
    int m, seg, par, f, cls, k0, k1;
    bool valid;
};
__device__ inline PrSegIdx pr_seg_idx(const PrParams &p)
{
    PrSegIdx q;
    q.m = (int)blockIdx.x * 64 + (int)threadIdx.x;
    q.seg = (int)blockIdx.y;
    q.par = (int)blockIdx.z & 1;
    q.f = (int)blockIdx.z >> 1;
    q.cls = pr_class(q.m);
    const int ns = pr_steps(p.N, q.par);
    q.k0 = q.seg * kPrSeg;
    q.k1 = q.k0 + kPrSeg < ns ? q.k0 + kPrSeg : ns;
    q.valid = q.m <= p.M && q.k0 < ns;
    return q;
}

// End states: st[f][par][seg][4][M + 1] = (cos y_a, cos y_b, sin y_a, sin y_b)
__device__ inline double *pr_state(double *st, const PrParams &p, const PrSegIdx &q, int seg, int e)
{
    const int nseg = pr_segments(p.N);
    return st + ((((int64_t)q.f * 2 + q.par) * nseg + seg) * 4 + e) * (p.M + 1) + q.m;
}

// Forward, pass 1: every segment from y_{k0-1} = y_{k0-2} = 0; keeps
// (y_{k1-1}, y_{k1-2}).
__global__ __launch_bounds__(64) void k_pr_fwd_local(const double *__restrict__ rhs, const double *__restrict__ fac,
                                                     double *__restrict__ st, PrParams p)
{
    const PrSegIdx q = pr_seg_idx(p);
    if (!q.valid) return;
    const int64_t W = p.M + 1, H = p.N + 1;
    const int FL = p.N + 1 + kPrPad;
    const double *L1 = fac + (int64_t)q.cls * 3 * FL, *L2 = L1 + FL;
    const double *rc = rhs + (int64_t)q.f * 2 * H * W + q.m, *rs = rc + H * W;
    double yc1 = 0, yc2 = 0, ys1 = 0, ys2 = 0;
#pragma unroll 8
    for (int k = q.k0; k < q.k1; ++k) {
        const int j = q.par + 2 * k;
        const double a = L1[j], b = L2[j];
        const double yc = rc[(int64_t)j * W] - a * yc1 - b * yc2;
        const double ys = rs[(int64_t)j * W] - a * ys1 - b * ys2;
        yc2 = yc1;
        yc1 = yc;
        ys2 = ys1;
        ys1 = ys;
    }
    *pr_state(st, p, q, q.seg, 0) = yc1;
    *pr_state(st, p, q, q.seg, 1) = yc2;
    *pr_state(st, p, q, q.seg, 2) = ys1;
    *pr_state(st, p, q, q.seg, 3) = ys2;
}

// Forward, pass 2: the start state of the segment from the earlier ones
// (S_{t+1} = P_t S_t + E_t, S_0 = 0), then the segment again from it, z
// into rhs.  prop = [4 classes][2 parities][segments][2 x 2].
__global__ __launch_bounds__(64) void k_pr_fwd_apply(double *__restrict__ rhs, const double *__restrict__ fac,
                                                     const double *__restrict__ st, const double *__restrict__ prop,
                                                     PrParams p)
{
    const PrSegIdx q = pr_seg_idx(p);
    if (!q.valid) return;
    const int64_t W = p.M + 1, H = p.N + 1;
    const int FL = p.N + 1 + kPrPad;
    const int nseg = pr_segments(p.N);
    double yc1 = 0, yc2 = 0, ys1 = 0, ys2 = 0;
    for (int t = 0; t < q.seg; ++t) {
        const double *P = prop + (((int64_t)q.cls * 2 + q.par) * nseg + t) * 4;
        const double c1 = P[0] * yc1 + P[1] * yc2 + *pr_state(const_cast<double *>(st), p, q, t, 0);
        const double c2 = P[2] * yc1 + P[3] * yc2 + *pr_state(const_cast<double *>(st), p, q, t, 1);
        const double s1 = P[0] * ys1 + P[1] * ys2 + *pr_state(const_cast<double *>(st), p, q, t, 2);
        const double s2 = P[2] * ys1 + P[3] * ys2 + *pr_state(const_cast<double *>(st), p, q, t, 3);
        yc1 = c1;
        yc2 = c2;
        ys1 = s1;
        ys2 = s2;
    }
    const double *L1 = fac + (int64_t)q.cls * 3 * FL, *L2 = L1 + FL, *DI = L2 + FL;
    double *rc = rhs + (int64_t)q.f * 2 * H * W + q.m, *rs = rc + H * W;
#pragma unroll 8
    for (int k = q.k0; k < q.k1; ++k) {
        const int j = q.par + 2 * k;
        const double a = L1[j], b = L2[j];
        const double yc = rc[(int64_t)j * W] - a * yc1 - b * yc2;
        const double ys = rs[(int64_t)j * W] - a * ys1 - b * ys2;
        rc[(int64_t)j * W] = yc * DI[j];
        rs[(int64_t)j * W] = ys * DI[j];
        yc2 = yc1;
        yc1 = yc;
        ys2 = ys1;
        ys1 = ys;
    }
}

// Backward, pass 1: every segment from x_{k1} = x_{k1+1} = 0, downwards;
// keeps (x_{k0}, x_{k0+1}).
__global__ __launch_bounds__(64) void k_pr_bwd_local(const double *__restrict__ rhs, const double *__restrict__ fac,
                                                     double *__restrict__ st, PrParams p)
{
    const PrSegIdx q = pr_seg_idx(p);
    if (!q.valid) return;
    const int64_t W = p.M + 1, H = p.N + 1;
    const int FL = p.N + 1 + kPrPad;
    const double *L1 = fac + (int64_t)q.cls * 3 * FL, *L2 = L1 + FL;
    const double *rc = rhs + (int64_t)q.f * 2 * H * W + q.m, *rs = rc + H * W;
    double xc1 = 0, xc2 = 0, xs1 = 0, xs2 = 0;
#pragma unroll 8
    for (int k = q.k1 - 1; k >= q.k0; --k) {
        const int j = q.par + 2 * k;
        const double c = L1[j + 2], d = L2[j + 4];
        const double xc = rc[(int64_t)j * W] - c * xc1 - d * xc2;
        const double xs = rs[(int64_t)j * W] - c * xs1 - d * xs2;
        xc2 = xc1;
        xc1 = xc;
        xs2 = xs1;
        xs1 = xs;
    }
    *pr_state(st, p, q, q.seg, 0) = xc1;
    *pr_state(st, p, q, q.seg, 1) = xc2;
    *pr_state(st, p, q, q.seg, 2) = xs1;
    *pr_state(st, p, q, q.seg, 3) = xs2;
}

// Backward, pass 2: the state above the segment from the later segments
// (T_{t-1} = Q_t T_t + F_t from the last one down, T_last = 0), then the
// segment again from it, x into out (the sin part of column 0 is zero).
template <typename T>
__global__ __launch_bounds__(64) void k_pr_bwd_apply(const double *__restrict__ rhs, const double *__restrict__ fac,
                                                     const double *__restrict__ st, const double *__restrict__ prop,
                                                     T *__restrict__ out, PrParams p)
{
    const PrSegIdx q = pr_seg_idx(p);
    if (!q.valid) return;
    const int64_t W = p.M + 1, H = p.N + 1;
    const int FL = p.N + 1 + kPrPad;
    const int nseg = pr_segments(p.N);
    const int last = (pr_steps(p.N, q.par) - 1) / kPrSeg;
    double xc1 = 0, xc2 = 0, xs1 = 0, xs2 = 0;
    for (int t = last; t > q.seg; --t) {
        const double *Q = prop + (((int64_t)q.cls * 2 + q.par) * nseg + t) * 4;
        const double c1 = Q[0] * xc1 + Q[1] * xc2 + *pr_state(const_cast<double *>(st), p, q, t, 0);
        const double c2 = Q[2] * xc1 + Q[3] * xc2 + *pr_state(const_cast<double *>(st), p, q, t, 1);
        const double s1 = Q[0] * xs1 + Q[1] * xs2 + *pr_state(const_cast<double *>(st), p, q, t, 2);
        const double s2 = Q[2] * xs1 + Q[3] * xs2 + *pr_state(const_cast<double *>(st), p, q, t, 3);
        xc1 = c1;
        xc2 = c2;
        xs1 = s1;
        xs2 = s2;
    }
    const double *L1 = fac + (int64_t)q.cls * 3 * FL, *L2 = L1 + FL;
    const double *rc = rhs + (int64_t)q.f * 2 * H * W + q.m, *rs = rc + H * W;
    T *oc = out + (int64_t)q.f * 2 * H * W + q.m, *os = oc + H * W;
#pragma unroll 8
    for (int k = q.k1 - 1; k >= q.k0; --k) {
        const int j = q.par + 2 * k;
        const double c = L1[j + 2], d = L2[j + 4];
        const double xc = rc[(int64_t)j * W] - c * xc1 - d * xc2;
        const double xs = rs[(int64_t)j * W] - c * xs1 - d * xs2;
        oc[(int64_t)j * W] = (T)xc;
        os[(int64_t)j * W] = (T)(q.m == 0 ? 0.0 : xs);
        xc2 = xc1;
        xc1 = xc;
        xs2 = xs1;
        xs1 = xs;
    }
}

// Homogeneous propagators of the segments (long double products of the
// double factors the kernels use): fwd[cls][par][seg] maps (y_{k0-1},
// y_{k0-2}) to (y_{k1-1}, y_{k1-2}); bwd[cls][par][seg] maps (x_{k1},
// x_{k1+1}) to (x_{k0}, x_{k0+1}).  fac as above (host copy).
void pr_propagators(int N, const std::vector<double> &fac, std::vector<double> &fwd, std::vector<double> &bwd)
{
    const int FL = N + 1 + kPrPad, nseg = pr_segments(N);
    fwd.assign((size_t)4 * 2 * nseg * 4, 0.0);
    bwd.assign((size_t)4 * 2 * nseg * 4, 0.0);
    for (int cls = 0; cls < 4; ++cls) {
        const double *L1 = fac.data() + (size_t)cls * 3 * FL, *L2 = L1 + FL;
        for (int par = 0; par < 2; ++par) {
            const int ns = pr_steps(N, par);
            for (int s = 0; s < nseg; ++s) {
                const int k0 = s * kPrSeg, k1 = k0 + kPrSeg < ns ? k0 + kPrSeg : ns;
                long double P[4] = {1, 0, 0, 1}, Q[4] = {1, 0, 0, 1};
                for (int k = k0; k < k1; ++k) {  // P = M_k P
                    const int j = par + 2 * k;
                    const long double a = L1[j], b = L2[j];
                    const long double r0 = -a * P[0] - b * P[2], r1 = -a * P[1] - b * P[3];
                    P[2] = P[0];
                    P[3] = P[1];
                    P[0] = r0;
                    P[1] = r1;
                }
                for (int k = k1 - 1; k >= k0; --k) {  // Q = M'_k Q
                    const int j = par + 2 * k;
                    const long double c = L1[j + 2], d = L2[j + 4];
                    const long double r0 = -c * Q[0] - d * Q[2], r1 = -c * Q[1] - d * Q[3];
                    Q[2] = Q[0];
                    Q[3] = Q[1];
                    Q[0] = r0;
                    Q[1] = r1;
                }
                double *pf = fwd.data() + (((size_t)cls * 2 + par) * nseg + s) * 4;
                double *pb = bwd.data() + (((size_t)cls * 2 + par) * nseg + s) * 4;
                for (int e = 0; e < 4; ++e) {
                    pf[e] = (double)P[e];
                    pb[e] = (double)Q[e];
                }
            }
        }
    }
}

// Standard coefficients (cos and sin parts) at (n, m) of a pr column (the
// conversion after eq. std_dfs), from cc[k * stride], cs[k * stride], k in
// the class range F(k):
//   class 0: F(n)
//   class 1: F(n-1)/2 - F(n+1)/2 (+ F(0)/2 at n = 1; 0 at n = 0)
//   class 2: F(n+1)/2 - F(n-1)/2
//   class 3: F(n)/2 - F(n-2)/4 - F(n+2)/4 (+ F(1)/4 at n = 1; 0 at n = 0)
// written as one weighted sum of the five entries n - 2 .. n + 2 whose
// weights the class selects: neighbouring lanes hold columns of alternating
// classes (even and odd m), and a branch per class would make every wave
// run both.  Entries of weight zero are not read.
template <typename T>
__device__ inline void pr_to_std_pair(const T *__restrict__ cc, const T *__restrict__ cs, int64_t stride, int cls,
                                      int n, int N, double &c, double &s)
{
    int lo, hi;
    pr_range(cls, N, lo, hi);
    // weights of F(n - 2) .. F(n + 2) (the n = 1 cases fold F(0) resp. F(1) in)
    double w[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (cls == 0) {
        w[2] = 1.0;
    } else if (cls == 1) {
        if (n > 0) {
            w[1] = n == 1 ? 1.0 : 0.5;
            w[3] = -0.5;
        }
    } else if (cls == 2) {
        w[1] = -0.5;
        w[3] = 0.5;
    } else if (n > 0) {
        w[0] = -0.25;
        w[2] = n == 1 ? 0.75 : 0.5;
        w[4] = -0.25;
    }
    c = 0.0;
    s = 0.0;
#pragma unroll
    for (int d = 0; d < 5; ++d) {
        const int k = n - 2 + d;
        if (w[d] != 0.0 && k >= lo && k <= hi) {
            c += w[d] * (double)cc[(int64_t)k * stride];
            s += w[d] * (double)cs[(int64_t)k * stride];
        }
    }
}

// Exp-form entry (n, m) of the pr expansion: standard coefficients of column
// |m| at |n|, then the map of eq. dfs_fourier_coeffs.
template <typename T>
__global__ __launch_bounds__(kPrThreads) void k_pr_synth(const T *__restrict__ pr, C2<T> *__restrict__ e, PrParams p)
{
    const int64_t Wd = 2 * p.M + 1, Hd = 2 * p.N + 1;
    // one row (f, a) per group of blocks, as in k_pr_rhs
    const int nbx = pr_row_blocks((int)Wd);
    const int row = (int)blockIdx.x / nbx;
    const int b = ((int)blockIdx.x - row * nbx) * kPrThreads + (int)threadIdx.x;
    if (b >= Wd) return;
    const int f = row / (int)Hd;
    const int a = row - f * (int)Hd;
    const int64_t t = (int64_t)row * Wd + b;
    const int n = a - p.N, m = b - p.M;
    const int an = n < 0 ? -n : n, am = m < 0 ? -m : m;
    const int64_t W = p.M + 1, H = p.N + 1;
    const T *pc = pr + (int64_t)f * 2 * H * W + am;
    const T *ps = pc + H * W;
    const int cls = pr_class(am);
    double c, s;
    pr_to_std_pair(pc, ps, W, cls, an, p.N, c, s);
    if (am == 0) s = 0.0;
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
    const int64_t blocks = (int64_t)p.F * (p.N + 1) * pr_row_blocks(p.M + 1);
    if (blocks > INT32_MAX) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_pr_rhs<T>, dim3((unsigned)blocks), dim3(kPrThreads), 0, s, (const C2<T> *)e, rhs, p);
    return hipGetLastError();
}

template <typename T> hipError_t launch_solve(double *rhs, const double *fac, double *st, const double *fwd,
                                              const double *bwd, void *out, const PrParams &p, hipStream_t s)
{
    const dim3 grid((unsigned)((p.M + 1 + 63) / 64), (unsigned)pr_segments(p.N), (unsigned)(2 * p.F));
    hipLaunchKernelGGL(k_pr_fwd_local, grid, dim3(64), 0, s, (const double *)rhs, fac, st, p);
    hipLaunchKernelGGL(k_pr_fwd_apply, grid, dim3(64), 0, s, rhs, fac, (const double *)st, fwd, p);
    hipLaunchKernelGGL(k_pr_bwd_local, grid, dim3(64), 0, s, (const double *)rhs, fac, st, p);
    hipLaunchKernelGGL(k_pr_bwd_apply<T>, grid, dim3(64), 0, s, (const double *)rhs, fac, (const double *)st, bwd,
                       (T *)out, p);
    return hipGetLastError();
}

template <typename T> hipError_t launch_synth(const void *pr, void *e, const PrParams &p, hipStream_t s)
{
    const int64_t blocks = (int64_t)p.F * (2 * p.N + 1) * pr_row_blocks(2 * p.M + 1);
    if (blocks > INT32_MAX) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_pr_synth<T>, dim3((unsigned)blocks), dim3(kPrThreads), 0, s, (const T *)pr, (C2<T> *)e,
                       p);
    return hipGetLastError();
}

// G = A^T W A of one class restricted to its range, factored along each
// parity chain as L D L^T (long double); tables as the solve kernels read them.
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
    double *prop = nullptr; // segment propagators: forward then backward, [4][2][segments][4] each
    double *st = nullptr;   // segment end states [F][2][segments][4][M + 1]
};

static void pr_free(nufft2_pr_s *h)
{
    if (h->fac) (void)hipFree(h->fac);
    if (h->rhs) (void)hipFree(h->rhs);
    if (h->prop) (void)hipFree(h->prop);
    if (h->st) (void)hipFree(h->st);
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
    std::vector<double> fwd, bwd;
    pr_propagators(h->N, fac, fwd, bwd);
    const size_t nprop = fwd.size();
    const size_t nst = (size_t)n_fields * 2 * pr_segments(h->N) * 4 * (M + 1);
    if (hipMalloc(&h->fac, sizeof(double) * fac.size()) != hipSuccess ||
        hipMalloc(&h->rhs, sizeof(double) * 2 * (size_t)n_fields * (N + 1) * (M + 1)) != hipSuccess ||
        hipMalloc(&h->prop, sizeof(double) * 2 * nprop) != hipSuccess ||
        hipMalloc(&h->st, sizeof(double) * nst) != hipSuccess) {
        (void)hipGetLastError();
        pr_free(h);
        return NUFFT2_ERR_ALLOC;
    }
    if (hipMemcpy(h->fac, fac.data(), sizeof(double) * fac.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->prop, fwd.data(), sizeof(double) * nprop, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->prop + nprop, bwd.data(), sizeof(double) * nprop, hipMemcpyHostToDevice) != hipSuccess) {
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
    if (e == hipSuccess) {
        const double *fwd = h->prop, *bwd = h->prop + (size_t)4 * 2 * pr_segments(h->N) * 4;
        e = h->prec == NUFFT2_FP32 ? launch_solve<float>(h->rhs, h->fac, h->st, fwd, bwd, pr_dev, p, h->stream)
                                   : launch_solve<double>(h->rhs, h->fac, h->st, fwd, bwd, pr_dev, p, h->stream);
    }
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
