// Latitude step of the Gauss-Legendre DFS analysis (section 5, the
// interpolation for the SHT model).  After the FFT in longitude, each phi
// mode m holds samples g_m(theta_j) at the J Gauss-Legendre colatitudes; the
// paper inverts the latitude "DFT" matrix with a precomputed LU
// factorisation.  In the standard DFS parity (cos(n theta), n = 0..J-1, for
// even m; sin(n theta), n = 1..J, for odd m) that matrix is two real J x J
// matrices, one per parity, shared by every m of that parity and every
// field.  The host forms their inverses from the LU factors once per plan;
// here the inverse of each parity multiplies all columns of that parity at
// once, which is a dense real product J x J times J x (2 x #m x F): the one
// dense contraction of the method, done on the matrix cores (MFMA 16x16x4
// in the plan precision) with LDS-staged tiles.  The epilogue writes the exp
// form of eq. std_dfs_exp directly: a cosine coefficient a_n goes to
// n = +-n as a_n / 2 (a_0 to n = 0), a sine coefficient b_n as -+ i b_n / 2.
#include <stdint.h>

#include "nufft2_internal.hpp"

namespace nufft2 {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// MFMA 16x16x4 in each precision.  Operands: lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16].  Result row held by lane l in slot r (column
// l % 16), measured on gfx950: 4 (l / 16) + r for f32, (l / 16) + 4 r for f64.
template <typename T> struct Acc;
template <> struct Acc<float> {
    using V = f32x4;
    static __device__ inline V mfma(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    static __device__ inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <> struct Acc<double> {
    using V = f64x4;
    static __device__ inline V mfma(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    static __device__ inline int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

constexpr int kTileM = 64;   // coefficient rows per workgroup
constexpr int kTileN = 128;  // real columns per workgroup (64 modes x re/im)
constexpr int kTileK = 16;   // samples per LDS stage
constexpr int kThreads = 256;
constexpr int kALoads = kTileM * kTileK / kThreads;  // staged A elements per thread
constexpr int kBLoads = kTileK * kTileN / kThreads;  // staged B elements per thread

// One workgroup (4 waves) computes a 64 x 128 tile of C = inv[p] * B_p for
// field f and parity p, where B_p[j][2t + q] is part q (re, im) of the
// phi-step sample A[f][j][c], c = 2t + 1 - p the t-th column of parity p
// (c = m + J - 1 and J is even, so even m sit in odd c).  Wave w owns rows
// 32 (w / 2) .. + 31 and columns 64 (w % 2) .. + 63 as 2 x 4 MFMA blocks, so
// each k-step reads 2 + 4 operands from LDS for 8 MFMAs.  The next K-tile's
// values are loaded into registers while the current one is multiplied.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_gl_latitude(const T *__restrict__ inv, const T *__restrict__ A,
                                                          T *__restrict__ out, int J, int tiles_m, int tiles_n0,
                                                          int tiles_n1)
{
    __shared__ T As[kTileM][kTileK + 1];
    __shared__ T Bs[kTileK][kTileN + 2];
    const int K = 2 * J - 1;
    // workgroup -> (field, parity, row tile, column tile)
    const int per_f = tiles_m * (tiles_n0 + tiles_n1);
    int b = blockIdx.x;
    const int f = b / per_f;
    b -= f * per_f;
    const int p = b < tiles_m * tiles_n0 ? 0 : 1;
    if (p) b -= tiles_m * tiles_n0;
    const int tn = p ? tiles_n1 : tiles_n0;
    const int tm_i = b / tn, tn_i = b - (b / tn) * tn;
    const int i0 = tm_i * kTileM, col0 = tn_i * kTileN;
    const int ncols = 2 * (p ? J : J - 1);  // real columns of this parity
    const T *invp = inv + (size_t)p * J * J;
    const T *Af = A + (size_t)f * J * K * 2;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 64;
    using V = typename Acc<T>::V;
    V acc[2][4];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = V{0, 0, 0, 0};

    // global values of K-tile j0 for this thread's staging slots
    T ra[kALoads], rb[kBLoads];
    auto fetch = [&](int j0) {
#pragma unroll
        for (int u = 0; u < kALoads; ++u) {
            const int e = tid + u * kThreads;
            const int r = e / kTileK, k = e - r * kTileK;
            const int i = i0 + r, j = j0 + k;
            ra[u] = (i < J && j < J) ? invp[(size_t)i * J + j] : (T)0;
        }
#pragma unroll
        for (int u = 0; u < kBLoads; ++u) {
            const int e = tid + u * kThreads;
            const int k = e / kTileN, cc = e - k * kTileN;
            const int j = j0 + k, col = col0 + cc;
            T v = (T)0;
            if (j < J && col < ncols) v = Af[((size_t)j * K + ((col & ~1) + 1 - p)) * 2 + (col & 1)];
            rb[u] = v;
        }
    };
    fetch(0);
    for (int j0 = 0; j0 < J; j0 += kTileK) {
#pragma unroll
        for (int u = 0; u < kALoads; ++u) {
            const int e = tid + u * kThreads;
            As[e / kTileK][e % kTileK] = ra[u];
        }
#pragma unroll
        for (int u = 0; u < kBLoads; ++u) {
            const int e = tid + u * kThreads;
            Bs[e / kTileN][e % kTileN] = rb[u];
        }
        __syncthreads();
        if (j0 + kTileK < J) fetch(j0 + kTileK);
#pragma unroll
        for (int kk = 0; kk < kTileK; kk += 4) {
            T a[2], bv[4];
#pragma unroll
            for (int x = 0; x < 2; ++x) a[x] = As[wr + 16 * x + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
            for (int y = 0; y < 4; ++y) bv[y] = Bs[kk + (lane >> 4)][wc + 16 * y + (lane & 15)];
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) acc[x][y] = Acc<T>::mfma(a[x], bv[y], acc[x][y]);
        }
        __syncthreads();
    }

    // epilogue: exp form, scaled by 1/(2J) (the longitude normalisation)
    const T scale = (T)1 / (T)(2 * J);
    T *of = out + (size_t)f * (2 * J + 1) * K * 2;
#pragma unroll
    for (int y = 0; y < 4; ++y) {
        const int col = col0 + wc + 16 * y + (lane & 15);
        if (col >= ncols) continue;
        const int q = col & 1;             // 0: real part of the coefficient, 1: imaginary
        const int c = (col & ~1) + 1 - p;  // column of the exp-form array
#pragma unroll
        for (int x = 0; x < 2; ++x) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + wr + 16 * x + Acc<T>::row(lane, r);
                if (i >= J) continue;
                const T v = acc[x][y][r] * scale;
                if (p == 0) {
                    const int n = i;  // cos(n theta)
                    if (n == 0) {
                        of[((size_t)J * K + c) * 2 + q] = v;
                        of[((size_t)0 * K + c) * 2 + q] = (T)0;          // n = -J
                        of[((size_t)(2 * J) * K + c) * 2 + q] = (T)0;    // n = +J
                    } else {
                        of[((size_t)(J + n) * K + c) * 2 + q] = v * (T)0.5;
                        of[((size_t)(J - n) * K + c) * 2 + q] = v * (T)0.5;
                    }
                } else {
                    const int n = i + 1;  // sin(n theta): e(+n) = -i b / 2, e(-n) = +i b / 2
                    // part q of b lands in part 1 - q of e; re(e(+n)) = Im b / 2, im(e(+n)) = -Re b / 2
                    const T h = v * (T)0.5;
                    const T plus = q ? h : -h;
                    of[((size_t)(J + n) * K + c) * 2 + (1 - q)] = plus;
                    of[((size_t)(J - n) * K + c) * 2 + (1 - q)] = -plus;
                    if (i == 0) of[((size_t)J * K + c) * 2 + q] = (T)0;  // n = 0
                }
            }
        }
    }
}

template <typename T>
hipError_t launch_t(int J, int F, const void *inv, const void *A, void *out, hipStream_t s)
{
    const int tiles_m = (J + kTileM - 1) / kTileM;
    const int tiles_n0 = (2 * (J - 1) + kTileN - 1) / kTileN;
    const int tiles_n1 = (2 * J + kTileN - 1) / kTileN;
    const int blocks = F * tiles_m * (tiles_n0 + tiles_n1);
    hipLaunchKernelGGL(k_gl_latitude<T>, dim3(blocks), dim3(kThreads), 0, s, (const T *)inv, (const T *)A, (T *)out,
                       J, tiles_m, tiles_n0, tiles_n1);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_gl_latitude(int prec, int J, int n_fields, const void *inv, const void *A, void *out,
                              hipStream_t s)
{
    if (J < 16 || (J & 1)) return hipErrorInvalidValue;
    if (prec == 1) return launch_t<float>(J, n_fields, inv, A, out, s);
    return launch_t<double>(J, n_fields, inv, A, out, s);
}

}  // namespace nufft2
