// Deconvolution + zero padding + the upsampled 2-D inverse FFT, as two
// pruned passes of batched Stockham FFTs staged in LDS.
//
// The grid value at fine cell (l_t, l_p) is
//     b[l_t, l_p] = sum_n sum_m c[n,m] corr_t[n] corr_p[m] e^{+2 pi i (n l_t / nft + m l_p / nfp)}
// (unnormalised inverse DFT of the deconvolved, zero-padded coefficients).
//
//   theta pass: for each phi mode m (a batch of columns per workgroup) the
//     length-nft transform over n of the K_theta deconvolved coefficients;
//     only the theta rows some point's taps reach are written, to
//     S[l_t][m] (modes along the row, K_phi long).
//   phi pass: for each reached theta row, the length-nfp transform over m of
//     S[l_t][:], written to the fine grid b[l_t][:].
// Doing theta first keeps the intermediate at nft x K_phi (half the size of
// the other order's K_theta x nfp), and only reached rows are transformed
// in the phi pass.
//
// Each transform is a radix-8/4/2 Stockham sequence: the first stage reads
// straight from global memory into registers, the middle stages go through
// LDS, the last stage writes straight to global memory (both contiguous in
// the index the threads step through).  Twiddles e^{2 pi i t / N} come from
// a table the host fills in FP64 (long double) and rounds once.
#include "nufft2_internal.hpp"

namespace nufft2 {

template <typename C> __device__ inline C cadd(C a, C b) { return {a.x + b.x, a.y + b.y}; }
template <typename C> __device__ inline C csub(C a, C b) { return {a.x - b.x, a.y - b.y}; }
template <typename C> __device__ inline C cmul(C a, C b)
{
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// multiply by +i
template <typename C> __device__ inline C cmuli(C a) { return {-a.y, a.x}; }

// In-register DFTs with the + sign: y_q = sum_r x_r e^{+2 pi i r q / R}.
template <typename C> __device__ inline void dft2(C *x)
{
    const C a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
}

template <typename C> __device__ inline void dft4(C &x0, C &x1, C &x2, C &x3)
{
    const C t0 = cadd(x0, x2), t1 = csub(x0, x2);
    const C t2 = cadd(x1, x3), t3 = cmuli(csub(x1, x3));
    x0 = cadd(t0, t2);
    x2 = csub(t0, t2);
    x1 = cadd(t1, t3);
    x3 = csub(t1, t3);
}

template <typename C> __device__ inline void dft4(C *x) { dft4(x[0], x[1], x[2], x[3]); }

template <typename C> __device__ inline void dft8(C *x)
{
    using R = decltype(x[0].x);
    C e0 = x[0], e1 = x[2], e2 = x[4], e3 = x[6];
    C o0 = x[1], o1 = x[3], o2 = x[5], o3 = x[7];
    dft4(e0, e1, e2, e3);
    dft4(o0, o1, o2, o3);
    const R c = (R)0.70710678118654752440084436210484903928;
    // o_q *= e^{+i pi q / 4}
    const C w1 = {c * (o1.x - o1.y), c * (o1.x + o1.y)};
    const C w2 = cmuli(o2);
    const C w3 = {-c * (o3.x + o3.y), c * (o3.x - o3.y)};
    x[0] = cadd(e0, o0);
    x[4] = csub(e0, o0);
    x[1] = cadd(e1, w1);
    x[5] = csub(e1, w1);
    x[2] = cadd(e2, w2);
    x[6] = csub(e2, w2);
    x[3] = cadd(e3, w3);
    x[7] = csub(e3, w3);
}

template <typename T, int R> __device__ inline void dft(cplx<T> *x)
{
    if constexpr (R == 2) dft2(x);
    else if constexpr (R == 4) dft4(x);
    else dft8(x);
}

// One Stockham stage of radix R over B sequences of length N held in LDS at
// s[i * IS + b * BS].  Each thread owns E / R butterflies; butterfly (j, b)
// reads elements j + r N/R, applies twiddles W_{Ns R}^{r k} with k = j mod Ns,
// transforms, and writes element ((j - k) R + k) + r Ns.
// BFAST: consecutive threads step through b (else through j).
template <typename T, int R, int E, bool BFAST, bool FIRST, bool LAST, class Loader, class Storer>
__device__ inline void stockham_stage(cplx<T> *s, int N, int logB, int B, int Ns, int IS, int BS,
                                      const cplx<T> *__restrict__ tw, const Loader &ld,
                                      const Storer &st)
{
    constexpr int Q = E / R;
    const int nbf = N / R;
    cplx<T> v[E];
    int jj[Q], bb[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int job = threadIdx.x + q * blockDim.x;
        int j, b;
        if (BFAST) {
            b = job & (B - 1);
            j = job >> logB;
        } else {
            j = job & (nbf - 1);
            b = job / nbf;
        }
        jj[q] = j;
        bb[q] = b;
        const int k = j & (Ns - 1);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = j + r * nbf;
            if (FIRST) v[q * R + r] = ld(i, b);
            else v[q * R + r] = s[i * IS + b * BS];
        }
        if (!FIRST) {
            const int stride = N / (Ns * R);
#pragma unroll
            for (int r = 1; r < R; ++r) v[q * R + r] = cmul(v[q * R + r], tw[r * k * stride]);
        }
    }
    if (!FIRST) __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        dft<T, R>(&v[q * R]);
        const int j = jj[q], b = bb[q];
        const int k = j & (Ns - 1);
        const int base = (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int o = base + r * Ns;
            if (LAST) st(o, b, v[q * R + r]);
            else s[o * IS + b * BS] = v[q * R + r];
        }
    }
    if (!LAST) __syncthreads();
}

template <typename T, int R, int E, bool BFAST, class Loader, class Storer>
__device__ inline void stockham_dispatch(bool first, bool last, cplx<T> *s, int N, int logB, int B,
                                         int Ns, int IS, int BS, const cplx<T> *tw,
                                         const Loader &ld, const Storer &st)
{
    if (first && last)
        stockham_stage<T, R, E, BFAST, true, true>(s, N, logB, B, Ns, IS, BS, tw, ld, st);
    else if (first)
        stockham_stage<T, R, E, BFAST, true, false>(s, N, logB, B, Ns, IS, BS, tw, ld, st);
    else if (last)
        stockham_stage<T, R, E, BFAST, false, true>(s, N, logB, B, Ns, IS, BS, tw, ld, st);
    else
        stockham_stage<T, R, E, BFAST, false, false>(s, N, logB, B, Ns, IS, BS, tw, ld, st);
}

// Full length-N transform (N = 2^logN >= 8) of B sequences: a radix 2 or 4
// stage first if logN is not a multiple of 3, then radix-8 stages.
template <typename T, int E, bool BFAST, class Loader, class Storer>
__device__ inline void fft_batch(cplx<T> *s, int logN, int logB, int IS, int BS,
                                 const cplx<T> *tw, const Loader &ld, const Storer &st)
{
    const int N = 1 << logN, B = 1 << logB;
    int rem = logN % 3;
    int nst = logN / 3 + (rem ? 1 : 0);
    int Ns = 1;
    for (int si = 0; si < nst; ++si) {
        const bool first = si == 0, last = si == nst - 1;
        const int R = (si == 0 && rem) ? (1 << rem) : 8;
        if (R == 8) stockham_dispatch<T, 8, E, BFAST>(first, last, s, N, logB, B, Ns, IS, BS, tw, ld, st);
        else if (R == 4) stockham_dispatch<T, 4, E, BFAST>(first, last, s, N, logB, B, Ns, IS, BS, tw, ld, st);
        else stockham_dispatch<T, 2, E, BFAST>(first, last, s, N, logB, B, Ns, IS, BS, tw, ld, st);
        Ns *= R;
    }
}

// FFT index i -> centred mode index a in [0, K), or -1 for zero padding.
__device__ inline int mode_of(int i, int K, int N)
{
    const int half = K >> 1, kmax = K - 1 - half;
    if (i <= kmax) return i + half;
    if (i >= N - half) return i - N + half;
    return -1;
}

template <typename T> struct ThetaLoad {
    const cplx<T> *coef;  // this field
    const T *ct, *cp;
    int Kt, Kp, nft, m0;
    __device__ cplx<T> operator()(int i, int b) const
    {
        const int m = m0 + b;
        const int a = mode_of(i, Kt, nft);
        if (a < 0 || m >= Kp) return {(T)0, (T)0};
        const cplx<T> c = coef[(int64_t)a * Kp + m];
        const T sc = ct[a] * cp[m];
        return {c.x * sc, c.y * sc};
    }
};

template <typename T> struct ThetaStore {
    cplx<T> *S;  // this field, [nft][Kp]
    const uint8_t *touched;
    int Kp, m0;
    __device__ void operator()(int l, int b, cplx<T> v) const
    {
        const int m = m0 + b;
        if (m < Kp && touched[l]) S[(int64_t)l * Kp + m] = v;
    }
};

template <typename T, int E>
__global__ __launch_bounds__(1024) void k_theta_pass(const cplx<T> *__restrict__ coeffs,
                                                     const T *__restrict__ corr_t,
                                                     const T *__restrict__ corr_p,
                                                     const cplx<T> *__restrict__ tw,
                                                     const uint8_t *__restrict__ touched,
                                                     cplx<T> *__restrict__ S, FFTParams fp)
{
    extern __shared__ unsigned char smem_raw[];
    cplx<T> *s = reinterpret_cast<cplx<T> *>(smem_raw);
    const int f = blockIdx.y;
    const int m0 = blockIdx.x * fp.theta_batch;
    ThetaLoad<T> ld{coeffs + (int64_t)f * fp.Kt * fp.Kp, corr_t, corr_p, fp.Kt, fp.Kp, fp.nft, m0};
    ThetaStore<T> st{S + (int64_t)f * fp.nft * fp.Kp, touched, fp.Kp, m0};
    // layout [i][b]: consecutive threads take consecutive columns
    fft_batch<T, E, true>(s, fp.log_nft, fp.log_theta_batch, fp.theta_batch, 1, tw, ld, st);
}

template <typename T> struct PhiLoad {
    const cplx<T> *S;  // this field, [nft][Kp]
    int Kp, nfp, l0;
    __device__ cplx<T> operator()(int i, int b) const
    {
        const int a = mode_of(i, Kp, nfp);
        if (a < 0) return {(T)0, (T)0};
        return S[(int64_t)(l0 + b) * Kp + a];
    }
};

template <typename T> struct PhiStore {
    cplx<T> *grid;  // this field, [nft][nfp]
    const uint8_t *touched;
    int nfp, l0;
    __device__ void operator()(int o, int b, cplx<T> v) const
    {
        const int l = l0 + b;
        if (touched[l]) grid[(int64_t)l * nfp + o] = v;
    }
};

template <typename T, int E>
__global__ __launch_bounds__(1024) void k_phi_pass(const cplx<T> *__restrict__ S,
                                                   const cplx<T> *__restrict__ tw,
                                                   const uint8_t *__restrict__ touched,
                                                   cplx<T> *__restrict__ grid, FFTParams fp)
{
    extern __shared__ unsigned char smem_raw[];
    cplx<T> *s = reinterpret_cast<cplx<T> *>(smem_raw);
    const int f = blockIdx.y;
    const int l0 = blockIdx.x * fp.phi_batch;
    // skip the workgroup when none of its rows is reached by any point
    __shared__ int any;
    if (threadIdx.x == 0) {
        int a = 0;
        for (int b = 0; b < fp.phi_batch; ++b) a |= touched[l0 + b];
        any = a;
    }
    __syncthreads();
    if (!any) return;
    PhiLoad<T> ld{S + (int64_t)f * fp.nft * fp.Kp, fp.Kp, fp.nfp, l0};
    PhiStore<T> st{grid + (int64_t)f * fp.nft * fp.nfp, touched, fp.nfp, l0};
    // layout [b][i]: consecutive threads take consecutive elements of a row
    fft_batch<T, E, false>(s, fp.log_nfp, fp.log_phi_batch, 1, 1 << fp.log_nfp, tw, ld, st);
}

constexpr int kElemsPerThread = 16;

hipError_t launch_theta_pass(int prec, const FFTParams &fp, const void *coeffs, const void *corr_t,
                             const void *corr_p, const void *tw_t, const uint8_t *rowtouched,
                             void *S, hipStream_t s)
{
    const int NB = fp.nft * fp.theta_batch;
    const int threads = NB / kElemsPerThread;
    const dim3 grid((fp.Kp + fp.theta_batch - 1) / fp.theta_batch, fp.n_fields);
    if (prec == 1) {
        const size_t lds = sizeof(float2) * (size_t)NB;
        auto kern = k_theta_pass<float, kElemsPerThread>;
        if (lds > 65536) (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(kern, grid, dim3(threads), lds, s, (const float2 *)coeffs,
                           (const float *)corr_t, (const float *)corr_p, (const float2 *)tw_t,
                           rowtouched, (float2 *)S, fp);
    } else {
        const size_t lds = sizeof(double2) * (size_t)NB;
        auto kern = k_theta_pass<double, kElemsPerThread>;
        if (lds > 65536) (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(kern, grid, dim3(threads), lds, s, (const double2 *)coeffs,
                           (const double *)corr_t, (const double *)corr_p, (const double2 *)tw_t,
                           rowtouched, (double2 *)S, fp);
    }
    return hipGetLastError();
}

hipError_t launch_phi_pass(int prec, const FFTParams &fp, const void *S, const void *tw_p,
                           const uint8_t *rowtouched, void *grid, hipStream_t s)
{
    const int NB = fp.nfp * fp.phi_batch;
    const int threads = NB / kElemsPerThread;
    const dim3 g(fp.nft / fp.phi_batch, fp.n_fields);
    if (prec == 1) {
        const size_t lds = sizeof(float2) * (size_t)NB;
        auto kern = k_phi_pass<float, kElemsPerThread>;
        if (lds > 65536) (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(kern, g, dim3(threads), lds, s, (const float2 *)S, (const float2 *)tw_p,
                           rowtouched, (float2 *)grid, fp);
    } else {
        const size_t lds = sizeof(double2) * (size_t)NB;
        auto kern = k_phi_pass<double, kElemsPerThread>;
        if (lds > 65536) (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(kern, g, dim3(threads), lds, s, (const double2 *)S, (const double2 *)tw_p,
                           rowtouched, (double2 *)grid, fp);
    }
    return hipGetLastError();
}

}  // namespace nufft2
