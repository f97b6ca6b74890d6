// Exponential-of-semicircle interpolation of the fine grid at the sorted
// departure points (the per-point stage of the type-2 NUFFT).
//
//   out[f][perm[r]] = sum_{a<w} phi_t[a] * sum_{b<w} phi_p[b] * b_f[(it + a) mod nft][(ip + b) mod nfp]
//   phi_x[a] = exp(beta * (sqrt(1 - z_a^2) - 1)),  z_a = (a - floor(w/2) - v_x) / (w/2)
//
// One workgroup per bin (a tile_t x tile_p block of first-tap cells).  The
// workgroup stages the (tile_t + w - 1) x (tile_p + w - 1) patch of one field
// at a time in LDS, and each thread sums the w x w taps of one point.  The
// kernel weights are computed once per point and reused for every field.
// The tap order (rows a outer, columns b inner) is fixed, so a point's value
// does not depend on where in its bin the sort placed it.
#include "nufft2_internal.hpp"

namespace nufft2 {

template <typename T> __device__ inline T es_kernel(T z, T beta);
template <> __device__ inline float es_kernel<float>(float z, float beta)
{
    float t = 1.0f - z * z;
    t = t > 0.0f ? t : 0.0f;
    return __expf(beta * (__fsqrt_rn(t) - 1.0f));
}
template <> __device__ inline double es_kernel<double>(double z, double beta)
{
    double t = 1.0 - z * z;
    t = t > 0.0 ? t : 0.0;
    return exp(beta * (sqrt(t) - 1.0));
}

template <typename T, int W>
__global__ __launch_bounds__(256) void k_gather(const cplx<T> *__restrict__ grid,
                                                const PointRec<T> *__restrict__ rec,
                                                const int32_t *__restrict__ perm,
                                                const int32_t *__restrict__ bincount,
                                                const int32_t *__restrict__ binstart,
                                                void *__restrict__ out, GatherParams gp)
{
    extern __shared__ unsigned char smem_raw[];
    cplx<T> *tile = reinterpret_cast<cplx<T> *>(smem_raw);
    const int bin = blockIdx.x;
    const int cnt = bincount[bin];
    if (cnt == 0) return;
    const int start = binstart[bin];
    const int bt = bin / gp.nbins_phi, bp = bin - bt * gp.nbins_phi;
    const int r0 = bt * gp.tile_t, c0 = bp * gp.tile_p;
    const int TR = gp.tile_t + W - 1, TC = gp.tile_p + W - 1;
    const T inv_hw = (T)2 / (T)W;
    const T beta = (T)gp.beta;
    constexpr int H = W / 2;

    for (int base = 0; base < cnt; base += blockDim.x) {
        const int r = base + (int)threadIdx.x;
        const bool valid = r < cnt;
        T wt[W], wp[W];
        int lr = 0, lc = 0, dst = 0;
        bool bad = false;
        if (valid) {
            const PointRec<T> pr = rec[start + r];
            dst = perm[start + r];
            lr = pr.it - r0;
            lc = pr.ip - c0;
            bad = !(pr.vt == pr.vt) || !(pr.vp == pr.vp);
#pragma unroll
            for (int a = 0; a < W; ++a) {
                wt[a] = es_kernel<T>(((T)(a - H) - pr.vt) * inv_hw, beta);
                wp[a] = es_kernel<T>(((T)(a - H) - pr.vp) * inv_hw, beta);
            }
            if (bad) lr = lc = 0;
        }
        for (int f = 0; f < gp.n_fields; ++f) {
            const cplx<T> *g = grid + (int64_t)f * gp.nft * gp.nfp;
            __syncthreads();
            for (int e = threadIdx.x; e < TR * TC; e += blockDim.x) {
                const int rr = e / TC, cc = e - rr * TC;
                const int gr = (r0 + rr) & (gp.nft - 1), gc = (c0 + cc) & (gp.nfp - 1);
                tile[e] = g[(int64_t)gr * gp.nfp + gc];
            }
            __syncthreads();
            if (valid) {
                T ax = 0, ay = 0;
#pragma unroll
                for (int a = 0; a < W; ++a) {
                    const cplx<T> *row = tile + (lr + a) * TC + lc;
                    T rx = 0, ry = 0;
#pragma unroll
                    for (int b = 0; b < W; ++b) {
                        const cplx<T> v = row[b];
                        rx += wp[b] * v.x;
                        ry += wp[b] * v.y;
                    }
                    ax += wt[a] * rx;
                    ay += wt[a] * ry;
                }
                if (bad) ax = ay = (T)NAN;
                if (gp.real_output)
                    reinterpret_cast<T *>(out)[(int64_t)f * gp.n_pts + dst] = ax;
                else
                    reinterpret_cast<cplx<T> *>(out)[(int64_t)f * gp.n_pts + dst] = {ax, ay};
            }
        }
    }
}

template <typename T, int W>
static hipError_t launch_w(const GatherParams &gp, const void *grid, const void *rec, const int32_t *perm,
                           const int32_t *bincount, const int32_t *binstart, void *out, hipStream_t s)
{
    const size_t lds = sizeof(cplx<T>) * (size_t)(gp.tile_t + W - 1) * (gp.tile_p + W - 1);
    auto kern = k_gather<T, W>;
    if (lds > 65536) (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(kern, dim3((unsigned)gp.nbins), dim3(256), lds, s, (const cplx<T> *)grid,
                       (const PointRec<T> *)rec, perm, bincount, binstart, out, gp);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_t(const GatherParams &gp, const void *grid, const void *rec, const int32_t *perm,
                           const int32_t *bincount, const int32_t *binstart, void *out, hipStream_t s)
{
    switch (gp.w) {
#define NUFFT2_W(X) case X: return launch_w<T, X>(gp, grid, rec, perm, bincount, binstart, out, s);
        NUFFT2_W(2) NUFFT2_W(3) NUFFT2_W(4) NUFFT2_W(5) NUFFT2_W(6) NUFFT2_W(7) NUFFT2_W(8)
        NUFFT2_W(9) NUFFT2_W(10) NUFFT2_W(11) NUFFT2_W(12) NUFFT2_W(13) NUFFT2_W(14)
        NUFFT2_W(15) NUFFT2_W(16)
#undef NUFFT2_W
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gather(int prec, const GatherParams &gp, const void *grid, const void *rec,
                         const int32_t *perm, const int32_t *bincount, const int32_t *binstart,
                         void *out, hipStream_t s)
{
    if (gp.n_pts == 0) return hipSuccess;
    if (prec == 1) return launch_t<float>(gp, grid, rec, perm, bincount, binstart, out, s);
    return launch_t<double>(gp, grid, rec, perm, bincount, binstart, out, s);
}

}  // namespace nufft2
