// Exponential-of-semicircle interpolation of the fine grid at the sorted
// departure points (the per-point stage of the type-2 NUFFT).
//
//   out[f][perm[r]] = sum_{a<w} phi_t[a] * sum_{b<w} phi_p[b] * b_f[(it + a) mod nft][(ip + b) mod nfp]
//   phi_x[a] = exp(beta * (sqrt(1 - z_a^2) - 1)),  z_a = (a - floor(w/2) - v_x) / (w/2)
//
// One workgroup per bin (a tile_t x tile_p block of first-tap cells).  The
// workgroup stages the (tile_t + w - 1) x (tile_p + w - 1) patch of up to
// FG fields at once in LDS, then each thread sums the w x w taps of one
// point for all staged fields (independent accumulators per field).  The
// column weights are computed once per point and field group, the row
// weights on the fly.  The tap
// order (rows a outer, columns b inner) is fixed, so a point's value does not
// depend on where in its bin the sort placed it.
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

constexpr int kGatherMaxFields = 4;

constexpr int kGatherThreads = 256;
constexpr int kLoadBatch = 4;

template <typename T, int W, int FG>
__global__ __launch_bounds__(kGatherThreads) void k_gather(const cplx<T> *__restrict__ grid,
                                                           const PointRec<T> *__restrict__ rec,
                                                           const int32_t *__restrict__ perm,
                                                           const int32_t *__restrict__ binstart,
                                                           void *__restrict__ out, GatherParams gp)
{
    extern __shared__ unsigned char smem_raw[];
    cplx<T> *tiles = reinterpret_cast<cplx<T> *>(smem_raw);
    // Plain order: consecutive bins go to different XCDs, which spreads the
    // non-empty bins (points cover only half of the doubled torus) evenly.
    const int bin = (int)blockIdx.x;
    const int start = binstart[bin];
    const int cnt = binstart[bin + 1] - start;
    if (cnt == 0) return;
    const int bt = bin / gp.nbins_phi, bp = bin - bt * gp.nbins_phi;
    const int r0 = bt * gp.tile_t, c0 = bp * gp.tile_p;
    const int TR = gp.tile_t + W - 1, TC = gp.tile_p + W - 1;
    const int tile_elems = TR * TC;
    const T inv_hw = (T)2 / (T)W;
    const T beta = (T)gp.beta;
    constexpr int H = W / 2;
    const int64_t field_stride = (int64_t)gp.nft * gp.nfp;

    // FG fields per pass; the last pass may hold fewer (fg)
    for (int f0 = 0; f0 < gp.n_fields; f0 += FG) {
        const int fg = min(FG, gp.n_fields - f0);
        __syncthreads();
        // Stage the patch: each thread issues the loads of up to kLoadBatch
        // elements (all fields) before it stores any of them, so that one
        // memory round trip serves the batch.
        for (int e0 = 0; e0 < tile_elems; e0 += kLoadBatch * kGatherThreads) {
            cplx<T> buf[kLoadBatch][FG];
#pragma unroll
            for (int u = 0; u < kLoadBatch; ++u) {
                const int e = e0 + u * kGatherThreads + (int)threadIdx.x;
                const int ec = e < tile_elems ? e : 0;
                const int rr = ec / TC, cc = ec - rr * TC;
                const int64_t off =
                    (int64_t)((r0 + rr) & (gp.nft - 1)) * gp.nfp + ((c0 + cc) & (gp.nfp - 1));
#pragma unroll
                for (int f = 0; f < FG; ++f) {
                    const int ff = f0 + (f < fg ? f : 0);
                    buf[u][f] = grid[(int64_t)ff * field_stride + off];
                }
            }
#pragma unroll
            for (int u = 0; u < kLoadBatch; ++u) {
                const int e = e0 + u * kGatherThreads + (int)threadIdx.x;
                if (e < tile_elems) {
#pragma unroll
                    for (int f = 0; f < FG; ++f) tiles[f * tile_elems + e] = buf[u][f];
                }
            }
        }
        __syncthreads();
        for (int base = 0; base < cnt; base += blockDim.x) {
            const int r = base + (int)threadIdx.x;
            if (r >= cnt) continue;
            const PointRec<T> pr = rec[start + r];
            const int dst = perm[start + r];
            const bool bad = !(pr.vt == pr.vt) || !(pr.vp == pr.vp);
            const int lr = bad ? 0 : pr.it - r0;
            const int lc = bad ? 0 : pr.ip - c0;
            T wp[W];
#pragma unroll
            for (int b = 0; b < W; ++b) wp[b] = es_kernel<T>(((T)(b - H) - pr.vp) * inv_hw, beta);
            T ax[FG], ay[FG];
#pragma unroll
            for (int f = 0; f < FG; ++f) ax[f] = ay[f] = (T)0;
            // rows stay a loop: unrolling it lets the compiler hoist all w*w*FG
            // LDS loads and run out of registers
#pragma unroll 1
            for (int a = 0; a < W; ++a) {
                const T wt = es_kernel<T>(((T)(a - H) - pr.vt) * inv_hw, beta);
                const cplx<T> *row = tiles + (lr + a) * TC + lc;
                T rx[FG], ry[FG];
#pragma unroll
                for (int f = 0; f < FG; ++f) rx[f] = ry[f] = (T)0;
#pragma unroll
                for (int b = 0; b < W; ++b) {
#pragma unroll
                    for (int f = 0; f < FG; ++f) {
                        // fields past fg read stale LDS; their sums are never stored
                        const cplx<T> v = row[f * tile_elems + b];
                        rx[f] += wp[b] * v.x;
                        ry[f] += wp[b] * v.y;
                    }
                }
#pragma unroll
                for (int f = 0; f < FG; ++f) {
                    ax[f] += wt * rx[f];
                    ay[f] += wt * ry[f];
                }
            }
#pragma unroll
            for (int f = 0; f < FG; ++f) {
                if (f < fg) {
                    const int64_t o = (int64_t)(f0 + f) * gp.n_pts + dst;
                    const T x = bad ? (T)NAN : ax[f], y = bad ? (T)NAN : ay[f];
                    if (gp.real_output) reinterpret_cast<T *>(out)[o] = x;
                    else reinterpret_cast<cplx<T> *>(out)[o] = {x, y};
                }
            }
        }
    }
}

template <typename T, int W, int FG>
static hipError_t launch_wf(const GatherParams &gp, const void *grid, const void *rec,
                            const int32_t *perm, const int32_t *binstart, void *out, hipStream_t s)
{
    const size_t lds = sizeof(cplx<T>) * (size_t)(gp.tile_t + W - 1) * (gp.tile_p + W - 1) * FG;
    auto kern = k_gather<T, W, FG>;
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(kern, dim3((unsigned)gp.nbins), dim3(kGatherThreads), lds, s,
                       (const cplx<T> *)grid, (const PointRec<T> *)rec, perm, binstart, out, gp);
    return hipGetLastError();
}

template <typename T, int W>
static hipError_t launch_w(const GatherParams &gp, const void *grid, const void *rec, const int32_t *perm,
                           const int32_t *binstart, void *out, hipStream_t s)
{
    switch (gp.fields_per_pass) {
    case 1: return launch_wf<T, W, 1>(gp, grid, rec, perm, binstart, out, s);
    case 2: return launch_wf<T, W, 2>(gp, grid, rec, perm, binstart, out, s);
    case 3: return launch_wf<T, W, 3>(gp, grid, rec, perm, binstart, out, s);
    case 4: return launch_wf<T, W, 4>(gp, grid, rec, perm, binstart, out, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
static hipError_t launch_t(const GatherParams &gp, const void *grid, const void *rec, const int32_t *perm,
                           const int32_t *binstart, void *out, hipStream_t s)
{
    switch (gp.w) {
#define NUFFT2_W(X) case X: return launch_w<T, X>(gp, grid, rec, perm, binstart, out, s);
        NUFFT2_W(2) NUFFT2_W(3) NUFFT2_W(4) NUFFT2_W(5) NUFFT2_W(6) NUFFT2_W(7) NUFFT2_W(8)
        NUFFT2_W(9) NUFFT2_W(10) NUFFT2_W(11) NUFFT2_W(12) NUFFT2_W(13) NUFFT2_W(14)
        NUFFT2_W(15) NUFFT2_W(16)
#undef NUFFT2_W
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gather(int prec, const GatherParams &gp, const void *grid, const void *rec,
                         const int32_t *perm, const int32_t *binstart, void *out, hipStream_t s)
{
    if (gp.n_pts == 0) return hipSuccess;
    if (prec == 1) return launch_t<float>(gp, grid, rec, perm, binstart, out, s);
    return launch_t<double>(gp, grid, rec, perm, binstart, out, s);
}

}  // namespace nufft2
