// Point setup: wrap each departure point onto the periodic fine grid in FP64,
// split it into a first-tap cell and an offset, and counting-sort the points
// by gather tile ("bin").
//
// Pipeline (all on the plan's stream):
//   k_fill_zero        clear bin counts and the theta-row marks
//   k_setpts_bin       per point: wrap/split, bin id, rank within the bin
//                      (atomic), mark the first-tap theta row
//   k_bin_scan         one workgroup: exclusive scan of the bin counts, and
//                      the set of theta rows any point's taps reach
//   k_setpts_scatter   per point: recompute the split, write the packed
//                      record at binstart[bin] + rank, and the permutation
//
// The order of points inside a bin depends on atomic arbitration; the output
// of an exec does not, because each point's sum is computed by one thread in a
// fixed tap order from the same grid values wherever it sits in its bin.
#include "nufft2_internal.hpp"

namespace nufft2 {

__global__ void k_fill_zero(uint32_t *p, int64_t n_words)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_words; i += stride)
        p[i] = 0u;
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s)
{
    const int64_t words = (int64_t)((bytes + 3) / 4);
    if (words == 0) return hipSuccess;
    int64_t blocks = (words + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t *)p, words);
    return hipGetLastError();
}

// Split one FP64 coordinate x (radians, any real) into (i0 mod nf, v).
// t = x * nf / 2pi is reduced into [0, nf) exactly (nf is a power of two, so
// t / nf and k * nf are exact); i0 = ceil(t - w/2) is the first tap, so the
// taps i0 .. i0 + w - 1 cover t with |t - l| <= w/2.  u = t - i0 is exact in
// FP64 and lies in (w/2 - 1, w/2]; the stored offset is v = u - floor(w/2),
// |v| <= 1, so that rounding it to FP32 costs at most 2^-25 cells.
template <typename T>
__device__ inline void split_axis(double x, const AxisParams &ax, int w, int32_t &i0m, T &v)
{
    const double nf = (double)ax.nf;
    double t = x * ax.to_grid;
    t = t - nf * floor(t / nf);
    if (t >= nf) t -= nf;             // t slightly below 0 rounds up to nf
    const double c = ceil(t - 0.5 * (double)w);
    const double u = t - c;
    int32_t i0 = (int32_t)c;
    i0 &= (ax.nf - 1);                // c >= -w/2 > -nf: masking is the positive modulus
    i0m = i0;
    v = (T)(u - (double)(w >> 1));
}

template <typename T>
__global__ void k_setpts_bin(const double *__restrict__ phi, const double *__restrict__ theta,
                             SetptsParams sp, int32_t *__restrict__ bincount,
                             int2 *__restrict__ keyrank, uint8_t *__restrict__ rowmark,
                             int32_t *__restrict__ flags)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < sp.n; j += stride) {
        const double ph = phi[j], th = theta[j];
        int32_t bin;
        if (!isfinite(ph) || !isfinite(th)) {
            atomicOr(flags, 1);
            bin = 0;
        } else {
            int32_t it, ip;
            T vt, vp;
            split_axis<T>(th, sp.th, sp.w, it, vt);
            split_axis<T>(ph, sp.ph, sp.w, ip, vp);
            bin = (it / sp.th.tile) * sp.nbins_phi + ip / sp.ph.tile;
            rowmark[it] = 1;
        }
        const int32_t rank = atomicAdd(&bincount[bin], 1);
        keyrank[j] = make_int2(bin, rank);
    }
}

// Block-wide exclusive scan of one int per thread (blockDim.x a multiple of 64).
__device__ inline int block_exclusive_scan(int x, int *lds, int &total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    int incl = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(incl, d, 64);
        if (lane >= d) incl += y;
    }
    if (lane == 63) lds[wid] = incl;
    __syncthreads();
    if (wid == 0) {
        const int wv = lane < nwaves ? lds[lane] : 0;
        int wi = wv;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int y = __shfl_up(wi, d, 64);
            if (lane >= d) wi += y;
        }
        if (lane < nwaves) lds[lane] = wi - wv;
        if (lane == nwaves - 1) lds[32] = wi;
    }
    __syncthreads();
    const int res = incl - x + lds[wid];
    total = lds[32];
    __syncthreads();
    return res;
}

// One workgroup of 1024 threads.  Each pass scans CHUNK * 1024 bins, every
// thread owning CHUNK consecutive bins.
__global__ __launch_bounds__(1024) void k_bin_scan(const int32_t *__restrict__ bincount,
                                                   int32_t *__restrict__ binstart, int64_t nbins,
                                                   const uint8_t *__restrict__ rowmark,
                                                   uint8_t *__restrict__ rowtouched, int nft, int w)
{
    constexpr int CHUNK = 16;
    __shared__ int lds[33];
    int carry = 0;
    for (int64_t base = 0; base < nbins; base += (int64_t)CHUNK * blockDim.x) {
        const int64_t mine = base + (int64_t)threadIdx.x * CHUNK;
        int vals[CHUNK];
        int sum = 0;
#pragma unroll
        for (int c = 0; c < CHUNK; ++c) {
            vals[c] = (mine + c < nbins) ? bincount[mine + c] : 0;
            sum += vals[c];
        }
        int total;
        int run = carry + block_exclusive_scan(sum, lds, total);
#pragma unroll
        for (int c = 0; c < CHUNK; ++c) {
            if (mine + c < nbins) binstart[mine + c] = run;
            run += vals[c];
        }
        carry += total;
    }
    // A theta row l is read by the gather iff some point's first tap row is
    // within w - 1 rows below it (cyclically).
    for (int l = threadIdx.x; l < nft; l += blockDim.x) {
        uint8_t t = 0;
        for (int a = 0; a < w; ++a) t |= rowmark[(l - a + nft) & (nft - 1)];
        rowtouched[l] = t;
    }
}

template <typename T>
__global__ void k_setpts_scatter(const double *__restrict__ phi, const double *__restrict__ theta,
                                 SetptsParams sp, const int2 *__restrict__ keyrank,
                                 const int32_t *__restrict__ binstart,
                                 PointRec<T> *__restrict__ rec, int32_t *__restrict__ perm)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < sp.n; j += stride) {
        const double ph = phi[j], th = theta[j];
        PointRec<T> r;
        if (!isfinite(ph) || !isfinite(th)) {
            r.it = 0;
            r.ip = 0;
            r.vt = (T)NAN;
            r.vp = (T)NAN;
        } else {
            split_axis<T>(th, sp.th, sp.w, r.it, r.vt);
            split_axis<T>(ph, sp.ph, sp.w, r.ip, r.vp);
        }
        const int2 kr = keyrank[j];
        const int32_t pos = binstart[kr.x] + kr.y;
        rec[pos] = r;
        perm[pos] = (int32_t)j;
    }
}

hipError_t launch_setpts(int prec, const SetptsParams &sp, const double *phi, const double *theta,
                         int32_t *bincount, int32_t *binstart, int64_t nbins, int2 *keyrank,
                         uint8_t *rowmark, uint8_t *rowtouched, void *rec, int32_t *perm,
                         int32_t *flags, hipStream_t s)
{
    hipError_t e;
    if ((e = launch_fill_zero(bincount, sizeof(int32_t) * (size_t)nbins, s)) != hipSuccess) return e;
    if ((e = launch_fill_zero(rowmark, (size_t)sp.th.nf, s)) != hipSuccess) return e;
    if ((e = launch_fill_zero(flags, sizeof(int32_t), s)) != hipSuccess) return e;
    const int threads = 256;
    int64_t blocks = (sp.n + threads - 1) / threads;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    if (sp.n > 0) {
        if (prec == 1)
            hipLaunchKernelGGL(k_setpts_bin<float>, dim3((unsigned)blocks), dim3(threads), 0, s, phi,
                               theta, sp, bincount, keyrank, rowmark, flags);
        else
            hipLaunchKernelGGL(k_setpts_bin<double>, dim3((unsigned)blocks), dim3(threads), 0, s, phi,
                               theta, sp, bincount, keyrank, rowmark, flags);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, s, bincount, binstart, nbins, rowmark,
                       rowtouched, sp.th.nf, sp.w);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (sp.n > 0) {
        if (prec == 1)
            hipLaunchKernelGGL(k_setpts_scatter<float>, dim3((unsigned)blocks), dim3(threads), 0, s,
                               phi, theta, sp, keyrank, binstart, (PointRec<float> *)rec, perm);
        else
            hipLaunchKernelGGL(k_setpts_scatter<double>, dim3((unsigned)blocks), dim3(threads), 0, s,
                               phi, theta, sp, keyrank, binstart, (PointRec<double> *)rec, perm);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace nufft2
