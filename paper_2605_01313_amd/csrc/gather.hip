// Exponential-of-semicircle interpolation of the fine grid at the sorted
// departure points (the per-point stage of the type-2 NUFFT).
//
//   out[f][perm[r]] = sum_{a<w} phi_t[a] * sum_{b<w} phi_p[b] * b_f[(it + a) mod nft][(ip + b) mod nfp]
//   phi_x[a] = exp(beta * (sqrt(1 - z_a^2) - 1)),  z_a = (a - floor(w/2) - v_x) / (w/2)
//
// One workgroup per bin (a tile_t x tile_p block of first-tap cells).  The
// workgroup stages the (tile_t + w - 1) x (tile_p + w - 1) patch of up to
// FG fields at once in LDS, then each thread sums the w x w taps of one
// point for all staged fields (independent accumulators per field; in FP64
// a bin of at most 128 points gives each point two threads, one per half of
// the rows).  Points are dealt to lanes so that the lanes the LDS serves
// together read different banks (the chunk loop and column_rotation).  The
// column weights are computed once per point and field group, the row
// weights on the fly.  The tap order (rows a outer, columns inner in one of
// two orders fixed by the point's own cell) does not depend on which lane or
// where in its bin the sort placed the point.
#include "nufft2_internal.hpp"

namespace nufft2 {

// ES kernel exp(beta (sqrt(1 - z^2) - 1)), clamped to e^{-beta} outside |z| <= 1.
// The second argument is es_constant(beta).  FP32 uses the hardware square
// root and base-2 exponential (about 1 ulp each, far inside a 1e-6 tolerance)
// with beta log2(e) folded in; FP64 uses the correctly rounded library calls.
template <typename T> __host__ __device__ inline T es_constant(double beta);
template <> __host__ __device__ inline float es_constant<float>(double beta)
{
    return (float)(beta * 1.4426950408889634);
}
template <> __host__ __device__ inline double es_constant<double>(double beta) { return beta; }

template <typename T> __device__ inline T es_kernel(T z, T k);
template <> __device__ inline float es_kernel<float>(float z, float k)
{
    const float t = fmaxf(1.0f - z * z, 0.0f);
    return __builtin_amdgcn_exp2f(__builtin_amdgcn_sqrtf(t) * k - k);
}
template <> __device__ inline double es_kernel<double>(double z, double k)
{
    double t = 1.0 - z * z;
    t = t > 0.0 ? t : 0.0;
    return exp(k * (sqrt(t) - 1.0));
}

constexpr int kGatherThreads = 256;
constexpr int kLoadBatch = 4;
// FP64 splits the rows of a point over two lanes when a chunk holds at most
// half a workgroup's points (see gather_body).
template <typename T> constexpr bool kSplitRows = sizeof(T) == 8;

// Lanes the LDS serves together for reads of one complex element: 16, in
// FP32 (8-byte reads, 128 bytes) and in FP64 (16-byte reads, 256 bytes over
// 64 four-byte banks).  A CPU model of the tap reads with these groups and
// bank slots (element offset modulo 16) reproduces the conflict rates
// measured on gfx950 with SQ_LDS_BANK_CONFLICT for the 2048^2 wind
// workload.  Lanes of such a group whose patch offsets differ modulo 16
// never collide on a bank, whatever tap they read.
template <typename T> constexpr int lds_lane_group() { return 16; }

// Departure points sit near a lattice of spacing 2 fine cells (the grid nodes
// at upsampling factor 2), so the patch offsets of the points of a bin share
// their parity and a plain layout leaves half of the banks idle.  Points on
// the two colours of a checkerboard over that lattice read their columns in
// two orders (0 .. w-1, or 1 .. w-1 then 0), which moves half of them to the
// other parity.  The order depends only on the point's own cell.
__device__ inline int column_rotation(int it, int ip) { return ((it >> 1) ^ (ip >> 1)) & 1; }

// blk: this workgroup's index in the stage (8 * ceil(nbins / 8) of them).
template <typename T, int W, int FG>
__device__ inline void gather_body(int blk, const cplx<T> *__restrict__ grid, const PointRec<T> *__restrict__ rec,
                                   const int32_t *__restrict__ perm, const int32_t *__restrict__ binlist,
                                   void *__restrict__ out, const GatherParams &gp)
{
    // The dynamic region starts right after the static LDS arrays below;
    // without the alignment a static array whose size is not a multiple of
    // 16 bytes misaligns every 16-byte complex read of the patch (a 4-6x
    // slower gather, measured).
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T> *tiles = reinterpret_cast<cplx<T> *>(smem_raw);
    // Workgroups are dealt to the 8 XCDs round-robin.  XCD x (= blk & 7)
    // takes the x-th eighth of the non-empty bins in bin order, so that the
    // bins running together on one XCD are neighbours and the halo rows and
    // columns their patches share come from that XCD's L2 (about 30% less
    // HBM traffic than plain bin order).  Only non-empty bins are dealt (the
    // points cover about half of the doubled torus), so the XCDs get equal
    // shares.  The grid has 8 * ceil(nbins / 8) workgroups.  Every setpts
    // with points writes each workgroup's entry (zero count: nothing to
    // do), so one load finds the bin; the number of non-empty bins, read
    // beside it, is zero after a setpts without points (whose table is not
    // rewritten above kDealtMaxBins bins).
    const int n_ne = binlist[gp.nbins];
    const int4 bi = bin_dealt(binlist, gp.nbins)[blk];  // {bin, first record, count, 0}
    if (n_ne == 0) return;
    const int bin = bi.x;
    const int start = bi.y;
    const int cnt = bi.z;
    if (cnt == 0) return;
    // the first chunk's records and destinations are requested now, so that
    // they arrive with the patch instead of after it
    PointRec<T> q0{};
    int d0 = 0;
    if ((int)threadIdx.x < cnt) {
        q0 = rec[start + (int)threadIdx.x];
        d0 = perm[start + (int)threadIdx.x];
    }
    const int bt = bin / gp.nbins_phi, bp = bin - bt * gp.nbins_phi;
    const int r0 = bt * gp.tile_t, c0 = bp * gp.tile_p;
    const int TR = gp.tile_t + W - 1, TC = gp.tile_p + W - 1;
    const int tile_elems = TR * TC;  // patch elements of one field
    // LDS row pitch (FP64 may pad rows; FP32 never does, so that a staged
    // element's LDS index is its patch index) and LDS elements per field
    const int TCP = sizeof(T) == 4 ? TC : gp.tile_pitch;
    const int plane = TR * TCP;
    const T inv_hw = (T)2 / (T)W;
    const T kc = es_constant<T>(gp.beta);
    constexpr int H = W / 2;
    constexpr int RU = sizeof(T) == 8 ? 2 : 1;
    constexpr int NK = lds_lane_group<T>();
    __shared__ int bucket[NK];  // per bank key: count, then start
    __shared__ short slot[kGatherThreads];  // lane -> point of the chunk (-1: none)
    __shared__ int dsts[kGatherThreads];    // destination of each point of the chunk
    __shared__ PointRec<T> recs[kGatherThreads];  // record of each point of the chunk
    __shared__ T xsum[kSplitRows<T> ? kGatherThreads / 2 * 2 * FG : 1];  // partial sums of split points
    const int64_t field_stride = (int64_t)gp.nft * gp.nfp;

    // FG fields per pass; the last pass may hold fewer (fg)
    for (int f0 = 0; f0 < gp.n_fields; f0 += FG) {
        const int fg = min(FG, gp.n_fields - f0);
        __syncthreads();
        // Stage the patch: each thread issues the loads of up to kLoadBatch
        // elements (all fields) before it stores any of them, so that one
        // memory round trip serves the batch.
        // A thread's elements of a batch are kGatherThreads apart.  In FP32
        // their (row, column) in the patch follow from the first one by the
        // fixed step (step_r rows, step_c columns, with a carry): one integer
        // division per batch instead of one per element (3% of the gather at
        // 256 x 512; in FP64, with two batches, the compiler's code for it
        // measured 1% slower, so FP64 divides per element).
        const int step_r = kGatherThreads / TC, step_c = kGatherThreads - step_r * TC;
        for (int e0 = 0; e0 < tile_elems; e0 += kLoadBatch * kGatherThreads) {
            cplx<T> buf[kLoadBatch][FG];
            int li[kLoadBatch];  // LDS index of each element (FP64)
            int rr = (e0 + (int)threadIdx.x) / TC;
            int cc = e0 + (int)threadIdx.x - rr * TC;
#pragma unroll
            for (int u = 0; u < kLoadBatch; ++u) {
                const int e = e0 + u * kGatherThreads + (int)threadIdx.x;
                if constexpr (sizeof(T) == 8) {
                    rr = (e < tile_elems ? e : 0) / TC;
                    cc = (e < tile_elems ? e : 0) - rr * TC;
                    li[u] = rr * TCP + cc;
                }
                const bool live = e < tile_elems;
                const int64_t off = live ? (int64_t)((r0 + rr) & (gp.nft - 1)) * gp.nfp + ((c0 + cc) & (gp.nfp - 1))
                                         : (int64_t)(r0 & (gp.nft - 1)) * gp.nfp + (c0 & (gp.nfp - 1));
#pragma unroll
                for (int f = 0; f < FG; ++f) {
                    const int ff = f0 + (f < fg ? f : 0);
                    buf[u][f] = grid[(int64_t)ff * field_stride + off];
                }
                if constexpr (sizeof(T) == 4) {
                    rr += step_r;
                    cc += step_c;
                    if (cc >= TC) {
                        cc -= TC;
                        ++rr;
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < kLoadBatch; ++u) {
                const int e = e0 + u * kGatherThreads + (int)threadIdx.x;
                if (e < tile_elems) {
                    const int l = sizeof(T) == 4 ? e : li[u];
#pragma unroll
                    for (int f = 0; f < FG; ++f) tiles[f * plane + l] = buf[u][f];
                }
            }
        }
        __syncthreads();
        for (int base = 0; base < cnt; base += kGatherThreads) {
            // Deal this chunk's points to lanes: counting-sort them by bank
            // key (patch offset of the first tap plus the column rotation,
            // modulo NK), then give sorted position k to lane
            // (k mod R) * NK + k / R.  Points R apart in key order share a
            // lane group, so a group holds distinct keys unless one key has
            // more than R points.  The order inside a key (atomic ranks) does
            // not matter: a point's sum does not depend on its lane.
            const int n = min(kGatherThreads, cnt - base);
            const int R = (n + NK - 1) / NK;
            const int t = (int)threadIdx.x;
            if (t < NK) bucket[t] = 0;
            slot[t] = -1;
            __syncthreads();
            int key = 0, rank = 0;
            if (t < n) {
                PointRec<T> q = q0;
                int d = d0;
                if (base > 0) {
                    q = rec[start + base + t];
                    d = perm[start + base + t];
                }
                dsts[t] = d;
                recs[t] = q;
                const bool qbad = !(q.vt == q.vt) || !(q.vp == q.vp);
                key = qbad ? 0 : ((q.it - r0) * TCP + (q.ip - c0) + column_rotation(q.it, q.ip)) & (NK - 1);
                rank = atomicAdd(&bucket[key], 1);
            }
            __syncthreads();
            if (t < NK) {
                // exclusive scan of the NK bucket counts within wave 0
                const int c = bucket[t];
                int incl = c;
#pragma unroll
                for (int d = 1; d < NK; d <<= 1) {
                    const int y = __shfl_up(incl, d, 64);
                    if (t >= d) incl += y;
                }
                bucket[t] = incl - c;
            }
            __syncthreads();
            if (t < n) {
                const int k = bucket[key] + rank;
                slot[(k % R) * NK + k / R] = (short)t;
            }
            __syncthreads();
            // In FP64 a bin of at most half a workgroup's points (one chunk,
            // which the dealing put on the lower half of the lanes) is split
            // by rows: lane t + 128 takes rows H1 .. w-1 of lane t's point
            // and hands its partial sums over through LDS, so that all four
            // waves work on the taps instead of two.  The choice depends on
            // the bin's count only, never on which chunk a point fell in, so
            // a point's sum stays independent of the order inside its bin.
            constexpr int HALF = kGatherThreads / 2;
            const bool split = kSplitRows<T> && cnt <= HALF;
            const bool upper = split && t >= HALF;
            const int mine = upper ? slot[t - HALF] : slot[t];
            constexpr int H1 = (W + 1) / 2;
            const int a_begin = upper ? H1 : 0, a_end = split && !upper ? H1 : W;
            T ax[FG], ay[FG];
#pragma unroll
            for (int f = 0; f < FG; ++f) ax[f] = ay[f] = (T)0;
            bool bad = true;
            int dst = 0;
            if (mine >= 0) {
            const PointRec<T> pr = recs[mine];
            dst = dsts[mine];
            bad = !(pr.vt == pr.vt) || !(pr.vp == pr.vp);
            const int lr = bad ? 0 : pr.it - r0;
            const int lc = bad ? 0 : pr.ip - c0;
            // step b reads column (b + rot) mod w; wp[b] is that column's weight
            const int rot = bad ? 0 : column_rotation(pr.it, pr.ip);
            const int last = rot ? 0 : W - 1;  // column of the final step
            T wp[W];
#pragma unroll
            for (int b = 0; b < W - 1; ++b) wp[b] = es_kernel<T>(((T)(b + rot - H) - pr.vp) * inv_hw, kc);
            wp[W - 1] = es_kernel<T>(((T)(last - H) - pr.vp) * inv_hw, kc);
            // rows stay a loop (two per iteration in FP64): unrolling it fully
            // lets the compiler hoist all w*w*FG LDS loads and run out of
            // registers
#pragma unroll RU
            for (int a = a_begin; a < a_end; ++a) {
                const T wt = es_kernel<T>(((T)(a - H) - pr.vt) * inv_hw, kc);
                const cplx<T> *row = tiles + (lr + a) * TCP + lc;
                const cplx<T> *rrow = row + rot;
                T rx[FG], ry[FG];
#pragma unroll
                for (int f = 0; f < FG; ++f) rx[f] = ry[f] = (T)0;
#pragma unroll
                for (int b = 0; b < W; ++b) {
#pragma unroll
                    for (int f = 0; f < FG; ++f) {
                        // fields past fg read stale LDS; their sums are never stored
                        const cplx<T> v = b < W - 1 ? rrow[f * plane + b] : row[f * plane + last];
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
            }
            if (split) {
                if (upper && mine >= 0) {
#pragma unroll
                    for (int f = 0; f < FG; ++f) {
                        xsum[(t - HALF) * 2 * FG + 2 * f] = ax[f];
                        xsum[(t - HALF) * 2 * FG + 2 * f + 1] = ay[f];
                    }
                }
                __syncthreads();
                if (!upper && mine >= 0) {
#pragma unroll
                    for (int f = 0; f < FG; ++f) {
                        ax[f] += xsum[t * 2 * FG + 2 * f];
                        ay[f] += xsum[t * 2 * FG + 2 * f + 1];
                    }
                }
            }
            if (mine < 0 || upper) continue;
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
__global__ __launch_bounds__(kGatherThreads) void k_gather(const cplx<T> *__restrict__ grid,
                                                           const PointRec<T> *__restrict__ rec,
                                                           const int32_t *__restrict__ perm,
                                                           const int32_t *__restrict__ binlist,
                                                           void *__restrict__ out, GatherParams gp)
{
    gather_body<T, W, FG>((int)blockIdx.x, grid, rec, perm, binlist, out, gp);
}

// Member j of a group class owns workgroups [j * per, (j + 1) * per); per is
// a multiple of 8, so a workgroup's XCD is the same as in a launch of its own.
template <typename T, int W, int FG>
__global__ __launch_bounds__(kGatherThreads) void k_gather_group(const GatherJob *__restrict__ jobs, int per)
{
    const int j = (int)blockIdx.x / per;
    const GatherJob J = jobs[j];
    gather_body<T, W, FG>((int)blockIdx.x - j * per, (const cplx<T> *)J.grid, (const PointRec<T> *)J.rec,
                          J.perm, J.binlist, J.out, J.gp);
}

// jobs == nullptr: one plan (the pointer arguments); otherwise n_members
// members of one group class described by jobs (device memory).
template <typename T, int W, int FG>
static hipError_t launch_wf(const GatherParams &gp, const void *grid, const void *rec,
                            const int32_t *perm, const int32_t *binlist, void *out, const GatherJob *jobs,
                            int n_members, hipStream_t s)
{
    const int pitch = sizeof(T) == 4 ? gp.tile_p + W - 1 : gp.tile_pitch;
    if (pitch < gp.tile_p + W - 1) return hipErrorInvalidValue;
    const size_t lds = sizeof(cplx<T>) * (size_t)(gp.tile_t + W - 1) * pitch * FG;
    const int per = (int)(8 * ((gp.nbins + 7) / 8));
    if (jobs) {
        auto kern = k_gather_group<T, W, FG>;
        if (lds > 65536)
            (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(kern, dim3((unsigned)(per * n_members)), dim3(kGatherThreads), lds, s, jobs, per);
    } else {
        auto kern = k_gather<T, W, FG>;
        if (lds > 65536)
            (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(kern, dim3((unsigned)per), dim3(kGatherThreads), lds, s, (const cplx<T> *)grid,
                           (const PointRec<T> *)rec, perm, binlist, out, gp);
    }
    return hipGetLastError();
}

template <typename T, int W>
static hipError_t launch_w(const GatherParams &gp, const void *grid, const void *rec, const int32_t *perm,
                           const int32_t *binlist, void *out, const GatherJob *jobs,
                           int n_members, hipStream_t s)
{
    switch (gp.fields_per_pass) {
    case 1: return launch_wf<T, W, 1>(gp, grid, rec, perm, binlist, out, jobs, n_members, s);
    case 2: return launch_wf<T, W, 2>(gp, grid, rec, perm, binlist, out, jobs, n_members, s);
    case 3: return launch_wf<T, W, 3>(gp, grid, rec, perm, binlist, out, jobs, n_members, s);
    case 4: return launch_wf<T, W, 4>(gp, grid, rec, perm, binlist, out, jobs, n_members, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
static hipError_t launch_t(const GatherParams &gp, const void *grid, const void *rec, const int32_t *perm,
                           const int32_t *binlist, void *out, const GatherJob *jobs,
                           int n_members, hipStream_t s)
{
    switch (gp.w) {
#define NUFFT2_W(X) case X: return launch_w<T, X>(gp, grid, rec, perm, binlist, out, jobs, n_members, s);
        NUFFT2_W(2) NUFFT2_W(3) NUFFT2_W(4) NUFFT2_W(5) NUFFT2_W(6) NUFFT2_W(7) NUFFT2_W(8)
        NUFFT2_W(9) NUFFT2_W(10) NUFFT2_W(11) NUFFT2_W(12) NUFFT2_W(13) NUFFT2_W(14)
        NUFFT2_W(15) NUFFT2_W(16)
#undef NUFFT2_W
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gather(int prec, const GatherParams &gp, const void *grid, const void *rec,
                         const int32_t *perm, const int32_t *binlist, void *out, hipStream_t s)
{
    if (gp.n_pts == 0) return hipSuccess;
    if (prec == 1) return launch_t<float>(gp, grid, rec, perm, binlist, out, nullptr, 0, s);
    return launch_t<double>(gp, grid, rec, perm, binlist, out, nullptr, 0, s);
}

// ---- vector rotation at the departure points (section 3, matrix Q) --------
//
// (u, v) interpolated at the departure point D, (east, north) components,
// expressed in the local frame of the arrival point A:
//   u' = p u + q v,  v' = -q u + p v,
//   p = (sin tA sin tD + (1 + cos tA cos tD) cos(pA - pD)) / (1 + cos eta),
//   q = (cos tA + cos tD) sin(pA - pD) / (1 + cos eta),
//   cos eta = sin tA sin tD cos(pA - pD) + cos tA cos tD  (= r_A . r_D).
// p and q in FP64 from the FP64 coordinates; u, v in place, in the caller's
// point order (complex: both parts; real output: the real values).
template <typename T>
__global__ __launch_bounds__(256) void k_rotate_uv(T *__restrict__ u, T *__restrict__ v, int comps, int64_t n,
                                                   const double *__restrict__ phi_a, const double *__restrict__ theta_a,
                                                   const double *__restrict__ phi_d, const double *__restrict__ theta_d)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double sa, ca, sd, cd, sp, cp;
    sincos(theta_a[j], &sa, &ca);
    sincos(theta_d[j], &sd, &cd);
    sincos(phi_a[j] - phi_d[j], &sp, &cp);
    const double den = 1.0 + (sa * sd * cp + ca * cd);
    const double p = (sa * sd + (1.0 + ca * cd) * cp) / den;
    const double q = (ca + cd) * sp / den;
    for (int c = 0; c < comps; ++c) {
        const double uu = (double)u[comps * j + c], vv = (double)v[comps * j + c];
        u[comps * j + c] = (T)(p * uu + q * vv);
        v[comps * j + c] = (T)(-q * uu + p * vv);
    }
}

hipError_t launch_rotate_uv(int prec, void *u, void *v, int comps, int64_t n, const double *phi_a,
                            const double *theta_a, const double *phi_d, const double *theta_d, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (prec == 1)
        hipLaunchKernelGGL(k_rotate_uv<float>, dim3(blocks), dim3(256), 0, s, (float *)u, (float *)v, comps, n,
                           phi_a, theta_a, phi_d, theta_d);
    else
        hipLaunchKernelGGL(k_rotate_uv<double>, dim3(blocks), dim3(256), 0, s, (double *)u, (double *)v, comps, n,
                           phi_a, theta_a, phi_d, theta_d);
    return hipGetLastError();
}

hipError_t launch_gather_group(int prec, const GatherParams &gp, const GatherJob *jobs, int n_members,
                               hipStream_t s)
{
    if (n_members < 1 || !jobs) return hipErrorInvalidValue;
    if (prec == 1) return launch_t<float>(gp, nullptr, nullptr, nullptr, nullptr, nullptr, jobs, n_members, s);
    return launch_t<double>(gp, nullptr, nullptr, nullptr, nullptr, nullptr, jobs, n_members, s);
}

}  // namespace nufft2
