// Point setup: wrap each departure point onto the periodic fine grid in FP64,
// split it into a first-tap cell and an offset, and counting-sort the points
// by gather tile ("bin").
//
// Pipeline (all on the plan's stream):
//   k_setpts_bin       per point: wrap/split, bin id, count the point in
//                      its bin (one atomic per bin and wave), mark the
//                      first-tap theta row
//   k_bin_scan         one workgroup: exclusive scan of the bin counts, the
//                      list of non-empty bins, the set of theta rows any
//                      point's taps reach; clears the marks for the next call
//   k_setpts_scatter   per point: recompute the split and the bin, take a
//                      rank in the bin by decrementing its count (one atomic
//                      per bin and wave), write the packed record at
//                      binstart[bin] + rank and the permutation; the
//                      decrements leave every count at zero for the next call
// For small plans (bins in one scan pass, points in one wave of 1024-thread
// workgroups) k_setpts_scatter_scan replaces the last two: each workgroup
// scans the counts itself (see there), so its points' ranks come from the
// bin kernel instead (written per point, and cleared counts by a ticket).
// Plans of several scan passes run the passes side by side
// (k_bin_scan_passes, k_setpts_scatter_passes).
//
// The order of points inside a bin depends on atomic arbitration; the output
// of an exec does not, because each point's sum is computed by one thread in a
// fixed tap order from the same grid values wherever it sits in its bin.
#include "nufft2_internal.hpp"

namespace nufft2 {

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
    t = t - nf * floor(t * ax.inv_nf);  // 1 / nf is exact: no division
    if (t >= nf) t -= nf;             // t slightly below 0 rounds up to nf
    const double c = ceil(t - 0.5 * (double)w);
    const double u = t - c;
    int32_t i0 = (int32_t)c;
    i0 &= (ax.nf - 1);                // c >= -w/2 > -nf: masking is the positive modulus
    i0m = i0;
    v = (T)(u - (double)(w >> 1));
}

// Lanes of a wave that share a bin are grouped with ballots (no memory
// traffic): the group's leader lane, this lane's place in its group, and on
// the leader the group's size (0 elsewhere).  Departure points arrive in
// grid order, so a wave touches only a few bins.
struct WaveGroup {
    int leader;
    int32_t offset, count;
};
__device__ inline WaveGroup wave_group(int32_t bin)
{
    const int lane = (int)__lane_id();
    uint64_t pending = __ballot(1);
    WaveGroup g{lane, 0, 0};
    while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int32_t lbin = __shfl(bin, leader, 64);
        const uint64_t grp = pending & __ballot(bin == lbin);
        if ((grp >> lane) & 1ull) {
            g.leader = leader;
            g.offset = (int32_t)__popcll(grp & ((1ull << lane) - 1ull));
        }
        if (lane == leader) g.count = (int32_t)__popcll(grp);
        pending &= ~grp;
    }
    return g;
}

// Rank of this lane's point among the points of its bin: every group leader
// adds its group's size with one atomic, all leaders in the same
// instruction, so the wave pays one atomic round trip.
__device__ inline int32_t wave_aggregated_rank(int32_t *__restrict__ bincount, int32_t bin)
{
    const WaveGroup g = wave_group(bin);
    int32_t base = 0;
    if (g.count > 0) base = atomicAdd(&bincount[bin], g.count);
    return __shfl(base, g.leader, 64) + g.offset;
}

// Counting only (the rank is not needed).
__device__ inline void wave_aggregated_count(int32_t *__restrict__ bincount, int32_t bin)
{
    const WaveGroup g = wave_group(bin);
    if (g.count > 0) atomicAdd(&bincount[bin], g.count);
}

// The same grouping, taking ranks from the top: every group leader
// subtracts its group's size from the bin's count; the ranks of the group
// are the old count minus the size, plus the lane's place in the group.
// Once every point of a bin has taken its rank the count is zero again.
__device__ inline int32_t wave_aggregated_rank_down(int32_t *__restrict__ bincount, int32_t bin)
{
    const WaveGroup g = wave_group(bin);
    int32_t base = 0;
    if (g.count > 0) base = atomicSub(&bincount[bin], g.count) - g.count;
    return __shfl(base, g.leader, 64) + g.offset;
}

// Bin of a first-tap cell: tiles are powers of two and the cell indices
// non-negative, so the quotients are shifts (the tile is uniform, its
// exponent a scalar).
__device__ inline int32_t bin_of(int32_t it, int32_t ip, const SetptsParams &sp)
{
    return (int32_t)((uint32_t)it >> __builtin_ctz((unsigned)sp.th.tile)) * sp.nbins_phi +
           (int32_t)((uint32_t)ip >> __builtin_ctz((unsigned)sp.ph.tile));
}

// Wrap/split of one point and its bin (non-finite coordinates: bin 0 and a
// NaN record).
template <typename T>
__device__ inline int32_t split_point(double ph, double th, const SetptsParams &sp, PointRec<T> &r)
{
    if (!isfinite(ph) || !isfinite(th)) {
        r.it = 0;
        r.ip = 0;
        r.vt = (T)NAN;
        r.vp = (T)NAN;
        return 0;
    }
    split_axis<T>(th, sp.th, sp.w, r.it, r.vt);
    split_axis<T>(ph, sp.ph, sp.w, r.ip, r.vp);
    return bin_of(r.it, r.ip, sp);
}

// The pair (p, q) of the matrix Q that takes a vector at departure point D
// to the local frame of arrival point A (section 3, after the semi-implicit
// forcing equations):
//   p = (sin tA sin tD + (1 + cos tA cos tD) cos(pA - pD)) / (1 + cos eta),
//   q = (cos tA + cos tD) sin(pA - pD) / (1 + cos eta),
//   cos eta = sin tA sin tD cos(pA - pD) + cos tA cos tD.
// FP64 plans evaluate it in FP64.  FP32 plans reduce the angles in FP64 and
// evaluate the trigonometric functions in FP32 (about 1e-7 relative in p
// and q, an order below the plan's tolerance).  Undefined for antipodal
// pairs (cos eta = -1).
__device__ inline void rotation_pair(double pa, double ta, double pd, double td, double *out)
{
    double sa, ca, sd, cd, sp, cp;
    sincos(ta, &sa, &ca);
    sincos(td, &sd, &cd);
    sincos(pa - pd, &sp, &cp);
    const double den = 1.0 + (sa * sd * cp + ca * cd);
    out[0] = (sa * sd + (1.0 + ca * cd) * cp) / den;
    out[1] = (ca + cd) * sp / den;
}
__device__ inline void rotation_pair(double pa, double ta, double pd, double td, float *out)
{
    const double two_pi = 6.283185307179586476925286766559;
    auto reduce = [&](double x) { return (float)(x - two_pi * rint(x * (1.0 / two_pi))); };
    float sa, ca, sd, cd, sp, cp;
    sincosf(reduce(ta), &sa, &ca);
    sincosf(reduce(td), &sd, &cd);
    sincosf(reduce(pa - pd), &sp, &cp);
    const float den = 1.0f + (sa * sd * cp + ca * cd);
    out[0] = (sa * sd + (1.0f + ca * cd) * cp) / den;
    out[1] = (ca + cd) * sp / den;
}

// Point j with coordinates (ph, th) (a thread of a 256-thread block; the
// caller skips j >= n).  KR: also write the point's (bin, rank) for the
// fused scan + scatter.
template <typename T, bool KR>
__device__ inline void setpts_bin_point(int64_t j, double ph, double th, const SetptsParams &sp,
                                        int32_t *__restrict__ bincount, int2 *__restrict__ keyrank,
                                        uint8_t *__restrict__ rowmark, int32_t *__restrict__ flags)
{
    int32_t bin;
    if (!isfinite(ph) || !isfinite(th)) {
        atomicOr(&flags[0], 1);
        bin = 0;
    } else {
        int32_t it, ip;
        T vt, vp;
        split_axis<T>(th, sp.th, sp.w, it, vt);
        split_axis<T>(ph, sp.ph, sp.w, ip, vp);
        bin = bin_of(it, ip, sp);
        rowmark[it] = 1;
    }
    if (KR) keyrank[j] = make_int2(bin, wave_aggregated_rank(bincount, bin));
    else wave_aggregated_count(bincount, bin);
}

// Points per thread (PPT) of the bin and scatter kernels of a single plan:
// a thread's points (256 apart, so that each wave still takes consecutive
// points) are loaded together, which keeps several loads in flight per
// thread.  Four per thread from kManyPoints points on (2048+ workgroups);
// below that one, so that smaller plans still spread over every CU.
constexpr int kSetptsThreads = 256;
constexpr int64_t kManyPoints = int64_t(1) << 21;

template <typename T, bool KR, int PPT>
__global__ __launch_bounds__(kSetptsThreads) void k_setpts_bin(const double *__restrict__ phi,
                                                               const double *__restrict__ theta, SetptsParams sp,
                                                               int32_t *__restrict__ bincount,
                                                               int2 *__restrict__ keyrank,
                                                               uint8_t *__restrict__ rowmark,
                                                               int32_t *__restrict__ flags)
{
    const int64_t j0 = (int64_t)blockIdx.x * (PPT * kSetptsThreads) + threadIdx.x;
    double ph[PPT], th[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int64_t j = j0 + q * kSetptsThreads;
        ph[q] = j < sp.n ? phi[j] : 0.0;
        th[q] = j < sp.n ? theta[j] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int64_t j = j0 + q * kSetptsThreads;
        if (j < sp.n) setpts_bin_point<T, KR>(j, ph[q], th[q], sp, bincount, keyrank, rowmark, flags);
    }
}

// Group launches: job_of_block[b] is the member that owns point block b;
// the member's points start at block jobs[j].block_begin.
template <typename T>
__global__ __launch_bounds__(256) void k_setpts_bin_group(const SetptsJob *__restrict__ jobs,
                                                          const int32_t *__restrict__ job_of_block)
{
    const SetptsJob J = jobs[job_of_block[blockIdx.x]];
    const int64_t j = (int64_t)((int)blockIdx.x - J.block_begin) * blockDim.x + threadIdx.x;
    if (j < J.sp.n) setpts_bin_point<T, false>(j, J.phi[j], J.theta[j], J.sp, J.bincount, J.keyrank, J.rowmark, J.flags);
}

// Block-wide exclusive scans of two ints per thread at once (one set of
// barriers for both; blockDim.x a multiple of 64, at most 32 waves).
// Returns the exclusive prefixes in x, y and the block totals in tx, ty.
__device__ inline void block_exclusive_scan2(int &x, int &y, int (*lds)[33], int &tx, int &ty)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    int ix = x, iy = y;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int ux = __shfl_up(ix, d, 64), uy = __shfl_up(iy, d, 64);
        if (lane >= d) {
            ix += ux;
            iy += uy;
        }
    }
    if (lane == 63) {
        lds[0][wid] = ix;
        lds[1][wid] = iy;
    }
    __syncthreads();
    if (wid == 0) {
        const int vx = lane < nwaves ? lds[0][lane] : 0, vy = lane < nwaves ? lds[1][lane] : 0;
        int wx = vx, wy = vy;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int ux = __shfl_up(wx, d, 64), uy = __shfl_up(wy, d, 64);
            if (lane >= d) {
                wx += ux;
                wy += uy;
            }
        }
        if (lane < nwaves) {
            lds[0][lane] = wx - vx;
            lds[1][lane] = wy - vy;
        }
        if (lane == nwaves - 1) {
            lds[0][32] = wx;
            lds[1][32] = wy;
        }
    }
    __syncthreads();
    x = ix - x + lds[0][wid];
    y = iy - y + lds[1][wid];
    tx = lds[0][32];
    ty = lds[1][32];
    __syncthreads();
}

// One workgroup of 1024 threads.  Each pass stages CHUNK * 1024 bin counts
// in LDS with coalesced loads, every thread scans CHUNK consecutive counts,
// and the starts go back out through LDS with coalesced stores.  binstart
// gets nbins + 1 entries (the last is the number of points); binlist gets the
// non-empty bins in increasing order and their number in entry nbins.  The kernel
// also leaves the counters, the row marks and the non-finite accumulator
// cleared for the next setpts, and publishes the non-finite flag in flags[1].
constexpr int kScanThreads = 1024;
constexpr int kScanChunk = 8;
// one padding slot after every kScanChunk counts keeps a thread's chunk in
// its own LDS banks
__device__ constexpr int scan_slot(int e) { return e + e / kScanChunk; }

// Compacted entries of a pass: three arrays (bin, first record, count) of
// kCmpLen ints; one padding slot every 32 entries, because the threads of a
// wave write entries kScanChunk apart (without it they would share 4 of the
// 32 banks).
constexpr int kCmpLen = kScanChunk * kScanThreads + kScanChunk * kScanThreads / 32;
__device__ constexpr int cmp_slot(int e) { return e + e / 32; }
static_assert(kDealtMaxBins == kScanChunk * kScanThreads, "the per-slot table needs all entries of one pass");

// One pass over PASS = CHUNK * 1024 bins starting at base (n of them):
// in[k] is this thread's count of bin base + k * 1024 + threadIdx.x (zero
// past the end).  Stages them in LDS, scans CHUNK consecutive counts per
// thread, and writes the starts (coalesced).  The pass's non-empty bins are
// compacted in LDS (cmp: bin, first record, count) and written out by
// consecutive threads: written from the scanning threads directly, each
// store instruction would touch 64 cache lines (CHUNK entries apart), which
// made the pass several times slower where most bins hold points.
__device__ __attribute__((always_inline)) inline void scan_pass(const int (&in)[kScanChunk], int64_t base, int n,
                                                              int *stage, int *cmp, int (*lds)[33], int &carry,
                                                              int &carry_ne, int32_t *__restrict__ binstart,
                                                              int32_t *__restrict__ binlist,
                                                              int4 *__restrict__ items, bool write_out = true)
{
#pragma unroll
    for (int k = 0; k < kScanChunk; ++k) stage[scan_slot(k * kScanThreads + (int)threadIdx.x)] = in[k];
    __syncthreads();
    int vals[kScanChunk];
    int sum = 0, ne = 0;
#pragma unroll
    for (int c = 0; c < kScanChunk; ++c) {
        vals[c] = stage[scan_slot((int)threadIdx.x * kScanChunk + c)];
        sum += vals[c];
        ne += vals[c] > 0 ? 1 : 0;
    }
    int total, ne_total;
    int run = sum, pos = ne;
    block_exclusive_scan2(run, pos, lds, total, ne_total);
    run += carry;
    const int first = (int)base + (int)threadIdx.x * kScanChunk;
#pragma unroll
    for (int c = 0; c < kScanChunk; ++c) {
        stage[scan_slot((int)threadIdx.x * kScanChunk + c)] = run;
        if (vals[c] > 0) {
            const int q = cmp_slot(pos);
            cmp[q] = first + c;
            cmp[kCmpLen + q] = run;
            cmp[2 * kCmpLen + q] = vals[c];
            ++pos;
        }
        run += vals[c];
    }
    __syncthreads();
    if (write_out) {
        for (int e = threadIdx.x; e < n; e += kScanThreads) binstart[base + e] = stage[scan_slot(e)];
        for (int e = threadIdx.x; e < ne_total; e += kScanThreads) {
            const int q = cmp_slot(e);
            const int b = cmp[q], s0 = cmp[kCmpLen + q], c0 = cmp[2 * kCmpLen + q];
            if (binlist) binlist[carry_ne + e] = b;
            items[carry_ne + e] = make_int4(b, s0, c0, 0);
        }
    }
    __syncthreads();
    carry += total;
    carry_ne += ne_total;
}

// The reached theta rows from this thread's row marks mk (rows t + i * 1024):
// row l is read by the gather iff some point's first tap row is within
// w - 1 rows below it (cyclically).  The marks go through LDS (marks, nft
// bytes) so the w-wide window reads hit LDS, not global memory.  Also
// publishes the non-finite flag (flag0: flags[0] as thread 0 read it) in
// flags[1] and clears the marks and flags[0] for the next call.
constexpr int kMaxRowsPerScanThread = 4;  // nf <= 4096
__device__ __attribute__((always_inline)) inline void reached_rows(const uint8_t (&mk)[kMaxRowsPerScanThread],
                                                                 int flag0, uint8_t *marks,
                                                                 uint8_t *__restrict__ rowmark,
                                                                 uint8_t *__restrict__ rowtouched, int nft, int w,
                                                                 int32_t *__restrict__ flags)
{
    const int t = (int)threadIdx.x;
    if (t == 0) {
        flags[1] = flag0;
        flags[0] = 0;
    }
#pragma unroll
    for (int i = 0; i < kMaxRowsPerScanThread; ++i) {
        const int l = t + i * kScanThreads;
        if (l < nft) {
            marks[l] = mk[i];
            rowmark[l] = 0;
        }
    }
    __syncthreads();
    for (int l = t; l < nft; l += kScanThreads) {
        uint8_t v = 0;
        for (int a = 0; a < w; ++a) v |= marks[(l - a + nft) & (nft - 1)];
        rowtouched[l] = v;
    }
}

// The gather's table of entries per workgroup (see bin_dealt) for a plan of
// at most kDealtMaxBins bins, written by the scanning workgroup after its
// single pass, from the n_ne entries that pass left compacted in cmp.
__device__ __attribute__((always_inline)) inline void write_dealt(int4 *__restrict__ dealt, int64_t nbins, int n_ne,
                                                                const int *cmp)
{
    const int per = (n_ne + 7) >> 3;
    const int slots = (int)gather_slots(nbins);
    for (int blk = threadIdx.x; blk < slots; blk += kScanThreads) {
        const int k = blk >> 3, item = (blk & 7) * per + k;
        int4 v = make_int4(0, 0, 0, 0);
        if (k < per && item < n_ne) {
            const int q = cmp_slot(item);
            v = make_int4(cmp[q], cmp[kCmpLen + q], cmp[2 * kCmpLen + q], 0);
        }
        dealt[blk] = v;
    }
}

// Passes whose counts are all loaded before the first scan (nbins up to
// kScanHoist * PASS): the kernel then waits on global memory once.
constexpr int kScanHoist = 4;

__device__ __attribute__((always_inline)) inline void bin_scan_body(int32_t *__restrict__ bincount, int32_t *__restrict__ binstart,
                                     int32_t *__restrict__ binlist, int64_t nbins, uint8_t *__restrict__ rowmark,
                                     uint8_t *__restrict__ rowtouched, int nft, int w,
                                     int32_t *__restrict__ flags)
{
    __shared__ int lds[2][33];
    __shared__ int stage[kScanChunk * kScanThreads + kScanThreads];
    __shared__ int cmp[3 * kCmpLen];  // compacted non-empty bins of a pass
    constexpr int PASS = kScanChunk * kScanThreads;
    const int t = (int)threadIdx.x;
    // the row marks and the non-finite accumulator are read with the counts
    uint8_t mk[kMaxRowsPerScanThread];
#pragma unroll
    for (int i = 0; i < kMaxRowsPerScanThread; ++i) {
        const int l = t + i * kScanThreads;
        mk[i] = l < nft ? rowmark[l] : (uint8_t)0;
    }
    const int flag0 = t == 0 ? flags[0] : 0;
    int4 *items = bin_items(binlist, nbins);
    int carry = 0, carry_ne = 0;
    if (nbins <= (int64_t)kScanHoist * PASS) {
        int h[kScanHoist][kScanChunk];
#pragma unroll
        for (int p = 0; p < kScanHoist; ++p)
#pragma unroll
            for (int k = 0; k < kScanChunk; ++k) {
                const int64_t e = (int64_t)p * PASS + k * kScanThreads + t;
                h[p][k] = e < nbins ? bincount[e] : 0;
            }
#pragma unroll
        for (int p = 0; p < kScanHoist; ++p) {
            const int64_t base = (int64_t)p * PASS;
            if (base < nbins)
                scan_pass(h[p], base, (int)((nbins - base) < PASS ? (nbins - base) : PASS), stage, cmp, lds,
                          carry, carry_ne, binstart, binlist, items);
        }
    } else {
        for (int64_t base = 0; base < nbins; base += PASS) {
            int h[kScanChunk];
#pragma unroll
            for (int k = 0; k < kScanChunk; ++k) {
                const int64_t e = base + k * kScanThreads + t;
                h[k] = e < nbins ? bincount[e] : 0;
            }
            scan_pass(h, base, (int)((nbins - base) < PASS ? (nbins - base) : PASS), stage, cmp, lds, carry,
                      carry_ne, binstart, binlist, items);
        }
    }
    if (t == 0) {
        binstart[nbins] = carry;
        binlist[nbins] = carry_ne;
    }
    if (nbins <= kDealtMaxBins) write_dealt(bin_dealt(binlist, nbins), nbins, carry_ne, cmp);
    reached_rows(mk, flag0, reinterpret_cast<uint8_t *>(stage), rowmark, rowtouched, nft, w, flags);
}

__global__ __launch_bounds__(kScanThreads) void k_bin_scan(int32_t *__restrict__ bincount,
                                                           int32_t *__restrict__ binstart,
                                                           int32_t *__restrict__ binlist,
                                                           int64_t nbins,
                                                           uint8_t *__restrict__ rowmark,
                                                           uint8_t *__restrict__ rowtouched,
                                                           int nft, int w,
                                                           int32_t *__restrict__ flags)
{
    bin_scan_body(bincount, binstart, binlist, nbins, rowmark, rowtouched, nft, w, flags);
}

// Group launch: one workgroup per member.
__global__ __launch_bounds__(kScanThreads) void k_bin_scan_group(const SetptsJob *__restrict__ jobs)
{
    const SetptsJob J = jobs[blockIdx.x];
    bin_scan_body(J.bincount, J.binstart, J.binlist, J.nbins, J.rowmark, J.rowtouched, J.sp.th.nf, J.sp.w,
                  J.flags);
}

template <typename T>
__device__ inline void setpts_scatter_point(int64_t j, const double *__restrict__ phi,
                                            const double *__restrict__ theta, const SetptsParams &sp,
                                            int32_t *__restrict__ bincount, const int32_t *__restrict__ binstart,
                                            PointRec<T> *__restrict__ rec, int32_t *__restrict__ perm)
{
    if (j < sp.n) {
        PointRec<T> r;
        const int32_t bin = split_point<T>(phi[j], theta[j], sp, r);
        const int32_t pos = binstart[bin] + wave_aggregated_rank_down(bincount, bin);
        rec[pos] = r;
        perm[pos] = (int32_t)j;
    }
}

// PPT points of one thread (j0, j0 + 256, ...; coordinates
// already loaded): every point's split and lane grouping first, then all
// their count decrements, so that the atomics' round trips overlap; each
// point then goes to start(bin) + its rank.
// ROT (the vector rotation, sp.pq): each point's (p, q) pair goes to
// pq[pos] as well, from its arrival point.
template <typename T, bool ROT, int PPT, class Start>
__device__ inline void setpts_scatter_points(int64_t j0, const double (&ph)[PPT],
                                             const double (&th)[PPT], const SetptsParams &sp,
                                             int32_t *__restrict__ bincount, const Start &start,
                                             PointRec<T> *__restrict__ rec, int32_t *__restrict__ perm)
{
    double pa[PPT], ta[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int64_t j = j0 + q * kSetptsThreads;
        const bool load = ROT && j < sp.n;
        pa[q] = load ? sp.phi_a[j] : 0.0;
        ta[q] = load ? sp.theta_a[j] : 0.0;
    }
    PointRec<T> r[PPT];
    int32_t bin[PPT], base[PPT];
    WaveGroup g[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        bin[q] = 0;
        base[q] = 0;
        g[q] = WaveGroup{0, 0, 0};
        if (j0 + q * kSetptsThreads < sp.n) {
            bin[q] = split_point<T>(ph[q], th[q], sp, r[q]);
            g[q] = wave_group(bin[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < PPT; ++q)
        if (j0 + q * kSetptsThreads < sp.n && g[q].count > 0)
            base[q] = atomicSub(&bincount[bin[q]], g[q].count) - g[q].count;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int64_t j = j0 + q * kSetptsThreads;
        if (j < sp.n) {
            const int32_t pos = start(bin[q]) + __shfl(base[q], g[q].leader, 64) + g[q].offset;
            rec[pos] = r[q];
            perm[pos] = (int32_t)j;
            if (ROT) rotation_pair(pa[q], ta[q], ph[q], th[q], reinterpret_cast<T *>(sp.pq) + 2 * (int64_t)pos);
        }
    }
}

// Above kDealtMaxBins bins the gather's per-slot table (see bin_dealt) is
// written here, by the scatter's threads (thread i of n: slots i, i + n,
// ...), from the entries the scan published: one workgroup could not write
// it fast enough.
__device__ inline void scatter_dealt(int64_t i, int64_t n, int32_t *__restrict__ binlist, int64_t nbins)
{
    if (nbins <= kDealtMaxBins) return;
    const int n_ne = binlist[nbins];
    const int per = (n_ne + 7) >> 3;
    const int4 *items = bin_items(binlist, nbins);
    int4 *dealt = bin_dealt(binlist, nbins);
    const int64_t slots = gather_slots(nbins);
    for (int64_t blk = i; blk < slots; blk += n) {
        const int k = (int)(blk >> 3), item = (int)(blk & 7) * per + k;
        dealt[blk] = (k < per && item < n_ne) ? items[item] : make_int4(0, 0, 0, 0);
    }
}

template <typename T, bool ROT, int PPT>
__global__ __launch_bounds__(kSetptsThreads) void k_setpts_scatter(const double *__restrict__ phi,
                                                                   const double *__restrict__ theta,
                                                                   SetptsParams sp,
                                                                   int32_t *__restrict__ bincount,
                                                                   const int32_t *__restrict__ binstart,
                                                                   PointRec<T> *__restrict__ rec,
                                                                   int32_t *__restrict__ perm,
                                                                   int32_t *__restrict__ binlist, int64_t nbins)
{
    const int64_t j0 = (int64_t)blockIdx.x * (PPT * kSetptsThreads) + threadIdx.x;
    double ph[PPT], th[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int64_t j = j0 + q * kSetptsThreads;
        ph[q] = j < sp.n ? phi[j] : 0.0;
        th[q] = j < sp.n ? theta[j] : 0.0;
    }
    setpts_scatter_points<T, ROT, PPT>(j0, ph, th, sp, bincount, [&](int32_t b) { return binstart[b]; }, rec, perm);
    scatter_dealt((int64_t)blockIdx.x * blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x, binlist, nbins);
}

template <typename T>
__global__ __launch_bounds__(256) void k_setpts_scatter_group(const SetptsJob *__restrict__ jobs,
                                                              const int32_t *__restrict__ job_of_block)
{
    const SetptsJob J = jobs[job_of_block[blockIdx.x]];
    const int64_t i = (int64_t)((int)blockIdx.x - J.block_begin) * blockDim.x + threadIdx.x;
    setpts_scatter_point<T>(i, J.phi, J.theta, J.sp, J.bincount, J.binstart, (PointRec<T> *)J.rec, J.perm);
    const int64_t member_threads = (J.sp.n + blockDim.x - 1) / blockDim.x * blockDim.x;
    scatter_dealt(i, member_threads, J.binlist, J.nbins);
}

// Scatter with the bin scan folded in, for plans whose bins fit one scan pass
// and whose points fit one wave of workgroups (kFusedMaxBlocks of 1024
// threads): every workgroup scans all bin counts in LDS (the same pass as
// k_bin_scan) and places its own points from those starts; workgroup 0 also
// writes the starts, the non-empty bin list and its entries, workgroup
// min(1, grid - 1) the reached rows and the non-finite flag, and the last
// workgroup to finish clears the counters for the next call.  A workgroup
// takes its ticket (flags[2]) after its counts went through its scan, so
// the last one clears them after every read.  One launch boundary and one
// single-workgroup kernel fewer than bin count -> scan -> scatter.
constexpr int kFusedMaxBlocks = 256;

template <typename T, bool ROT>
__global__ __launch_bounds__(kScanThreads) void k_setpts_scatter_scan(
    const double *__restrict__ phi, const double *__restrict__ theta, SetptsParams sp,
    int32_t *__restrict__ bincount, int32_t *__restrict__ binstart, int32_t *__restrict__ binlist, int nbins,
    const int2 *__restrict__ keyrank, uint8_t *__restrict__ rowmark, uint8_t *__restrict__ rowtouched, int nft,
    int32_t *__restrict__ flags, PointRec<T> *__restrict__ rec, int32_t *__restrict__ perm)
{
    __shared__ int lds[2][33];
    __shared__ int stage[kScanChunk * kScanThreads + kScanThreads];
    __shared__ int cmp[3 * kCmpLen];
    __shared__ int last;
    const int t = (int)threadIdx.x;
    const int64_t j = (int64_t)blockIdx.x * kScanThreads + t;
    const bool out_wg = blockIdx.x == 0;
    const bool rows_wg = (int)blockIdx.x == (gridDim.x > 1 ? 1 : 0);
    // every load of the workgroup first: its points, all counts, the marks
    double ph = 0.0, th = 0.0;
    int2 kr = make_int2(0, 0);
    if (j < sp.n) {
        ph = phi[j];
        th = theta[j];
        kr = keyrank[j];
    }
    int h[kScanChunk];
#pragma unroll
    for (int k = 0; k < kScanChunk; ++k) {
        const int e = k * kScanThreads + t;
        h[k] = e < nbins ? bincount[e] : 0;
    }
    uint8_t mk[kMaxRowsPerScanThread];
    int flag0 = 0;
#pragma unroll
    for (int i = 0; i < kMaxRowsPerScanThread; ++i) {
        const int l = t + i * kScanThreads;
        mk[i] = rows_wg && l < nft ? rowmark[l] : (uint8_t)0;
    }
    if (rows_wg && t == 0) flag0 = flags[0];
    int4 *items = bin_items(binlist, nbins);
    int carry = 0, carry_ne = 0;
    scan_pass(h, 0, nbins, stage, cmp, lds, carry, carry_ne, binstart, binlist, items, out_wg);
    // stage[scan_slot(b)] now holds the first record of bin b
    if (out_wg) {
        if (t == 0) {
            binstart[nbins] = carry;
            binlist[nbins] = carry_ne;
        }
        write_dealt(bin_dealt(binlist, nbins), nbins, carry_ne, cmp);
    }
    // the ticket goes out now (the scan has consumed every count this
    // workgroup read); its answer is needed only at the end
    int ticket = 0;
    if (t == 0) ticket = atomicAdd(&flags[2], 1);
    if (j < sp.n) {
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
        const int32_t pos = stage[scan_slot(kr.x)] + kr.y;
        rec[pos] = r;
        perm[pos] = (int32_t)j;
        if (ROT) rotation_pair(sp.phi_a[j], sp.theta_a[j], ph, th, reinterpret_cast<T *>(sp.pq) + 2 * (int64_t)pos);
    }
    if (rows_wg) {
        // with one workgroup it also wrote the per-slot table from cmp above
        if (out_wg) __syncthreads();
        reached_rows(mk, flag0, reinterpret_cast<uint8_t *>(cmp), rowmark, rowtouched, nft, sp.w, flags);
    }
    if (t == 0) last = ticket == (int)gridDim.x - 1;
    __syncthreads();
    if (last) {
        for (int e = t; e < nbins; e += kScanThreads) bincount[e] = 0;
        if (t == 0) flags[2] = 0;
    }
}

// Plans with more bins than one scan pass: the passes run side by side, one
// workgroup each (k_bin_scan_passes), instead of one after another in one
// workgroup.  Pass workgroup b scans its bins into pass-local starts
// (lstart; the counts stay for the scatter's ranks), writes its non-empty
// entries with pass-local first records to stage[b * PASS + i], and its
// totals {points, non-empty bins} to passtot[b]; workgroup 0 also derives
// the reached rows and publishes the non-finite flag.  The scatter
// (k_setpts_scatter_passes) then adds the prefix of the pass totals: it
// places the points, writes the global starts, the bin list, its entries and
// the gather's table.
constexpr int kScanPass = kScanChunk * kScanThreads;
constexpr int kMaxScanPasses = 128;  // nbins <= 2^20
static_assert(kMaxScanPasses <= 2 * 64, "the scatter scans the pass totals in its first two waves");

__global__ __launch_bounds__(kScanThreads) void k_bin_scan_passes(int32_t *__restrict__ bincount, int64_t nbins,
                                                                  int32_t *__restrict__ lstart,
                                                                  int4 *__restrict__ stage, int2 *__restrict__ passtot,
                                                                  uint8_t *__restrict__ rowmark,
                                                                  uint8_t *__restrict__ rowtouched, int nft, int w,
                                                                  int32_t *__restrict__ flags)
{
    __shared__ int lds[2][33];
    __shared__ int stg[kScanChunk * kScanThreads + kScanThreads];
    __shared__ int cmp[3 * kCmpLen];
    const int t = (int)threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kScanPass;
    const int n = (int)((nbins - base) < kScanPass ? (nbins - base) : kScanPass);
    const bool rows_wg = blockIdx.x == 0;
    int h[kScanChunk];
#pragma unroll
    for (int k = 0; k < kScanChunk; ++k) {
        const int e = k * kScanThreads + t;
        h[k] = e < n ? bincount[base + e] : 0;
    }
    uint8_t mk[kMaxRowsPerScanThread];
#pragma unroll
    for (int i = 0; i < kMaxRowsPerScanThread; ++i) {
        const int l = t + i * kScanThreads;
        mk[i] = rows_wg && l < nft ? rowmark[l] : (uint8_t)0;
    }
    const int flag0 = rows_wg && t == 0 ? flags[0] : 0;
    int carry = 0, carry_ne = 0;
    // pass-local starts; entries to this pass's stage region
    scan_pass(h, base, n, stg, cmp, lds, carry, carry_ne, lstart, nullptr, stage + base);
    if (t == 0) passtot[blockIdx.x] = make_int2(carry, carry_ne);
    if (rows_wg) reached_rows(mk, flag0, reinterpret_cast<uint8_t *>(stg), rowmark, rowtouched, nft, w, flags);
}

template <typename T, bool ROT, int PPT>
__global__ __launch_bounds__(kSetptsThreads) void k_setpts_scatter_passes(
    const double *__restrict__ phi, const double *__restrict__ theta, SetptsParams sp,
    int32_t *__restrict__ bincount, const int32_t *__restrict__ lstart, const int4 *__restrict__ stage,
    const int2 *__restrict__ passtot, int npass, int32_t *__restrict__ binstart, int32_t *__restrict__ binlist,
    int64_t nbins, PointRec<T> *__restrict__ rec, int32_t *__restrict__ perm)
{
    __shared__ int2 pre[kMaxScanPasses + 1];  // exclusive prefix of the pass totals
    __shared__ int2 half0;                    // totals of passes 0..63
    const int t = (int)threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.x * (PPT * kSetptsThreads) + t;
    double ph[PPT], th[PPT];
    int2 inc = t < npass ? passtot[t] : make_int2(0, 0);
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int64_t j = j0 + q * kSetptsThreads;
        ph[q] = j < sp.n ? phi[j] : 0.0;
        th[q] = j < sp.n ? theta[j] : 0.0;
    }
    // pass b's totals on thread b: inclusive scan in each of the first two
    // waves, then the second adds the first's total
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int yx = __shfl_up(inc.x, d, 64), yy = __shfl_up(inc.y, d, 64);
        if ((t & 63) >= d) {
            inc.x += yx;
            inc.y += yy;
        }
    }
    if (t == 63) half0 = inc;
    __syncthreads();
    if (t < kMaxScanPasses) {
        if (t >= 64) {
            inc.x += half0.x;
            inc.y += half0.y;
        }
        pre[t + 1] = inc;
        if (t == 0) pre[0] = make_int2(0, 0);
    }
    __syncthreads();
    setpts_scatter_points<T, ROT, PPT>(j0, ph, th, sp, bincount,
                             [&](int32_t b) { return lstart[b] + pre[b / kScanPass].x; }, rec, perm);
    // the tables, grid-stride over bins, entries and gather slots
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + t, gstride = (int64_t)gridDim.x * blockDim.x;
    const int n_ne = pre[npass].y;
    int4 *items = bin_items(binlist, nbins);
    int4 *dealt = bin_dealt(binlist, nbins);
    for (int64_t i = gid; i < nbins; i += gstride) binstart[i] = lstart[i] + pre[i / kScanPass].x;
    // entry i of the global list: the last pass b with pre[b].y <= i (then
    // i < pre[b + 1].y; passes without entries share their prefix with the
    // next one)
    auto entry = [&](int i) {
        int b = 0, hi = npass - 1;
        while (b < hi) {
            const int mid = (b + hi + 1) >> 1;
            if (pre[mid].y <= i) b = mid;
            else hi = mid - 1;
        }
        const int4 e = stage[(int64_t)b * kScanPass + (i - pre[b].y)];
        return make_int4(e.x, e.y + pre[b].x, e.z, 0);
    };
    for (int64_t i = gid; i < n_ne; i += gstride) {
        const int4 e = entry((int)i);
        binlist[i] = e.x;
        items[i] = e;
    }
    const int per = (n_ne + 7) >> 3;
    const int64_t slots = gather_slots(nbins);
    for (int64_t blk = gid; blk < slots; blk += gstride) {
        const int k = (int)(blk >> 3), item = (int)(blk & 7) * per + k;
        dealt[blk] = (k < per && item < n_ne) ? entry(item) : make_int4(0, 0, 0, 0);
    }
    if (gid == 0) {
        binstart[nbins] = pre[npass].x;
        binlist[nbins] = n_ne;
    }
}

// The launches of one precision; ROT: with the vector rotation's pairs;
// PPT: points per thread of the bin and scatter kernels.
template <typename T, bool ROT, int PPT>
static hipError_t launch_setpts_b(const SetptsParams &sp, const double *phi, const double *theta,
                                  int32_t *bincount, int32_t *binstart, int32_t *binlist, int64_t nbins,
                                  int2 *keyrank, uint8_t *rowmark, uint8_t *rowtouched, void *rec, int32_t *perm,
                                  int32_t *flags, int4 *stage, int2 *passtot, int32_t *lstart, hipStream_t s)
{
    // bincount, rowmark, flags[0] and the ticket flags[2] are zero on entry:
    // the plan clears them once and every path below leaves them cleared.
    hipError_t e;
    const int threads = kSetptsThreads;
    const int64_t blocks = (sp.n + PPT * kSetptsThreads - 1) / (PPT * kSetptsThreads);
    const int64_t fused_blocks = (sp.n + kScanThreads - 1) / kScanThreads;
    const bool fused = sp.n > 0 && nbins <= (int64_t)kScanChunk * kScanThreads && fused_blocks <= kFusedMaxBlocks &&
                       sp.th.nf <= kMaxRowsPerScanThread * kScanThreads;
    PointRec<T> *r = (PointRec<T> *)rec;
    if (sp.n > 0) {
        auto kern = fused ? k_setpts_bin<T, true, PPT> : k_setpts_bin<T, false, PPT>;
        hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(threads), 0, s, phi, theta, sp, bincount, keyrank,
                           rowmark, flags);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (fused) {
        hipLaunchKernelGGL((k_setpts_scatter_scan<T, ROT>), dim3((unsigned)fused_blocks), dim3(kScanThreads), 0, s,
                           phi, theta, sp, bincount, binstart, binlist, (int)nbins, keyrank, rowmark, rowtouched,
                           sp.th.nf, flags, r, perm);
        return hipGetLastError();
    }
    const int64_t npass = (nbins + kScanPass - 1) / kScanPass;
    if (sp.n > 0 && npass > 1 && npass <= kMaxScanPasses && stage && passtot && lstart &&
        sp.th.nf <= kMaxRowsPerScanThread * kScanThreads) {
        hipLaunchKernelGGL(k_bin_scan_passes, dim3((unsigned)npass), dim3(kScanThreads), 0, s, bincount, nbins,
                           lstart, stage, passtot, rowmark, rowtouched, sp.th.nf, sp.w, flags);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL((k_setpts_scatter_passes<T, ROT, PPT>), dim3((unsigned)blocks), dim3(threads), 0, s, phi, theta,
                           sp, bincount, lstart, stage, passtot, (int)npass, binstart, binlist, nbins, r, perm);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(kScanThreads), 0, s, bincount, binstart, binlist, nbins,
                       rowmark, rowtouched, sp.th.nf, sp.w, flags);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (sp.n > 0) {
        hipLaunchKernelGGL((k_setpts_scatter<T, ROT, PPT>), dim3((unsigned)blocks), dim3(threads), 0, s, phi, theta, sp,
                           bincount, binstart, r, perm, binlist, nbins);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T, bool ROT>
static hipError_t launch_setpts_t(const SetptsParams &sp, const double *phi, const double *theta,
                                  int32_t *bincount, int32_t *binstart, int32_t *binlist, int64_t nbins,
                                  int2 *keyrank, uint8_t *rowmark, uint8_t *rowtouched, void *rec, int32_t *perm,
                                  int32_t *flags, int4 *stage, int2 *passtot, int32_t *lstart, hipStream_t s)
{
    if (sp.n >= kManyPoints)
        return launch_setpts_b<T, ROT, 4>(sp, phi, theta, bincount, binstart, binlist, nbins, keyrank, rowmark,
                                          rowtouched, rec, perm, flags, stage, passtot, lstart, s);
    return launch_setpts_b<T, ROT, 1>(sp, phi, theta, bincount, binstart, binlist, nbins, keyrank, rowmark,
                                      rowtouched, rec, perm, flags, stage, passtot, lstart, s);
}

hipError_t launch_setpts(int prec, const SetptsParams &sp, const double *phi, const double *theta,
                         int32_t *bincount, int32_t *binstart, int32_t *binlist, int64_t nbins,
                         int2 *keyrank,
                         uint8_t *rowmark, uint8_t *rowtouched, void *rec, int32_t *perm,
                         int32_t *flags, int4 *stage, int2 *passtot, int32_t *lstart, hipStream_t s)
{
    const bool rot = sp.pq != nullptr;
    if (prec == 1)
        return rot ? launch_setpts_t<float, true>(sp, phi, theta, bincount, binstart, binlist, nbins, keyrank, rowmark,
                                                  rowtouched, rec, perm, flags, stage, passtot, lstart, s)
                   : launch_setpts_t<float, false>(sp, phi, theta, bincount, binstart, binlist, nbins, keyrank, rowmark,
                                                   rowtouched, rec, perm, flags, stage, passtot, lstart, s);
    return rot ? launch_setpts_t<double, true>(sp, phi, theta, bincount, binstart, binlist, nbins, keyrank, rowmark,
                                               rowtouched, rec, perm, flags, stage, passtot, lstart, s)
               : launch_setpts_t<double, false>(sp, phi, theta, bincount, binstart, binlist, nbins, keyrank, rowmark,
                                                rowtouched, rec, perm, flags, stage, passtot, lstart, s);
}

hipError_t launch_setpts_group(int prec, const SetptsJob *jobs, int n_members, const int32_t *job_of_block,
                               int n_blocks, hipStream_t s)
{
    if (n_members < 1 || !jobs || (n_blocks > 0 && !job_of_block)) return hipErrorInvalidValue;
    hipError_t e;
    if (n_blocks > 0) {
        if (prec == 1)
            hipLaunchKernelGGL(k_setpts_bin_group<float>, dim3(n_blocks), dim3(256), 0, s, jobs, job_of_block);
        else
            hipLaunchKernelGGL(k_setpts_bin_group<double>, dim3(n_blocks), dim3(256), 0, s, jobs, job_of_block);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_bin_scan_group, dim3(n_members), dim3(kScanThreads), 0, s, jobs);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (n_blocks > 0) {
        if (prec == 1)
            hipLaunchKernelGGL(k_setpts_scatter_group<float>, dim3(n_blocks), dim3(256), 0, s, jobs, job_of_block);
        else
            hipLaunchKernelGGL(k_setpts_scatter_group<double>, dim3(n_blocks), dim3(256), 0, s, jobs, job_of_block);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace nufft2
