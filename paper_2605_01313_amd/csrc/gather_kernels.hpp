// Exponential-of-semicircle interpolation of the fine grid at the sorted
// departure points (the per-point stage of the type-2 NUFFT).
//
//   out[f][perm[r]] = sum_{a<w} phi_t[a] * sum_{b<w} phi_p[b] * b_f[(it + a) mod nft][(ip + b) mod nfp]
//   phi_x[a] = exp(beta * (sqrt(1 - z_a^2) - 1)),  z_a = (a - floor(w/2) - v_x) / (w/2)
//
// The grid b_f is complex, or real for real-field plans (whose coefficients
// are Hermitian, so that the upsampled grid is real): then every tap is one
// real product and the output is real.
//
// One workgroup per bin (a tile_t x tile_p block of first-tap cells).  The
// workgroup stages the (tile_t + w - 1) x (tile_p + w - 1) patch of up to
// FG fields at once in LDS, then each thread sums the w x w taps of one
// point for all staged fields (independent accumulators per field; in FP64
// a bin of at most 128 points gives each point two threads, one per half of
// the rows).  Points are dealt to lanes so that the lanes the LDS serves
// together read different banks (the chunk loop and column_rotation).  The
// tap order (rows a outer, columns inner in one of two orders fixed by the
// point's own cell) does not depend on which lane or where in its bin the
// sort placed the point.
//
// Kernel weights: FP32 plans of width >= 7 evaluate each tap's weight as a
// degree-8 polynomial in the point's centred offset (coefficients from the
// plan, interpolated in long double, within 1e-7 of the kernel; mirrored
// taps share the even and odd parts of one polynomial); FP64 plans of width
// >= 7 do the same with degree-14 polynomials (within 2e-15) for all but the
// two edge taps, which are evaluated directly.  The direct form is used
// otherwise, in FP32 written as exp(-beta z^2 / (1 + sqrt(1 - z^2))), which
// has no cancellation near the kernel's peak.
#pragma once

#include "nufft2_internal.hpp"

namespace nufft2 {

// ES kernel exp(beta (sqrt(1 - z^2) - 1)), clamped to e^{-beta} outside |z| <= 1.
// The second argument is es_constant(beta).  FP32 folds beta log2(e) into the
// base-2 exponential; FP64 uses the correctly rounded library calls (the
// cancellation in sqrt(t) - 1 costs at most beta ulp of the exponent, far
// inside a 1e-12 tolerance).
template <typename T> __host__ __device__ inline T es_constant(double beta);
template <> __host__ __device__ inline float es_constant<float>(double beta)
{
    return (float)(beta * 1.4426950408889634);
}
template <> __host__ __device__ inline double es_constant<double>(double beta) { return beta; }

template <typename T> __device__ inline T es_kernel(T z, T k);
template <> __device__ inline float es_kernel<float>(float z, float k)
{
    const float z2 = fminf(z * z, 1.0f);
    return __builtin_amdgcn_exp2f(-k * z2 * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_sqrtf(1.0f - z2)));
}
template <> __device__ inline double es_kernel<double>(double z, double k)
{
    double t = 1.0 - z * z;
    t = t > 0.0 ? t : 0.0;
    return exp(k * (sqrt(t) - 1.0));
}

// Weights of the W taps along both axes for a point with offsets v0 and v1
// (natural column order), into w0 and w1.
template <typename T, int W>
__device__ __forceinline__ void tap_weights2(T v0, T v1, const GatherParams &gp, T (&w0)[W], T (&w1)[W])
{
    constexpr int H = W / 2;
    if constexpr (sizeof(T) == 4 && W >= kPolyMinW) {
        if (gp.wpoly) {
            // u: the offset relative to the centre of its range (0 for odd
            // w, -1/2 for even w)
            const float u0 = (W & 1) ? v0 : v0 + 0.5f;
            const float u1 = (W & 1) ? v1 : v1 + 0.5f;
            // read through the constant address space: the same for every
            // lane, so the coefficients come in by scalar loads into SGPRs
            // (a plain global pointer gets per-lane vector loads); both axes
            // use each coefficient as it arrives
            using cfloat = const __attribute__((address_space(4))) float;
            cfloat *c = (cfloat *)gp.wpoly;
            // The kernel is even, so tap w-1-b at offset u weighs what tap b
            // weighs at -u: with p_b(u) = E(u^2) + u O(u^2), one even and
            // one odd part give both taps of a mirrored pair (the fits at
            // symmetric nodes agree with this up to rounding), and the
            // middle tap of an odd width is its even part alone.
            static_assert(kPolyCoefs % 2 == 1, "even part of degree kPolyCoefs - 1");
            const float t0 = u0 * u0, t1 = u1 * u1;
#pragma unroll
            for (int b = 0; b < (W + 1) / 2; ++b) {
                const float ce = c[b * kPolyCoefs + kPolyCoefs - 1];
                float e0 = ce, e1 = ce;
#pragma unroll
                for (int j = kPolyCoefs - 3; j >= 0; j -= 2) {
                    const float cj = c[b * kPolyCoefs + j];
                    e0 = fmaf(e0, t0, cj);
                    e1 = fmaf(e1, t1, cj);
                }
                if ((W & 1) && b == W / 2) {
                    w0[b] = e0;
                    w1[b] = e1;
                    break;
                }
                const float co = c[b * kPolyCoefs + kPolyCoefs - 2];
                float o0 = co, o1 = co;
#pragma unroll
                for (int j = kPolyCoefs - 4; j >= 1; j -= 2) {
                    const float cj = c[b * kPolyCoefs + j];
                    o0 = fmaf(o0, t0, cj);
                    o1 = fmaf(o1, t1, cj);
                }
                w0[b] = fmaf(u0, o0, e0);
                w0[W - 1 - b] = fmaf(-u0, o0, e0);
                w1[b] = fmaf(u1, o1, e1);
                w1[W - 1 - b] = fmaf(-u1, o1, e1);
            }
            return;
        }
    }
    const T inv_hw = (T)2 / (T)W;
    const T kc = es_constant<T>(gp.beta);
#pragma unroll
    for (int b = 0; b < W; ++b) {
        w0[b] = es_kernel<T>(((T)(b - H) - v0) * inv_hw, kc);
        w1[b] = es_kernel<T>(((T)(b - H) - v1) * inv_hw, kc);
    }
}

// FP64 tap-weight polynomials in the power basis: t = u^2 and its powers
// tp[k] = t^k, k <= (kPolyCoefs64 - 1) / 2, computed once per point and axis,
// so that every coefficient enters as a multiplicand (a scalar operand of one
// FMA) rather than as the addend of a Horner step (which the compiler feeds
// through two vector moves per coefficient).  |t| <= 1/4: the terms decrease
// with k and are summed from the highest degree down.
constexpr int kPow64 = (kPolyCoefs64 + 1) / 2;
__device__ __forceinline__ void powers_f64(double u, double (&tp)[kPow64])
{
    tp[0] = 1.0;
    tp[1] = u * u;
#pragma unroll
    for (int k = 2; k < kPow64; ++k) tp[k] = tp[k - 1] * tp[1];
}

// Even and odd parts of the polynomial of row r of the table c at t:
// p_r(u) = e + u o.
using cdouble = const __attribute__((address_space(4))) double;
__device__ __forceinline__ void poly_parts_f64(cdouble *c, int r, const double (&tp)[kPow64], double &e, double &o)
{
    constexpr int D = kPolyCoefs64;
    static_assert(D % 2 == 1, "even part of degree D - 1");
    cdouble *q = c + r * D;
    e = q[D - 1] * tp[kPow64 - 1];
#pragma unroll
    for (int k = kPow64 - 2; k >= 1; --k) e = fma(q[2 * k], tp[k], e);
    e += q[0];
    o = q[D - 2] * tp[kPow64 - 2];
#pragma unroll
    for (int k = kPow64 - 3; k >= 1; --k) o = fma(q[2 * k + 1], tp[k], o);
    o += q[1];
}

// The plan's FP64 table, read through the constant address space (scalar
// loads into SGPRs).  The pointer is made opaque where it is taken, so that
// the compiler cannot hoist the loads of the whole table out of the point
// loop (which would hold every coefficient in registers across it).
__device__ __forceinline__ cdouble *poly_table_f64(const GatherParams &gp)
{
    cdouble *c = (cdouble *)gp.wpoly;
    __asm__ volatile("" : "+s"(c));
    return c;
}

// FP64 weights of the W taps along one axis for a point with offset v: taps
// 1 .. W - 2 from the plan's polynomials when it has them (mirrored taps
// share the even and odd parts of one polynomial, as in FP32), taps 0 and
// W - 1 directly (the kernel's square-root edge lies in their intervals,
// where no polynomial of modest degree follows it to 1e-15).
template <int W>
__device__ __forceinline__ void tap_weights_f64(double v, const GatherParams &gp, double (&wt)[W])
{
    constexpr int H = W / 2;
    const double inv_hw = 2.0 / (double)W;
    const double kc = gp.beta;
    if constexpr (W >= kPolyMinW64) {
        if (gp.wpoly) {
            const double u = (W & 1) ? v : v + 0.5;
            cdouble *c = poly_table_f64(gp);
            double tp[kPow64];
            powers_f64(u, tp);
#pragma unroll
            for (int b = 1; b < (W + 1) / 2; ++b) {
                double e, o;
                poly_parts_f64(c, b, tp, e, o);
                if ((W & 1) && b == W / 2) {
                    wt[b] = e;
                    break;
                }
                wt[b] = fma(u, o, e);
                wt[W - 1 - b] = fma(-u, o, e);
            }
            wt[0] = es_kernel<double>(((double)(-H) - v) * inv_hw, kc);
            wt[W - 1] = es_kernel<double>(((double)(W - 1 - H) - v) * inv_hw, kc);
            return;
        }
    }
#pragma unroll
    for (int b = 0; b < W; ++b) wt[b] = es_kernel<double>(((double)(b - H) - v) * inv_hw, kc);
}

// FP64 weight of tap a for the offset v (a is the same for every lane of
// the wave, so that the coefficients come in by scalar loads): the row's
// polynomial at the powers tp of the centred offset u for interior taps,
// the kernel itself for the edge taps and for plans without polynomials.
template <int W>
__device__ __forceinline__ double row_weight_f64(int a, double v, double u, const double (&tp)[kPow64],
                                                 const GatherParams &gp)
{
    constexpr int H = W / 2;
    if constexpr (W >= kPolyMinW64) {
        if (gp.wpoly && a > 0 && a < W - 1) {
            double e, o;
            poly_parts_f64(poly_table_f64(gp), a, tp, e, o);
            return fma(u, o, e);
        }
    }
    return es_kernel<double>(((double)(a - H) - v) * (2.0 / (double)W), gp.beta);
}

// Accumulation a += w v for real and complex grid values.
__device__ inline void acc_fma(float &a, float w, float v) { a = fmaf(w, v, a); }
__device__ inline void acc_fma(double &a, double w, double v) { a = fma(w, v, a); }
__device__ inline void acc_fma(float2 &a, float w, float2 v)
{
    a.x = fmaf(w, v.x, a.x);
    a.y = fmaf(w, v.y, a.y);
}
__device__ inline void acc_fma(double2 &a, double w, double2 v)
{
    a.x = fma(w, v.x, a.x);
    a.y = fma(w, v.y, a.y);
}
__device__ inline void acc_add(float &a, float b) { a += b; }
__device__ inline void acc_add(double &a, double b) { a += b; }
__device__ inline void acc_add(float2 &a, float2 b) { a.x += b.x; a.y += b.y; }
__device__ inline void acc_add(double2 &a, double2 b) { a.x += b.x; a.y += b.y; }
template <typename T> __device__ inline T nan_of(T) { return (T)NAN; }
__device__ inline float2 nan_of(float2) { return {NAN, NAN}; }
__device__ inline double2 nan_of(double2) { return {NAN, NAN}; }
__device__ inline float real_of(float a) { return a; }
__device__ inline double real_of(double a) { return a; }
__device__ inline float real_of(float2 a) { return a.x; }
__device__ inline double real_of(double2 a) { return a.x; }

// 16-byte vector of the plan's real type (a staging chunk).  Native
// vector types: a copy is one value, not a struct copy (which the compiler
// lowers to a memory copy through the stack when a barrier sits between
// the load and the store).
template <typename T> struct VecOf { using type = double __attribute__((ext_vector_type(2))); };
template <> struct VecOf<float> { using type = float __attribute__((ext_vector_type(4))); };

template <typename T, bool RG> struct GridElem { using type = cplx<T>; };
template <typename T> struct GridElem<T, true> { using type = T; };

// Workgroup size: FP32 bins (about 128 points at the default tile) run on
// kGatherThreadsF32 threads, FP64 on 256 (whose bins of at most 128 points
// split their rows over two lanes).
constexpr int kGatherThreadsF32 = 256;
template <typename T> constexpr int gather_threads() { return sizeof(T) == 4 ? kGatherThreadsF32 : 256; }
constexpr int kLoadBatch = 4;
// FP64 splits the rows of a point over two lanes when a chunk holds at most
// half a workgroup's points (see gather_body).
template <typename T> constexpr bool kSplitRows = sizeof(T) == 8;

// Lanes the LDS serves together: 16 for reads of 8 bytes (FP32 complex,
// FP64 real: 128 bytes over 32 banks) and of 16 bytes (FP64 complex: 256
// bytes over 64 four-byte banks), 32 for reads of 4 bytes (FP32 real).  A
// CPU model of the tap reads with these groups and bank slots (element
// offset modulo the group) reproduces the conflict rates measured on gfx950
// with SQ_LDS_BANK_CONFLICT for the 2048^2 wind workload.  Lanes of such a
// group whose patch offsets differ modulo the group size never collide on a
// bank, whatever tap they read.
template <typename E> constexpr int lds_lane_group() { return sizeof(E) == 4 ? 32 : 16; }

// Departure points sit near a lattice of spacing 2 fine cells (the grid nodes
// at upsampling factor 2), so the patch offsets of the points of a bin share
// their parity and a plain layout leaves half of the banks idle.  Points on
// the two colours of a checkerboard over that lattice read their columns in
// two orders (0 .. w-1, or 1 .. w-1 then 0), which moves half of them to the
// other parity.  The order depends only on the point's own cell.
__device__ inline int column_rotation(int it, int ip) { return ((it >> 1) ^ (ip >> 1)) & 1; }

// Tile shapes with compile-time patch geometry (TT x TP first-tap cells):
// every tap's LDS offset is then an immediate.  TT = TP = 0: the plan's
// tile at run time.
template <int TT, int TP> struct TileShape {
    static constexpr bool fixed = TT > 0;
};

// Deal the points of the chunk starting at base to lanes: counting-sort
// them by bank key (patch offset of the first tap plus the column rotation,
// modulo NK), then give sorted position k to lane (k mod R) * NK + k / R.
// Points R apart in key order share a lane group, so a group holds distinct
// keys unless one key has more than R points.  The order inside a key
// (atomic ranks) does not matter: a point's sum does not depend on its lane.
// Every thread of the workgroup calls it (it has barriers); it touches only
// the dealing arrays (bucket, slot, dsts, recs), not the patch.  Chunk 0's
// records (q0, d0) were loaded by the caller.
template <typename T, int NK, int NT>
__device__ __forceinline__ void deal_chunk(int base, int cnt, int start, PointRec<T> q0, int d0, int r0,
                                           int c0, int TCP, const PointRec<T> *__restrict__ rec,
                                           const int32_t *__restrict__ perm, int *bucket, short *slot, int *dsts,
                                           PointRec<T> *recs)
{
    const int n = min(NT, cnt - base);
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
}

// blk: this workgroup's index in the stage (8 * ceil(nbins / 8) of them).
template <typename T, bool RG, int W, int FG, int TT, int TP>
__device__ inline void gather_body(int blk, const typename GridElem<T, RG>::type *__restrict__ grid,
                                   const PointRec<T> *__restrict__ rec, const int32_t *__restrict__ perm,
                                   const int32_t *__restrict__ binlist, void *__restrict__ out,
                                   const GatherParams &gp)
{
    using E = typename GridElem<T, RG>::type;
    // The dynamic region starts right after the static LDS arrays below;
    // without the alignment a static array whose size is not a multiple of
    // 16 bytes misaligns every 16-byte complex read of the patch (a 4-6x
    // slower gather, measured).
    extern __shared__ __align__(16) unsigned char smem_raw[];
    E *tiles = reinterpret_cast<E *>(smem_raw);
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
    constexpr bool FIXED = TileShape<TT, TP>::fixed;
    // Chunk 0 is dealt while the patch loads are in flight where that was
    // measured faster: compile-time tiles (one or two load batches) and
    // FP64 real grids.  Elsewhere the batches held across the dealing cost
    // more registers than the overlap gains (FP64 complex: 15% slower).
    constexpr bool kEarlyDeal = FIXED || (sizeof(T) == 8 && RG);
    const int tile_t = FIXED ? TT : gp.tile_t;
    const int tile_p = FIXED ? TP : gp.tile_p;
    const int bt = bin / gp.nbins_phi, bp = bin - bt * gp.nbins_phi;
    const int r0 = bt * tile_t, c0 = bp * tile_p;
    const int TR = tile_t + W - 1, TC = tile_p + W - 1;
    // The patch is staged in 16-byte chunks of V consecutive elements (4
    // real or 2 complex FP32 values, 2 real or 1 complex FP64 value): c0 and
    // the grid width are multiples of V, so a chunk never straddles the
    // torus seam and is 16-byte aligned in memory.  LDS rows hold NC whole
    // chunks (TCP = NC V elements; 16-byte elements may pad rows further)
    // so that the stores are 16-byte aligned too.
    constexpr int V = 16 / (int)sizeof(E);
    const int NC = (TC + V - 1) / V;
    const int TCP = sizeof(E) != 16 ? NC * V : gp.tile_pitch;
    const int plane = TR * TCP;
    constexpr int H = W / 2;
    constexpr int NK = lds_lane_group<E>();
    constexpr int NT = gather_threads<T>();
    static_assert(NT % NK == 0 && NK <= 64, "lane groups tile the workgroup; the key scan runs in wave 0");
    __shared__ int bucket[NK];  // per bank key: count, then start
    __shared__ short slot[NT];  // lane -> point of the chunk (-1: none)
    __shared__ int dsts[NT];    // destination of each point of the chunk
    __shared__ PointRec<T> recs[NT];  // record of each point of the chunk
    __shared__ E xsum[kSplitRows<T> ? NT / 2 * FG : 1];  // partial sums of split points
    const int64_t field_stride = (int64_t)gp.nft * gp.nfp;

    // FG fields per pass; the last pass may hold fewer (fg)
    for (int f0 = 0; f0 < gp.n_fields; f0 += FG) {
        const int fg = min(FG, gp.n_fields - f0);
        __syncthreads();
        // Stage the patch: each thread issues the loads of up to kLoadBatch
        // chunks (all fields, one offset for all of them) before it stores
        // any of them, so that one memory round trip serves the batch.
        using Vec = typename VecOf<T>::type;
        const int nchunk = TR * NC;
        const E *gridf[FG];
#pragma unroll
        for (int f = 0; f < FG; ++f) gridf[f] = grid + (int64_t)(f0 + (f < fg ? f : 0)) * field_stride;
        for (int j0 = 0; j0 < nchunk; j0 += kLoadBatch * NT) {
            Vec buf[kLoadBatch][FG];
            int lo[kLoadBatch];
            // Loads past the patch are clamped to its first chunk and not
            // stored (unconditional loads keep the buffer in registers);
            // with a compile-time tile, batches wholly past the patch are
            // left out.
#pragma unroll
            for (int u = 0; u < kLoadBatch; ++u) {
                lo[u] = -1;
                if (!FIXED || j0 + u * NT < nchunk) {
                    const int j = j0 + u * NT + (int)threadIdx.x;
                    const int jj = j < nchunk ? j : 0;
                    const int r = jj / NC, k = jj - r * NC;
                    const int off = ((r0 + r) & (gp.nft - 1)) * gp.nfp + ((c0 + k * V) & (gp.nfp - 1));
                    lo[u] = j < nchunk ? r * TCP + k * V : -1;
#pragma unroll
                    for (int f = 0; f < FG; ++f) buf[u][f] = *reinterpret_cast<const Vec *>(gridf[f] + off);
                }
            }
            // chunk 0's dealing waits only for its records (requested
            // before the patch), so it runs while the patch is in flight
            if (kEarlyDeal && j0 == 0) deal_chunk<T, NK, NT>(0, cnt, start, q0, d0, r0, c0, TCP, rec, perm, bucket, slot, dsts, recs);
#pragma unroll
            for (int u = 0; u < kLoadBatch; ++u) {
                if (lo[u] >= 0) {
#pragma unroll
                    for (int f = 0; f < FG; ++f) *reinterpret_cast<Vec *>(tiles + f * plane + lo[u]) = buf[u][f];
                }
            }
        }
        __syncthreads();
        for (int base = 0; base < cnt; base += NT) {
            if (base > 0 || !kEarlyDeal) deal_chunk<T, NK, NT>(base, cnt, start, q0, d0, r0, c0, TCP, rec, perm, bucket, slot, dsts, recs);
            const int n = min(NT, cnt - base);
            const int t = (int)threadIdx.x;
            // In FP64 a bin of at most half a workgroup's points (one chunk,
            // which the dealing put on the lower half of the lanes) is split
            // by rows: lane t + 128 takes rows H1 .. w-1 of lane t's point
            // and hands its partial sums over through LDS, so that all four
            // waves work on the taps instead of two.  The choice depends on
            // the bin's count only, never on which chunk a point fell in, so
            // a point's sum stays independent of the order inside its bin.
            constexpr int HALF = NT / 2;
            static_assert(HALF % 64 == 0, "the split halves are whole waves");
            const bool split = kSplitRows<T> && cnt <= HALF;
            const bool upper = split && t >= HALF;
            const int mine = upper ? slot[t - HALF] : slot[t];
            constexpr int H1 = (W + 1) / 2;
            E acc[FG];
#pragma unroll
            for (int f = 0; f < FG; ++f) acc[f] = E{};
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
                // FP32 takes the row weights with the column weights; FP64
                // computes them row by row below
                T pw[W], wp[W], pt[W];
                if constexpr (sizeof(T) == 4) tap_weights2<T, W>(bad ? (T)0 : pr.vp, bad ? (T)0 : pr.vt, gp, pw, pt);
                else tap_weights_f64<W>(bad ? 0.0 : pr.vp, gp, pw);
#pragma unroll
                for (int b = 0; b < W; ++b) wp[b] = rot ? pw[(b + 1) % W] : pw[b];
                const E *row0 = tiles + lr * TCP + lc;
                if constexpr (sizeof(T) == 4) {
                    // FP32: every row unrolled, its taps at immediate offsets
                    // when the tile is fixed; the scheduling barrier after
                    // each row keeps the compiler from hoisting every row's
                    // LDS reads (and running out of registers)
                    const E *rrow = row0 + rot;
                    const E *lrow = row0 + last;
#pragma unroll
                    for (int a = 0; a < W; ++a) {
                        E r[FG];
#pragma unroll
                        for (int f = 0; f < FG; ++f) r[f] = E{};
#pragma unroll
                        for (int b = 0; b < W; ++b) {
#pragma unroll
                            for (int f = 0; f < FG; ++f) {
                                // fields past fg read stale LDS; their sums are never stored
                                const E v = b < W - 1 ? rrow[a * TCP + f * plane + b] : lrow[a * TCP + f * plane];
                                acc_fma(r[f], wp[b], v);
                            }
                        }
#pragma unroll
                        for (int f = 0; f < FG; ++f) acc_fma(acc[f], pt[a], r[f]);
                        __builtin_amdgcn_sched_barrier(0);
                    }
                } else {
                    // FP64: rows stay a loop (two per iteration), row weights
                    // on the fly; split points take their half of the rows.
                    // The row range is the same for every lane of a wave
                    // (the split halves are whole waves), which readfirstlane
                    // tells the compiler, so that the row index is scalar.
                    const int a_begin = __builtin_amdgcn_readfirstlane(upper ? H1 : 0);
                    const int a_end = __builtin_amdgcn_readfirstlane(split && !upper ? H1 : W);
                    const double ut = (W & 1) ? pr.vt : pr.vt + 0.5;
                    double tpt[kPow64];
                    powers_f64(ut, tpt);
#pragma unroll 2
                    for (int a = a_begin; a < a_end; ++a) {
                        const T wt = row_weight_f64<W>(a, pr.vt, ut, tpt, gp);
                        const E *row = row0 + a * TCP;
                        const E *rrow = row + rot;
                        E r[FG];
#pragma unroll
                        for (int f = 0; f < FG; ++f) r[f] = E{};
#pragma unroll
                        for (int b = 0; b < W; ++b) {
#pragma unroll
                            for (int f = 0; f < FG; ++f) {
                                const E v = b < W - 1 ? rrow[f * plane + b] : row[f * plane + last];
                                acc_fma(r[f], wp[b], v);
                            }
                        }
#pragma unroll
                        for (int f = 0; f < FG; ++f) acc_fma(acc[f], wt, r[f]);
                    }
                }
            }
            if (split) {
                if (upper && mine >= 0) {
#pragma unroll
                    for (int f = 0; f < FG; ++f) xsum[(t - HALF) * FG + f] = acc[f];
                }
                __syncthreads();
                if (!upper && mine >= 0) {
#pragma unroll
                    for (int f = 0; f < FG; ++f) acc_add(acc[f], xsum[t * FG + f]);
                }
            }
            if (mine < 0 || upper) continue;
            if (gp.pq && gp.rot_u >= f0 && gp.rot_u < f0 + fg) {
                // vector rotation: (u, v) -> (p u + q v, -q u + p v) with the
                // point's pair from setpts (both fields are in this pass)
                const T *pq = reinterpret_cast<const T *>(gp.pq) + 2 * ((int64_t)start + base + mine);
                const T p = pq[0], q = pq[1];
                E u{}, v{};
#pragma unroll
                for (int f = 0; f < FG; ++f) {
                    if (f0 + f == gp.rot_u) u = acc[f];
                    if (f0 + f == gp.rot_v) v = acc[f];
                }
                E ru{}, rv{};
                acc_fma(ru, p, u);
                acc_fma(ru, q, v);
                acc_fma(rv, -q, u);
                acc_fma(rv, p, v);
#pragma unroll
                for (int f = 0; f < FG; ++f) {
                    if (f0 + f == gp.rot_u) acc[f] = ru;
                    if (f0 + f == gp.rot_v) acc[f] = rv;
                }
            }
#pragma unroll
            for (int f = 0; f < FG; ++f) {
                if (f < fg) {
                    const int64_t o = (int64_t)(f0 + f) * gp.n_pts + dst;
                    const E x = bad ? nan_of(E{}) : acc[f];
                    if (RG || gp.real_output) reinterpret_cast<T *>(out)[o] = real_of(x);
                    else reinterpret_cast<E *>(out)[o] = x;
                }
            }
        }
    }
}

template <typename T, bool RG, int W, int FG, int TT, int TP>
__global__ __launch_bounds__(gather_threads<T>()) void k_gather(const typename GridElem<T, RG>::type *__restrict__ grid,
                                                           const PointRec<T> *__restrict__ rec,
                                                           const int32_t *__restrict__ perm,
                                                           const int32_t *__restrict__ binlist,
                                                           void *__restrict__ out, GatherParams gp)
{
    gather_body<T, RG, W, FG, TT, TP>((int)blockIdx.x, grid, rec, perm, binlist, out, gp);
}

// Member j of a group class owns workgroups [j * per, (j + 1) * per); per is
// a multiple of 8, so a workgroup's XCD is the same as in a launch of its own.
template <typename T, bool RG, int W, int FG, int TT, int TP>
__global__ __launch_bounds__(gather_threads<T>()) void k_gather_group(const GatherJob *__restrict__ jobs, int per)
{
    const int j = (int)blockIdx.x / per;
    const GatherJob J = jobs[j];
    gather_body<T, RG, W, FG, TT, TP>((int)blockIdx.x - j * per,
                                      (const typename GridElem<T, RG>::type *)J.grid, (const PointRec<T> *)J.rec,
                                      J.perm, J.binlist, J.out, J.gp);
}

// jobs == nullptr: one plan (the pointer arguments); otherwise n_members
// members of one group class described by jobs (device memory).
template <typename T, bool RG, int W, int FG, int TT, int TP>
static hipError_t launch_tile(const GatherParams &gp, const void *grid, const void *rec, const int32_t *perm,
                              const int32_t *binlist, void *out, const GatherJob *jobs, int n_members,
                              hipStream_t s)
{
    using E = typename GridElem<T, RG>::type;
    constexpr int V = 16 / (int)sizeof(E);
    const int pitch = sizeof(E) != 16 ? (gp.tile_p + W - 1 + V - 1) / V * V : gp.tile_pitch;
    if (pitch < gp.tile_p + W - 1 || gp.tile_p % V != 0 || gp.nfp % V != 0) return hipErrorInvalidValue;
    const size_t lds = sizeof(E) * (size_t)(gp.tile_t + W - 1) * pitch * FG;
    const int per = (int)(8 * ((gp.nbins + 7) / 8));
    if (jobs) {
        auto kern = k_gather_group<T, RG, W, FG, TT, TP>;
        if (lds > 65536)
            (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(kern, dim3((unsigned)(per * n_members)), dim3(gather_threads<T>()), lds, s, jobs, per);
    } else {
        auto kern = k_gather<T, RG, W, FG, TT, TP>;
        if (lds > 65536)
            (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(kern, dim3((unsigned)per), dim3(gather_threads<T>()), lds, s, (const E *)grid,
                           (const PointRec<T> *)rec, perm, binlist, out, gp);
    }
    return hipGetLastError();
}

// The default tiles of FP32 plans (16 x 32 complex, 16 x 64 real-field)
// have compile-time patch geometry; other tiles and FP64 take it at run time.
template <typename T, bool RG, int W, int FG>
static hipError_t launch_wf(const GatherParams &gp, const void *grid, const void *rec,
                            const int32_t *perm, const int32_t *binlist, void *out, const GatherJob *jobs,
                            int n_members, hipStream_t s)
{
    if constexpr (sizeof(T) == 4 && !RG) {
        if (gp.tile_t == 16 && gp.tile_p == 32)
            return launch_tile<T, RG, W, FG, 16, 32>(gp, grid, rec, perm, binlist, out, jobs, n_members, s);
    }
    if constexpr (sizeof(T) == 4 && RG) {
        if (gp.tile_t == 16 && gp.tile_p == 64)
            return launch_tile<T, RG, W, FG, 16, 64>(gp, grid, rec, perm, binlist, out, jobs, n_members, s);
    }
    return launch_tile<T, RG, W, FG, 0, 0>(gp, grid, rec, perm, binlist, out, jobs, n_members, s);
}

template <typename T, bool RG, int W>
static hipError_t launch_w(const GatherParams &gp, const void *grid, const void *rec, const int32_t *perm,
                           const int32_t *binlist, void *out, const GatherJob *jobs,
                           int n_members, hipStream_t s)
{
    switch (gp.fields_per_pass) {
    case 1: return launch_wf<T, RG, W, 1>(gp, grid, rec, perm, binlist, out, jobs, n_members, s);
    case 2: return launch_wf<T, RG, W, 2>(gp, grid, rec, perm, binlist, out, jobs, n_members, s);
    case 3: return launch_wf<T, RG, W, 3>(gp, grid, rec, perm, binlist, out, jobs, n_members, s);
    case 4: return launch_wf<T, RG, W, 4>(gp, grid, rec, perm, binlist, out, jobs, n_members, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, bool RG>
static hipError_t launch_t(const GatherParams &gp, const void *grid, const void *rec, const int32_t *perm,
                           const int32_t *binlist, void *out, const GatherJob *jobs,
                           int n_members, hipStream_t s)
{
    switch (gp.w) {
#define NUFFT2_W(X) case X: return launch_w<T, RG, X>(gp, grid, rec, perm, binlist, out, jobs, n_members, s);
        NUFFT2_W(2) NUFFT2_W(3) NUFFT2_W(4) NUFFT2_W(5) NUFFT2_W(6) NUFFT2_W(7) NUFFT2_W(8)
        NUFFT2_W(9) NUFFT2_W(10) NUFFT2_W(11) NUFFT2_W(12) NUFFT2_W(13) NUFFT2_W(14)
        NUFFT2_W(15) NUFFT2_W(16)
#undef NUFFT2_W
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
static hipError_t launch_prec(const GatherParams &gp, const void *grid, const void *rec, const int32_t *perm,
                              const int32_t *binlist, void *out, const GatherJob *jobs, int n_members, hipStream_t s)
{
    if (gp.real_grid) return launch_t<T, true>(gp, grid, rec, perm, binlist, out, jobs, n_members, s);
    return launch_t<T, false>(gp, grid, rec, perm, binlist, out, jobs, n_members, s);
}

}  // namespace nufft2
