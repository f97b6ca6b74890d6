// Deconvolution + zero padding + the upsampled 2-D inverse FFT, as two
// pruned passes of batched Stockham FFTs staged in LDS.
//
// The grid value at fine cell (l_t, l_p) is
//     b[l_t, l_p] = sum_n sum_m c[n,m] corr_t[n] corr_p[m] e^{+2 pi i (n l_t / nft + m l_p / nfp)}
// (unnormalised inverse DFT of the deconvolved, zero-padded coefficients).
//
//   theta pass: for each phi mode m (a batch of columns per workgroup), the
//     transform over n of the deconvolved coefficients c[n][m] corr_t[n] corr_p[m].  Because
//     K_theta <= nft / 2 (upsampling factor 2), the even and odd output rows
//     are two independent half-length transforms:
//         b[2q + r] = sum_n (x_n e^{2 pi i n r / nft}) e^{2 pi i n q / (nft/2)},
//     with n taken modulo nft/2 (no two modes collide).  Each workgroup does
//     one parity, so there are twice as many workgroups, each with half the
//     LDS.  Only the theta rows some point's taps reach are written, to
//     S[l_t][m] (modes along the row, K_phi long).
//   phi pass: for each reached theta row, the length-nfp transform over m of
//     S[l_t][:], written to the fine grid b[l_t][:].
// Doing theta first keeps the intermediate at nft x K_phi (half the size of
// the other order's K_theta x nfp), and only reached rows enter the phi pass.
//
// Each transform is a Stockham sequence of radix-16 stages (radix 8 for
// kernels with 8 elements per thread), a smaller radix first when log2 N is
// not a multiple of 4 (3), with the length fixed at compile time.
// The first stage reads straight from global memory into registers, the
// middle stages go through LDS (one padding slot every 32 elements against
// bank conflicts), the last stage writes straight to global memory; both are
// contiguous in the index consecutive threads step through.  Twiddles come
// from two short tables staged in LDS at kernel start.
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

// Radix 16 as 4 x 4: with r = 4a + b and q = c + 4d,
// y_{c + 4d} = sum_b e^{2 pi i b d / 4} [e^{2 pi i b c / 16} sum_a x_{4a + b} e^{2 pi i a c / 4}].
template <typename C> __device__ inline void dft16(C *x)
{
    using R = decltype(x[0].x);
    const R c1 = (R)0.92387953251128675612818318939678828682;  // cos(pi / 8)
    const R s1 = (R)0.38268343236508977172845998403039886676;  // sin(pi / 8)
    const R h = (R)0.70710678118654752440084436210484903928;
#pragma unroll
    for (int b = 0; b < 4; ++b) dft4(x[b], x[4 + b], x[8 + b], x[12 + b]);
    // x[4c + b] *= e^{2 pi i b c / 16}; b c in {1, 2, 3, 4, 6, 9}
    auto rot = [](C v, R cr, R ci) { return C{v.x * cr - v.y * ci, v.x * ci + v.y * cr}; };
    auto rot2 = [h](C v) { return C{h * (v.x - v.y), h * (v.x + v.y)}; };    // e^{i pi / 4}
    auto rot6 = [h](C v) { return C{-h * (v.x + v.y), h * (v.x - v.y)}; };   // e^{3 i pi / 4}
    x[5] = rot(x[5], c1, s1);
    x[6] = rot2(x[6]);
    x[7] = rot(x[7], s1, c1);
    x[9] = rot2(x[9]);
    x[10] = cmuli(x[10]);
    x[11] = rot6(x[11]);
    x[13] = rot(x[13], s1, c1);
    x[14] = rot6(x[14]);
    x[15] = rot(x[15], -c1, -s1);
#pragma unroll
    for (int c = 0; c < 4; ++c) dft4(x[4 * c], x[4 * c + 1], x[4 * c + 2], x[4 * c + 3]);
    // y_{c + 4d} sits in x[4c + d]: transpose the 4 x 4 block
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int d = c + 1; d < 4; ++d) {
            const C t = x[4 * c + d];
            x[4 * c + d] = x[4 * d + c];
            x[4 * d + c] = t;
        }
}

template <int R, typename C> __device__ inline void dft(C *x)
{
    if constexpr (R == 2) dft2(x);
    else if constexpr (R == 4) dft4(x);
    else if constexpr (R == 8) dft8(x);
    else dft16(x);
}

// Stage plan for N = 2^LOGN with E elements per thread: radix-16 stages
// when a thread holds 16 elements (one butterfly), else radix 8; a first
// stage of the remaining smaller radix when log2 N is not a multiple.
template <int LOGN, int E> struct StagePlan {
    static constexpr int LR = E >= 16 ? 4 : 3;
    static constexpr int REM = LOGN % LR;
    static constexpr int NST = LOGN / LR + (REM ? 1 : 0);
    static constexpr int radix(int s) { return (s == 0 && REM) ? (1 << REM) : (1 << LR); }
    static constexpr int ns(int s)
    {
        int v = 1;
        for (int i = 0; i < s; ++i) v *= radix(i);
        return v;
    }
};

// Twiddles e^{2 pi i t / N} as a product of two short tables held in LDS:
// lo[t mod 64] * hi[t / 64] (N/64 + 64 entries instead of N), so that a
// stage's twiddle reads go out with its data reads instead of waiting on
// the L2.  The host fills both tables from long double and rounds once; the
// product adds at most about one rounding of the plan precision.
constexpr int kTwLoBits = 6;
constexpr int kTwLo = 1 << kTwLoBits;
constexpr int tw_hi_len(int n) { return n > kTwLo ? n / kTwLo : 1; }
constexpr int tw_lds_len(int n) { return kTwLo + tw_hi_len(n); }

template <typename C>
__device__ inline C twiddle(const C *tw, int t)
{
    return cmul(tw[t & (kTwLo - 1)], tw[kTwLo + (t >> kTwLoBits)]);
}

// LDS slot of element i of a sequence: one padding slot every 32 elements.
__device__ constexpr int lds_slot(int i) { return i + (i >> 5); }
constexpr int lds_seq_len(int n) { return n + (n >> 5); }

// LDS address of element i of sequence b.
// BFAST (consecutive threads step through b): lds_slot(i) * IS + b, IS = B.
// Otherwise (threads step through i): lds_slot(i) + b * BS with BS the padded
// sequence length.  (An odd pitch B + 1 for BFAST was measured no faster and
// costs LDS that lowers the number of workgroups per CU.)
template <bool BFAST>
__device__ inline int lds_addr(int i, int b, int IS, int BS)
{
    if constexpr (BFAST) return lds_slot(i) * IS + b;
    else return lds_slot(i) + b * BS;
}

// Job q of this thread in a stage of radix R over B sequences of length N.
template <int N, int R, bool BFAST>
__device__ inline void job_of(int q, int logB, int &j, int &b)
{
    constexpr int NBF = N / R;
    const int job = threadIdx.x + q * blockDim.x;
    if constexpr (BFAST) {
        b = job & ((1 << logB) - 1);
        j = job >> logB;
    } else {
        j = job & (NBF - 1);
        b = job / NBF;
    }
}

// One Stockham stage: butterfly (j, b) takes elements j + r N/R, applies
// W_{NS R}^{r k} (k = j mod NS), transforms, and writes element
// ((j - k) R + k) + r NS.  The first stage takes element i of sequence b
// from ld(i, b) (global memory); the last hands element o to st(o, b, v).
// The first stage also runs the prologue in two halves: pro.fetch() issues
// its small loads before the stage's data loads and pro.commit() stores
// them to LDS after.  Vector loads complete in issue order, so waiting for
// the prologue's loads then does not wait for the data as well (a loop of
// loads and stores placed after the data loads costs one full memory round
// trip per iteration).
template <typename T, int LOGN, int S, int E, bool BFAST, class Loader, class Storer, class Pro>
__device__ inline void stockham_stage(cplx<T> *s, int logB, int IS, int BS,
                                      const cplx<T> *__restrict__ tws, const Loader &ld,
                                      const Storer &st, const Pro &pro)
{
    using P = StagePlan<LOGN, E>;
    constexpr int N = 1 << LOGN;
    constexpr int R = P::radix(S), NS = P::ns(S);
    constexpr bool FIRST = S == 0, LAST = S == P::NST - 1;
    constexpr int Q = E / R;
    constexpr int NBF = N / R;
    cplx<T> v[E];
    int jj[Q], bb[Q];
    typename Pro::Regs pre{};
    if constexpr (FIRST) pre = pro.fetch();
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        int j, b;
        job_of<N, R, BFAST>(q, logB, j, b);
        jj[q] = j;
        bb[q] = b;
        if constexpr (FIRST) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[q * R + r] = ld(j + r * NBF, b);
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) v[q * R + r] = s[lds_addr<BFAST>(j + r * NBF, b, IS, BS)];
            const int k = j & (NS - 1);
            constexpr int STRIDE = N / (NS * R);
#pragma unroll
            for (int r = 1; r < R; ++r) v[q * R + r] = cmul(v[q * R + r], twiddle(tws, r * k * STRIDE));
        }
    }
    if constexpr (FIRST) {
        pro.commit(pre);
        // a one-stage transform stores right away: what the prologue put in
        // LDS (the theta pass's row flags) must be visible to every thread
        if constexpr (LAST) __syncthreads();
    } else {
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        dft<R>(&v[q * R]);
        const int j = jj[q], b = bb[q];
        const int k = j & (NS - 1);
        const int base = (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int o = base + r * NS;
            if constexpr (LAST) st(o, b, v[q * R + r]);
            else s[lds_addr<BFAST>(o, b, IS, BS)] = v[q * R + r];
        }
    }
    if constexpr (!LAST) __syncthreads();
}

template <typename T, int LOGN, int S, int E, bool BFAST, class Loader, class Storer, class Pro>
__device__ inline void fft_stages(cplx<T> *s, int logB, int IS, int BS, const cplx<T> *tws,
                                  const Loader &ld, const Storer &st, const Pro &pro)
{
    if constexpr (S < StagePlan<LOGN, E>::NST) {
        stockham_stage<T, LOGN, S, E, BFAST>(s, logB, IS, BS, tws, ld, st, pro);
        fft_stages<T, LOGN, S + 1, E, BFAST>(s, logB, IS, BS, tws, ld, st, pro);
    }
}

// Prologue that copies the twiddle tables into LDS (needed from stage 1 on):
// one entry per thread is fetched early, any beyond the block size (small
// blocks only) are copied by a loop at commit.
template <typename C> struct TwiddleCopy {
    C *dst;
    const C *src;
    int n;
    struct Regs {
        C tw;
    };
    __device__ Regs fetch() const
    {
        const int e = threadIdx.x;
        return Regs{src[e < n ? e : 0]};
    }
    __device__ void commit(const Regs &r) const
    {
        const int e = threadIdx.x;
        if (e < n) dst[e] = r.tw;
        for (int x = e + (int)blockDim.x; x < n; x += blockDim.x) dst[x] = src[x];
    }
};

// Workgroup id -> work item, so that each XCD (workgroups are dealt to the 8
// XCDs round-robin) takes a contiguous run of work items and neighbouring
// items share that XCD's L2.
__device__ inline int xcd_remap(int id, int total)
{
    const int q = total >> 3, rem = total & 7;
    const int x = id & 7, k = id >> 3;
    return x * q + (x < rem ? x : rem) + k;
}

// Centred mode index of FFT slot i in a length-L transform (-1: zero padding).
__device__ inline int mode_of(int i, int K, int L)
{
    const int half = K >> 1, kmax = K - 1 - half;
    if (i <= kmax) return i + half;
    if (i >= L - half) return i - L + half;
    return -1;
}

// Even rows (parity 0): x_n = c[n][m] corr_t[n] corr_p[m];
// odd rows (parity 1):   x_n = c[n][m] corr_t[n] corr_p[m] e^{2 pi i n / nft}.
// fac holds the two theta factor tables ([2][Kt] complex); cpm is corr_p of
// the thread's column, which is the same for all its jobs (the block size is
// a multiple of the column batch).
// The transformed columns are col0 .. col0 + ncols - 1 of the coefficient
// rows (all of them, or the m >= 0 half of a real field's); m counts from col0.
template <typename T> struct ThetaLoad {
    const cplx<T> *coef;  // this field, column col0 first
    const cplx<T> *fac;   // this parity's factors
    T cpm;
    int Kt, Kp, ncols, L, m0;
    int m_major;          // 1: column m's modes are contiguous ([Kp][Kt])
    // Loads are unconditional (clamped indices) so that the compiler issues
    // every element's loads before the first wait; padding slots select 0.
    __device__ cplx<T> operator()(int i, int b) const
    {
        const int m = m0 + b;
        const int a = mode_of(i, Kt, L);
        const bool live = a >= 0 && m < ncols;
        const int ac = live ? a : 0, mc = live ? m : 0;
        const cplx<T> f = fac[ac];
        const cplx<T> x = cmul(coef[m_major ? mc * Kt + ac : ac * Kp + mc], cplx<T>{f.x * cpm, f.y * cpm});
        return live ? x : cplx<T>{(T)0, (T)0};
    }
};

template <typename T> struct ThetaStore {
    cplx<T> *S;              // this field, [nft][ncols]
    const uint8_t *reached;  // LDS copy: reached[q] for output row 2q + parity
    int ncols, m0, parity;
    __device__ void operator()(int q, int b, cplx<T> v) const
    {
        const int m = m0 + b;
        const int l = 2 * q + parity;
        if (m < ncols && reached[q]) S[l * ncols + m] = v;
    }
};

// Prologue of the theta pass: the twiddle tables and this parity's row flags
// go to LDS, fetched ahead of the first stage's loads.  Flags travel four
// rows at a time: chunk c holds touched[8c .. 8c + 7] (touched is allocated
// 256-byte aligned and L is a multiple of 4), of which bytes parity,
// 2 + parity, 4 + parity and 6 + parity are rows 4c .. 4c + 3 of this
// parity.  A block has at least L / E threads, so E / 4 chunks per thread
// cover the L / 4 chunks.
template <typename C, int E> struct ThetaPro {
    static constexpr int FC = E / 4;
    C *tw_dst;
    const C *tw_src;
    int tw_n;
    uint8_t *flags_dst;
    const uint8_t *touched;
    int L, parity;
    struct Regs {
        C tw;
        uint2 fl[FC];
    };
    __device__ Regs fetch() const
    {
        Regs r;
        const int e = threadIdx.x;
        r.tw = tw_src[e < tw_n ? e : 0];
        const uint2 *src = reinterpret_cast<const uint2 *>(touched);
        const int nc = L >> 2;
#pragma unroll
        for (int k = 0; k < FC; ++k) {
            const int c = e + k * (int)blockDim.x;
            r.fl[k] = k * (int)blockDim.x < nc ? src[c < nc ? c : 0] : make_uint2(0u, 0u);
        }
        return r;
    }
    __device__ void commit(const Regs &r) const
    {
        const int e = threadIdx.x;
        if (e < tw_n) tw_dst[e] = r.tw;
        for (int x = e + (int)blockDim.x; x < tw_n; x += blockDim.x) tw_dst[x] = tw_src[x];
        const int nc = L >> 2;
        const unsigned sh = 8u * (unsigned)parity;
#pragma unroll
        for (int k = 0; k < FC; ++k) {
            const int c = e + k * (int)blockDim.x;
            if (c < nc) {
                const unsigned a = (r.fl[k].x >> sh) & 0x00ff00ffu;
                const unsigned b = (r.fl[k].y >> sh) & 0x00ff00ffu;
                const unsigned lo = (a | (a >> 8)) & 0xffffu, hi = (b | (b >> 8)) & 0xffffu;
                reinterpret_cast<uint32_t *>(flags_dst)[c] = lo | (hi << 16);
            }
        }
    }
};

template <typename T> constexpr int theta_max_threads() { return sizeof(T) == 4 ? 1024 : 512; }
// row flags of one parity, rounded up to 16 bytes to keep the data aligned
constexpr int theta_flag_bytes(int L) { return (L + 15) & ~15; }

// One workgroup per (field, batch of B phi modes, output parity); item is
// the work item of this workgroup.  The work item order puts the two
// parities of a batch next to each other, so that the XCD-aware mapping runs
// them on the same XCD and the second read of the coefficient batch hits its
// L2.
//
// FB: the column batch at compile time (0: fp.theta_batch at run time); a
// fixed batch turns the per-element LDS address arithmetic into constants.
template <typename T, int LOGL, int E, int FB>
__device__ inline void theta_body(int item, const cplx<T> *__restrict__ coeffs, const cplx<T> *__restrict__ fac_t,
                                  const T *__restrict__ corr_p, const cplx<T> *__restrict__ tws,
                                  const uint8_t *__restrict__ touched, cplx<T> *__restrict__ S,
                                  const FFTParams &fp)
{
    // 16-byte aligned whatever size the static LDS arrays have
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int L = 1 << LOGL;
    cplx<T> *tw = reinterpret_cast<cplx<T> *>(smem_raw);
    uint8_t *flags = reinterpret_cast<uint8_t *>(tw + tw_lds_len(L));
    cplx<T> *s = reinterpret_cast<cplx<T> *>(flags + theta_flag_bytes(L));
    const int B = FB > 0 ? FB : fp.theta_batch;
    const int logB = FB > 0 ? __builtin_ctz(FB > 0 ? FB : 1) : fp.log_theta_batch;
    const int ntiles = (fp.ncols + B - 1) / B;
    const int parity = item & 1;
    const int tile = item >> 1;
    const int f = tile / ntiles;
    const int m0 = (tile - f * ntiles) * B;
    const int mt = m0 + ((int)threadIdx.x & (B - 1));
    const T cpm = corr_p[fp.col0 + (mt < fp.ncols ? mt : 0)];
    ThetaLoad<T> ld{coeffs + (int64_t)f * fp.Kt * fp.Kp + (fp.m_major ? (int64_t)fp.col0 * fp.Kt : fp.col0),
                    fac_t + parity * fp.Kt, cpm, fp.Kt, fp.Kp, fp.ncols, L, m0, fp.m_major};
    ThetaStore<T> st{S + (int64_t)f * fp.nft * fp.ncols, flags, fp.ncols, m0, parity};
    ThetaPro<cplx<T>, E> pro{tw, tws, tw_lds_len(L), flags, touched, L, parity};
    fft_stages<T, LOGL, 0, E, true>(s, logB, B, 1, tw, ld, st, pro);
}

template <typename T, int LOGL, int E, int FB>
__global__ __launch_bounds__(theta_max_threads<T>()) void k_theta_pass(
    const cplx<T> *__restrict__ coeffs, const cplx<T> *__restrict__ fac_t,
    const T *__restrict__ corr_p, const cplx<T> *__restrict__ tws,
    const uint8_t *__restrict__ touched, cplx<T> *__restrict__ S, FFTParams fp)
{
    theta_body<T, LOGL, E, FB>(xcd_remap(blockIdx.x, gridDim.x), coeffs, fac_t, corr_p, tws, touched, S, fp);
}

// Members of a group class share every shape parameter, so member j owns
// work items [j * per, (j + 1) * per) of the class grid (per even: the two
// parities of a batch stay with one member and one XCD).
template <typename T, int LOGL, int E, int FB>
__global__ __launch_bounds__(theta_max_threads<T>()) void k_theta_group(const ThetaJob *__restrict__ jobs,
                                                                        int per)
{
    const int item = xcd_remap(blockIdx.x, gridDim.x);
    const int j = item / per;
    const ThetaJob J = jobs[j];
    theta_body<T, LOGL, E, FB>(item - j * per, (const cplx<T> *)J.coeffs, (const cplx<T> *)J.fac_t,
                           (const T *)J.corr_p, (const cplx<T> *)J.tws, J.touched, (cplx<T> *)J.S, J.fp);
}

template <typename T> struct PhiStore {
    cplx<T> *grid;  // this field, [nft][N] (N: the transform length)
    const uint8_t *touched;
    int N, l0;
    __device__ void operator()(int o, int b, cplx<T> v) const
    {
        const int l = l0 + b;
        if (touched[l]) grid[(int64_t)l * N + o] = v;
    }
};

template <typename T> struct PhiLoad {
    const cplx<T> *S;  // this field, [nft][Kp]
    int Kp, nfp, l0;
    __device__ cplx<T> operator()(int i, int b) const
    {
        const int a = mode_of(i, Kp, nfp);
        const cplx<T> v = S[(int64_t)(l0 + b) * Kp + (a < 0 ? 0 : a)];
        return a < 0 ? cplx<T>{(T)0, (T)0} : v;
    }
};

// Complex-to-real phi transform of a real field's row.  The row's modes are
// X[m], m = 0 .. M (M = ncols - 1 < nfp / 4), and X[-m] = conj X[m]; the
// real row x[l] = sum_m X[m] e^{2 pi i m l / nfp} comes out of one complex
// transform of length N2 = nfp / 2 as z[j] = x[2j] + i x[2j + 1], whose
// input is Z[k] = (X[k] + X[k + N2]) + i (X[k] - X[k + N2]) e^{2 pi i k / nfp}
// (even and odd samples, interleaved).  With the band limit only one of the
// two terms is non-zero:
//   Z[k]      = X[k] (1 + i e^{2 pi i k / nfp})              k <= M
//   Z[N2 - k] = conj(X[k]) (1 + i e^{-2 pi i k / nfp})      1 <= k <= M
// and zero between.  X[0] enters by its real part, so the row is the real
// part of the series of the m >= 0 half with the m > 0 terms doubled (for a
// real field: the series).  tab[k] = e^{2 pi i k / nfp}, k <= M.
template <typename T> struct PhiLoadC2R {
    const cplx<T> *S;    // this field, [nft][ncols]
    const cplx<T> *tab;
    int ncols, N2, l0;
    __device__ cplx<T> operator()(int k, int b) const
    {
        const int M = ncols - 1;
        const bool lo = k <= M, hi = k >= N2 - M && k > 0;
        const int m = lo ? k : (hi ? N2 - k : 0);
        const cplx<T> x = S[(int64_t)(l0 + b) * ncols + m];
        const cplx<T> e = tab[m];
        // lo: X (1 - s, c); hi: conj(X) (1 + s, c), with e = (c, s)
        const cplx<T> xm = lo ? cplx<T>{x.x, k == 0 ? (T)0 : x.y} : cplx<T>{x.x, -x.y};
        const cplx<T> f = lo ? cplx<T>{(T)1 - e.y, e.x} : cplx<T>{(T)1 + e.y, e.x};
        const cplx<T> z = cmul(xm, f);
        return (lo || hi) ? z : cplx<T>{(T)0, (T)0};
    }
};

// One workgroup per (field, batch of B reached theta rows); blk is the
// workgroup's index in the stage.  LOGN: log2 of the transform length (nfp,
// or nfp / 2 for the complex-to-real rows of real fields).
template <typename T, int LOGN, int E, bool C2R>
__device__ inline void phi_body(int blk, const cplx<T> *__restrict__ S, const cplx<T> *__restrict__ tws,
                                const cplx<T> *__restrict__ c2r, const uint8_t *__restrict__ touched,
                                cplx<T> *__restrict__ grid, const FFTParams &fp)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int N = 1 << LOGN;
    cplx<T> *tw = reinterpret_cast<cplx<T> *>(smem_raw);
    cplx<T> *s = tw + tw_lds_len(N);
    const int nrb = fp.nft / fp.phi_batch;
    const int f = blk / nrb;
    const int l0 = (blk - f * nrb) * fp.phi_batch;
    // skip the workgroup when none of its rows is reached by any point
    int any = 0;
    for (int b = 0; b < fp.phi_batch; ++b) any |= touched[l0 + b];
    if (!any) return;
    PhiStore<T> st{grid + (int64_t)f * fp.nft * N, touched, N, l0};
    TwiddleCopy<cplx<T>> pro{tw, tws, tw_lds_len(N)};
    if constexpr (C2R) {
        PhiLoadC2R<T> ld{S + (int64_t)f * fp.nft * fp.ncols, c2r, fp.ncols, N, l0};
        fft_stages<T, LOGN, 0, E, false>(s, fp.log_phi_batch, 1, lds_seq_len(N), tw, ld, st, pro);
    } else {
        PhiLoad<T> ld{S + (int64_t)f * fp.nft * fp.ncols, fp.ncols, N, l0};
        fft_stages<T, LOGN, 0, E, false>(s, fp.log_phi_batch, 1, lds_seq_len(N), tw, ld, st, pro);
    }
}

template <typename T, int LOGN, int E, bool C2R>
__global__ __launch_bounds__(256) void k_phi_pass(const cplx<T> *__restrict__ S,
                                                  const cplx<T> *__restrict__ tws,
                                                  const cplx<T> *__restrict__ c2r,
                                                  const uint8_t *__restrict__ touched,
                                                  cplx<T> *__restrict__ grid, FFTParams fp)
{
    phi_body<T, LOGN, E, C2R>((int)blockIdx.x, S, tws, c2r, touched, grid, fp);
}

// Member j of a group class owns workgroups [j * per, (j + 1) * per).
template <typename T, int LOGN, int E, bool C2R>
__global__ __launch_bounds__(256) void k_phi_group(const PhiJob *__restrict__ jobs, int per)
{
    const int j = (int)blockIdx.x / per;
    const PhiJob J = jobs[j];
    phi_body<T, LOGN, E, C2R>((int)blockIdx.x - j * per, (const cplx<T> *)J.S, (const cplx<T> *)J.tws,
                              (const cplx<T> *)J.c2r, J.touched, (cplx<T> *)J.grid, J.fp);
}

constexpr int kElemsPerThread = 16;

// Column batch given a compile-time instance for transforms of length
// 2^LOGL: the batch the plan takes for the large lengths (0: none).
template <typename T, int LOGL> constexpr int theta_fixed_batch()
{
    if (LOGL == 11) return sizeof(T) == 4 ? 4 : 2;
    if (LOGL == 10) return sizeof(T) == 4 ? 8 : 4;
    return 0;
}

// jobs == nullptr: one plan (the pointer arguments); otherwise n_members
// members of one group class described by jobs (device memory).
template <typename T, int LOGL, int FB>
static hipError_t launch_theta_b(const FFTParams &fp, const void *coeffs, const void *fac_t,
                                 const void *corr_p, const void *tws_t, const uint8_t *touched,
                                 void *S, const ThetaJob *jobs, int n_members, hipStream_t s)
{
    const int L = 1 << LOGL;
    const int ept = fp.theta_ept == 8 ? 8 : kElemsPerThread;
    const int threads = L * fp.theta_batch / ept;
    if (threads < 1 || threads > theta_max_threads<T>() || threads % fp.theta_batch != 0 ||
        (FB > 0 && fp.theta_batch != FB))
        return hipErrorInvalidConfiguration;
    const size_t lds = sizeof(cplx<T>) * ((size_t)lds_seq_len(L) * fp.theta_batch + tw_lds_len(L)) +
                       theta_flag_bytes(L);
    const int ntiles = (fp.ncols + fp.theta_batch - 1) / fp.theta_batch;
    const int per = 2 * ntiles * fp.n_fields;
    if (jobs) {
        auto kern = ept == 8 ? k_theta_group<T, LOGL, 8, FB> : k_theta_group<T, LOGL, kElemsPerThread, FB>;
        if (lds > 65536)
            (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(kern, dim3(per * n_members), dim3(threads), lds, s, jobs, per);
    } else {
        auto kern = ept == 8 ? k_theta_pass<T, LOGL, 8, FB> : k_theta_pass<T, LOGL, kElemsPerThread, FB>;
        if (lds > 65536)
            (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(kern, dim3(per), dim3(threads), lds, s, (const cplx<T> *)coeffs,
                           (const cplx<T> *)fac_t, (const T *)corr_p, (const cplx<T> *)tws_t, touched,
                           (cplx<T> *)S, fp);
    }
    return hipGetLastError();
}

template <typename T, int LOGL>
static hipError_t launch_theta_t(const FFTParams &fp, const void *coeffs, const void *fac_t,
                                 const void *corr_p, const void *tws_t, const uint8_t *touched,
                                 void *S, const ThetaJob *jobs, int n_members, hipStream_t s)
{
    constexpr int FB = theta_fixed_batch<T, LOGL>();
    if constexpr (FB > 0) {
        if (fp.theta_batch == FB)
            return launch_theta_b<T, LOGL, FB>(fp, coeffs, fac_t, corr_p, tws_t, touched, S, jobs, n_members, s);
    }
    return launch_theta_b<T, LOGL, 0>(fp, coeffs, fac_t, corr_p, tws_t, touched, S, jobs, n_members, s);
}

template <typename T, int LOGN, bool C2R>
static hipError_t launch_phi_t(const FFTParams &fp, const void *S, const void *tw_p, const void *c2r,
                               const uint8_t *touched, void *grid, const PhiJob *jobs, int n_members,
                               hipStream_t s)
{
    const int N = 1 << LOGN;
    const int ept = fp.phi_ept == 8 ? 8 : kElemsPerThread;
    const int threads = N * fp.phi_batch / ept;
    if (threads < 1 || threads > 256) return hipErrorInvalidConfiguration;
    const size_t lds = sizeof(cplx<T>) * ((size_t)lds_seq_len(N) * fp.phi_batch + tw_lds_len(N));
    const int per = (fp.nft / fp.phi_batch) * fp.n_fields;
    if (jobs) {
        auto kern = ept == 8 ? k_phi_group<T, LOGN, 8, C2R> : k_phi_group<T, LOGN, kElemsPerThread, C2R>;
        if (lds > 65536)
            (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(kern, dim3(per * n_members), dim3(threads), lds, s, jobs, per);
    } else {
        auto kern = ept == 8 ? k_phi_pass<T, LOGN, 8, C2R> : k_phi_pass<T, LOGN, kElemsPerThread, C2R>;
        if (lds > 65536)
            (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(kern, dim3(per), dim3(threads), lds, s, (const cplx<T> *)S, (const cplx<T> *)tw_p,
                           (const cplx<T> *)c2r, touched, (cplx<T> *)grid, fp);
    }
    return hipGetLastError();
}

template <typename T>
static hipError_t theta_dispatch(const FFTParams &fp, const void *coeffs, const void *fac_t,
                                 const void *corr_p, const void *tws_t, const uint8_t *touched,
                                 void *S, const ThetaJob *jobs, int n_members, hipStream_t s)
{
    switch (fp.log_nft - 1) {
#define NUFFT2_L(X)                                                                                        \
    case X: return launch_theta_t<T, X>(fp, coeffs, fac_t, corr_p, tws_t, touched, S, jobs, n_members, s);
        NUFFT2_L(4) NUFFT2_L(5) NUFFT2_L(6) NUFFT2_L(7) NUFFT2_L(8) NUFFT2_L(9)
        NUFFT2_L(10) NUFFT2_L(11)
#undef NUFFT2_L
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
static hipError_t phi_dispatch(const FFTParams &fp, const void *S, const void *tw_p, const void *c2r,
                               const uint8_t *touched, void *grid, const PhiJob *jobs, int n_members,
                               hipStream_t s)
{
    if (fp.c2r) {
        switch (fp.log_phi_len) {
#define NUFFT2_N(X) case X: return launch_phi_t<T, X, true>(fp, S, tw_p, c2r, touched, grid, jobs, n_members, s);
            NUFFT2_N(4) NUFFT2_N(5) NUFFT2_N(6) NUFFT2_N(7) NUFFT2_N(8) NUFFT2_N(9) NUFFT2_N(10)
            NUFFT2_N(11)
#undef NUFFT2_N
        default: return hipErrorInvalidValue;
        }
    }
    switch (fp.log_phi_len) {
#define NUFFT2_N(X) case X: return launch_phi_t<T, X, false>(fp, S, tw_p, c2r, touched, grid, jobs, n_members, s);
        NUFFT2_N(5) NUFFT2_N(6) NUFFT2_N(7) NUFFT2_N(8) NUFFT2_N(9) NUFFT2_N(10)
        NUFFT2_N(11) NUFFT2_N(12)
#undef NUFFT2_N
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_theta_pass(int prec, const FFTParams &fp, const void *coeffs, const void *fac_t,
                             const void *corr_p, const void *tws_t, const uint8_t *rowtouched,
                             void *S, hipStream_t s)
{
    if (prec == 1) return theta_dispatch<float>(fp, coeffs, fac_t, corr_p, tws_t, rowtouched, S, nullptr, 0, s);
    return theta_dispatch<double>(fp, coeffs, fac_t, corr_p, tws_t, rowtouched, S, nullptr, 0, s);
}

hipError_t launch_phi_pass(int prec, const FFTParams &fp, const void *S, const void *tw_p, const void *c2r,
                           const uint8_t *rowtouched, void *grid, hipStream_t s)
{
    if (prec == 1) return phi_dispatch<float>(fp, S, tw_p, c2r, rowtouched, grid, nullptr, 0, s);
    return phi_dispatch<double>(fp, S, tw_p, c2r, rowtouched, grid, nullptr, 0, s);
}

hipError_t launch_theta_group(int prec, const FFTParams &fp, const ThetaJob *jobs, int n_members, hipStream_t s)
{
    if (n_members < 1 || !jobs) return hipErrorInvalidValue;
    if (prec == 1) return theta_dispatch<float>(fp, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, jobs, n_members, s);
    return theta_dispatch<double>(fp, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, jobs, n_members, s);
}

hipError_t launch_phi_group(int prec, const FFTParams &fp, const PhiJob *jobs, int n_members, hipStream_t s)
{
    if (n_members < 1 || !jobs) return hipErrorInvalidValue;
    if (prec == 1) return phi_dispatch<float>(fp, nullptr, nullptr, nullptr, nullptr, nullptr, jobs, n_members, s);
    return phi_dispatch<double>(fp, nullptr, nullptr, nullptr, nullptr, nullptr, jobs, n_members, s);
}

// ---- DFS analysis: grid values on Grid [0] -> exp-form coefficients -------
//
// Section 4 computes the standard-DFS coefficients with an FFT in phi and
// cosine / sine transforms in theta (cosine for even m, sine for odd m) and
// eq. dfs_fourier_coeffs maps them to exp form.  The same coefficients come
// from one complex transform per phi mode over the doubled theta circle:
// the glide reflection f(phi, 2 pi - theta) = f(phi + pi, theta) extends
// phi mode m of row i to row 2J - 1 - i with the factor (-1)^m, i.e. the
// even (cosine) extension for even m and the odd (sine) one for odd m.
// Both steps are forward transforms, done here as conj(FFT_+(conj x)) with
// the +i Stockham kernels; the loaders and storers do the conjugations.

// phi step: row i of field f (length L = 2J, real) -> A[f][i][m + J - 1].
template <typename T> struct AnaRowLoad {
    const T *vals;  // this field, [J][L]
    int L, i0;
    __device__ cplx<T> operator()(int k, int b) const { return {vals[(int64_t)(i0 + b) * L + k], (T)0}; }
};
// The zonal filter of section 4, when on (cut != nullptr), keeps at row i
// only the wavenumbers |m| <= cut[i] (the integer part of M_zf(theta_i)).
//
// Layout of A (one field): lb < 0, rows [J][K] (what the Gauss-Legendre
// latitude product reads); lb >= 0, column blocks [2J >> lb][J][1 << lb],
// block width = the theta step's columns per workgroup, so that each theta
// workgroup reads one contiguous run instead of short segments of J rows
// 8 K elements apart.  A blocked field takes 2J x J elements (the width is
// a power of two that divides 2J = K + 1; the last block's last slot is
// never written or read).
__device__ inline int64_t ana_index(int i, int col, int J, int K, int lb)
{
    if (lb < 0) return (int64_t)i * K + col;
    return (((int64_t)(col >> lb) * J + i) << lb) + (col & ((1 << lb) - 1));
}
template <typename T> struct AnaRowStore {
    cplx<T> *A;  // this field
    const int32_t *cut;
    int J, K, i0, lb;
    __device__ void operator()(int o, int b, cplx<T> v) const
    {
        // frequency o <-> m = o (o < J) or o - 2J (o > J); o = J (Nyquist) is dropped
        if (o == J) return;
        const int m = o < J ? o : o - 2 * J;
        const bool keep = !cut || (m < 0 ? -m : m) <= cut[i0 + b];
        A[ana_index(i0 + b, m + J - 1, J, K, lb)] = keep ? cplx<T>{v.x, -v.y} : cplx<T>{(T)0, (T)0};
    }
};

template <typename T, int LOGN, int E>
__global__ __launch_bounds__(256) void k_analysis_phi(const T *__restrict__ vals, const cplx<T> *__restrict__ tws,
                                                      const int32_t *__restrict__ cut, cplx<T> *__restrict__ A,
                                                      int J, int rows_per_wg, int log_rows_per_wg, int lb,
                                                      int64_t fstride)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int N = 1 << LOGN;  // = 2J
    cplx<T> *tw = reinterpret_cast<cplx<T> *>(smem_raw);
    cplx<T> *s = tw + tw_lds_len(N);
    const int K = 2 * J - 1;
    const int nrb = J / rows_per_wg;
    const int f = (int)blockIdx.x / nrb;
    const int i0 = ((int)blockIdx.x - f * nrb) * rows_per_wg;
    AnaRowLoad<T> ld{vals + (int64_t)f * J * N, N, i0};
    AnaRowStore<T> st{A + (int64_t)f * fstride, cut, J, K, i0, lb};
    TwiddleCopy<cplx<T>> pro{tw, tws, tw_lds_len(N)};
    fft_stages<T, LOGN, 0, E, false>(s, log_rows_per_wg, 1, lds_seq_len(N), tw, ld, st, pro);
}

// theta step: columns m0 .. m0 + B - 1 of A (the phi modes), doubled to
// length 2J with the glide sign, forward transform over theta, then the
// half-cell phase and the normalisation: ft[n][m] = Z[n] e^{-i n pi/(2J)} / (2J)^2.
template <typename T> struct AnaColLoad {
    const cplx<T> *A;  // this field, layout as for AnaRowStore
    int J, K, m0, lb;
    __device__ cplx<T> operator()(int i, int b) const
    {
        const int mi = m0 + b;
        const int mc = mi < K ? mi : K - 1;
        const int r = i < J ? i : 2 * J - 1 - i;
        const cplx<T> v = A[ana_index(r, mc, J, K, lb)];
        const bool neg = i >= J && (((mc - (J - 1)) & 1) != 0);
        const T sre = neg ? -v.x : v.x, sim = neg ? -v.y : v.y;
        return {sre, -sim};  // conj
    }
};
template <typename T> struct AnaColStore {
    cplx<T> *out;          // this field, [K][K] (rows n, or rows m when m_major)
    const cplx<T> *phase;  // [K]: e^{-i n pi/(2J)} / (2J)^2, n = -(J-1) .. J-1
    int J, K, m0, m_major;
    __device__ void operator()(int o, int b, cplx<T> v) const
    {
        const int mi = m0 + b;
        if (mi >= K || o == J) return;
        const int n = o < J ? o : o - 2 * J;
        const cplx<T> z{v.x, -v.y};  // conj back: forward transform
        const int64_t o2 = m_major ? (int64_t)mi * K + (n + J - 1) : (int64_t)(n + J - 1) * K + mi;
        out[o2] = cmul(z, phase[n + J - 1]);
    }
};

template <typename T, int LOGN, int E>
__global__ __launch_bounds__(512) void k_analysis_theta(const cplx<T> *__restrict__ A,
                                                        const cplx<T> *__restrict__ tws,
                                                        const cplx<T> *__restrict__ phase,
                                                        cplx<T> *__restrict__ out, int J, int cols_per_wg,
                                                        int log_cols_per_wg, int m_major, int lb,
                                                        int64_t fstride)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int N = 1 << LOGN;  // = 2J
    cplx<T> *tw = reinterpret_cast<cplx<T> *>(smem_raw);
    cplx<T> *s = tw + tw_lds_len(N);
    const int K = 2 * J - 1;
    const int ntiles = (K + cols_per_wg - 1) / cols_per_wg;
    const int f = (int)blockIdx.x / ntiles;
    const int m0 = ((int)blockIdx.x - f * ntiles) * cols_per_wg;
    AnaColLoad<T> ld{A + (int64_t)f * fstride, J, K, m0, lb};
    AnaColStore<T> st{out + (int64_t)f * K * K, phase, J, K, m0, m_major};
    TwiddleCopy<cplx<T>> pro{tw, tws, tw_lds_len(N)};
    fft_stages<T, LOGN, 0, E, true>(s, log_cols_per_wg, cols_per_wg, 1, tw, ld, st, pro);
}

// phi step only: rows per workgroup so that it transforms 4096 elements
template <typename T, int LOGN>
static hipError_t launch_analysis_rows_t(const AnalysisParams &ap, const void *vals, const void *tws, void *A,
                                         hipStream_t s, int lb = -1)
{
    constexpr int N = 1 << LOGN;
    const int J = N / 2;
    int rb = 4096 / N;
    if (rb > J) rb = J;
    int lrb = 0;
    while ((1 << lrb) < rb) ++lrb;
    const int threads = N * rb / kElemsPerThread;
    if (threads < 1 || threads > 256) return hipErrorInvalidConfiguration;
    const size_t lds = sizeof(cplx<T>) * ((size_t)lds_seq_len(N) * rb + tw_lds_len(N));
    auto kern = k_analysis_phi<T, LOGN, kElemsPerThread>;
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(kern, dim3((J / rb) * ap.n_fields), dim3(threads), lds, s, (const T *)vals,
                       (const cplx<T> *)tws, ap.zonal_cut, (cplx<T> *)A, J, rb, lrb, lb,
                       lb < 0 ? (int64_t)J * (2 * J - 1) : (int64_t)2 * J * J);
    return hipGetLastError();
}

template <typename T, int LOGN>
static hipError_t launch_analysis_t(const AnalysisParams &ap, const void *vals, const void *tws, const void *phase,
                                    void *A, void *out, hipStream_t s)
{
    constexpr int N = 1 << LOGN;
    const int J = N / 2;
    // theta step: columns per workgroup so that a workgroup has 64..512
    // threads and at most 80 KB of LDS (two workgroups per CU); wider tiles
    // make longer row segments of the output
    int cb = 1;
    while (N * cb / kElemsPerThread < 64) cb *= 2;
    while (cb < 16 && N * cb * 2 / kElemsPerThread <= 512 &&
           sizeof(cplx<T>) * ((size_t)lds_seq_len(N) * cb * 2 + tw_lds_len(N)) <= 80 * 1024)
        cb *= 2;
    int lcb = 0;
    while ((1 << lcb) < cb) ++lcb;
    const int threads = N * cb / kElemsPerThread;
    if (threads < 1 || threads > 512 || threads % cb != 0 || cb > N) return hipErrorInvalidConfiguration;
    const size_t lds = sizeof(cplx<T>) * ((size_t)lds_seq_len(N) * cb + tw_lds_len(N));
    // A in column blocks of the theta tile's width (one column, where the
    // tile is one column wide, stays in rows: a column-major A would make
    // the phi step's stores single elements J apart)
    const int lb = cb >= 2 ? lcb : -1;
    const int64_t fstride = lb < 0 ? (int64_t)J * (2 * J - 1) : (int64_t)2 * J * J;
    {
        const hipError_t e = launch_analysis_rows_t<T, LOGN>(ap, vals, tws, A, s, lb);
        if (e != hipSuccess) return e;
    }
    {
        auto kern = k_analysis_theta<T, LOGN, kElemsPerThread>;
        if (lds > 65536)
            (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        const int K = 2 * J - 1;
        const int ntiles = (K + cb - 1) / cb;
        hipLaunchKernelGGL(kern, dim3(ntiles * ap.n_fields), dim3(threads), lds, s, (const cplx<T> *)A,
                           (const cplx<T> *)tws, (const cplx<T> *)phase, (cplx<T> *)out, J, cb, lcb, ap.m_major,
                           lb, fstride);
    }
    return hipGetLastError();
}

template <typename T>
static hipError_t analysis_dispatch(const AnalysisParams &ap, const void *vals, const void *tws, const void *phase,
                                    void *A, void *out, hipStream_t s)
{
    switch (ap.log_len) {
#define NUFFT2_A(X) case X: return launch_analysis_t<T, X>(ap, vals, tws, phase, A, out, s);
        NUFFT2_A(5) NUFFT2_A(6) NUFFT2_A(7) NUFFT2_A(8) NUFFT2_A(9) NUFFT2_A(10) NUFFT2_A(11) NUFFT2_A(12)
#undef NUFFT2_A
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_analysis(int prec, const AnalysisParams &ap, const void *vals, const void *tws, const void *phase,
                           void *A, void *out, hipStream_t s)
{
    if (prec == 1) return analysis_dispatch<float>(ap, vals, tws, phase, A, out, s);
    return analysis_dispatch<double>(ap, vals, tws, phase, A, out, s);
}

template <typename T>
static hipError_t analysis_rows_dispatch(const AnalysisParams &ap, const void *vals, const void *tws, void *A,
                                         hipStream_t s)
{
    switch (ap.log_len) {
#define NUFFT2_A(X) case X: return launch_analysis_rows_t<T, X>(ap, vals, tws, A, s);
        NUFFT2_A(5) NUFFT2_A(6) NUFFT2_A(7) NUFFT2_A(8) NUFFT2_A(9) NUFFT2_A(10) NUFFT2_A(11) NUFFT2_A(12)
#undef NUFFT2_A
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_analysis_rows(int prec, const AnalysisParams &ap, const void *vals, const void *tws, void *A,
                                hipStream_t s)
{
    if (prec == 1) return analysis_rows_dispatch<float>(ap, vals, tws, A, s);
    return analysis_rows_dispatch<double>(ap, vals, tws, A, s);
}

}  // namespace nufft2
