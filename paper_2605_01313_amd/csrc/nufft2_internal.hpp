// Internal declarations shared by the host plan code and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nufft2 {

template <typename T> struct cplx_sel;
template <> struct cplx_sel<float> { using type = float2; };
template <> struct cplx_sel<double> { using type = double2; };
template <typename T> using cplx = typename cplx_sel<T>::type;

// One departure point after setpts: the first tap's fine-grid cell in each
// direction (already reduced modulo the grid size) and the offset
// v = (t - i0) - floor(w/2), with t the point's coordinate in grid units.
template <typename T> struct PointRec;
template <> struct alignas(16) PointRec<float> { int32_t it, ip; float vt, vp; };
template <> struct alignas(8) PointRec<double> { int32_t it, ip; double vt, vp; };

// Coordinate split parameters (one per direction).
struct AxisParams {
    double to_grid;   // nf / (2 pi)
    double inv_nf;    // 1 / nf (exact)
    int32_t nf;       // fine grid size (power of two)
    int32_t tile;     // bin tile size along this axis (power of two)
};

struct SetptsParams {
    AxisParams th, ph;
    int32_t w;
    int32_t nbins_phi;
    int64_t n;
    // vector rotation: the arrival points (caller's order) and the output
    // (p, q) pairs in sorted order (plan precision); all null otherwise
    const double *phi_a, *theta_a;
    void *pq;
};

// The bin list of a plan: nbins + 1 int32 (the non-empty bins in order, then
// their number), padded to 16 bytes, then nbins int4 {bin, first record,
// record count, 0} for the non-empty bins in the same order.
__host__ __device__ inline int64_t bin_items_offset(int64_t nbins) { return (nbins + 1 + 3) & ~(int64_t)3; }
__host__ __device__ inline int4 *bin_items(int32_t *binlist, int64_t nbins)
{
    return reinterpret_cast<int4 *>(binlist + bin_items_offset(nbins));
}
__host__ __device__ inline const int4 *bin_items(const int32_t *binlist, int64_t nbins)
{
    return reinterpret_cast<const int4 *>(binlist + bin_items_offset(nbins));
}
// The gather launches one workgroup per slot, 8 * ceil(nbins / 8) of them.
// kDealtMaxBins: the bins of one scan pass.
constexpr int64_t kDealtMaxBins = 8192;
__host__ __device__ inline int64_t gather_slots(int64_t nbins) { return 8 * ((nbins + 7) / 8); }
__host__ __device__ inline int4 *bin_dealt(int32_t *binlist, int64_t nbins) { return bin_items(binlist, nbins) + nbins; }
__host__ __device__ inline const int4 *bin_dealt(const int32_t *binlist, int64_t nbins)
{
    return bin_items(binlist, nbins) + nbins;
}
inline size_t binlist_bytes(int64_t nbins)
{
    return sizeof(int32_t) * (size_t)bin_items_offset(nbins) + sizeof(int4) * (size_t)(nbins + gather_slots(nbins));
}

// ---- launchers (each returns the hipError_t of its launch) ----
hipError_t launch_setpts(int prec, const SetptsParams &sp, const double *phi, const double *theta,
                         int32_t *bincount, int32_t *binstart, int32_t *binlist, int64_t nbins,
                         int2 *keyrank,
                         uint8_t *rowmark, uint8_t *rowtouched, void *rec, int32_t *perm,
                         int32_t *flags, int4 *stage, int2 *passtot, int32_t *lstart, hipStream_t s);
// Workspace of the side-by-side scan passes for plans of more than
// kDealtMaxBins bins: stage holds nbins int4, lstart nbins int32, passtot
// one int2 per pass.
inline int64_t scan_passes(int64_t nbins) { return (nbins + kDealtMaxBins - 1) / kDealtMaxBins; }

// One member of a group for the setpts kernels (device memory; the
// pointers as in launch_setpts).  Its n_pts points are point blocks
// block_begin .. block_begin + ceil(n_pts / 256) - 1 of the group launch.
struct SetptsJob {
    const double *phi, *theta;
    SetptsParams sp;
    int32_t *bincount, *binstart, *binlist;
    int64_t nbins;
    int2 *keyrank;
    uint8_t *rowmark, *rowtouched;
    void *rec;
    int32_t *perm, *flags;
    int32_t block_begin, pad;
};
// All members of one precision: point kernels over n_blocks blocks
// (job_of_block: member of each block), the scan one workgroup per member.
hipError_t launch_setpts_group(int prec, const SetptsJob *jobs, int n_members, const int32_t *job_of_block,
                               int n_blocks, hipStream_t s);

struct FFTParams {
    int32_t Kt, Kp;       // modes
    int32_t nft, nfp;     // fine grid
    int32_t log_nft, log_nfp;
    int32_t n_fields;
    int32_t theta_batch, log_theta_batch;   // columns per theta-pass workgroup
    int32_t phi_batch, log_phi_batch;       // rows per phi-pass workgroup
    int32_t theta_ept, phi_ept;             // elements per thread in each pass: 8 or 16
    // Columns the theta pass transforms: coefficient columns col0 ..
    // col0 + ncols - 1, written to S rows of ncols entries.  Complex plans:
    // all Kp columns.  Real-field (Hermitian) plans: the m >= 0 half
    // (col0 = Kp / 2, ncols = Kp / 2 + 1), and the phi pass is a
    // complex-to-real transform of length nfp done as a complex transform of
    // length nfp / 2 (c2r = 1), whose output is the real grid row.
    int32_t col0, ncols;
    int32_t c2r;
    int32_t log_phi_len;                    // log2 of the phi-pass transform length
    // 1: the coefficients are stored m-major ([F][Kp][Kt]: each column's
    // Kt modes contiguous), so the theta pass reads whole columns
    int32_t m_major;
};

// fac_t: complex [2][Kt]: corr_t[a], then corr_t[a] e^{2 pi i n / nft}
// (n = a - Kt/2); corr_p: real [Kp]; tws_t / tws_p: twiddle tables of the
// nft/2- and nfp-point transforms (64 low entries, then the high entries).
hipError_t launch_theta_pass(int prec, const FFTParams &fp, const void *coeffs, const void *fac_t,
                             const void *corr_p, const void *tws_t, const uint8_t *rowtouched,
                             void *S, hipStream_t s);
// c2r: for fp.c2r, the table e^{2 pi i k / nfp}, k < fp.ncols (complex, plan
// precision), else unused.
hipError_t launch_phi_pass(int prec, const FFTParams &fp, const void *S, const void *tws_p, const void *c2r,
                           const uint8_t *rowtouched, void *grid, hipStream_t s);

// One member of a group class for the theta / phi passes (device memory;
// the pointers as in launch_theta_pass / launch_phi_pass).  Members of a
// class share every FFTParams field.
struct ThetaJob {
    const void *coeffs, *fac_t, *corr_p, *tws;
    const uint8_t *touched;
    void *S;
    FFTParams fp;
};
struct PhiJob {
    const void *S, *tws, *c2r;
    const uint8_t *touched;
    void *grid;
    FFTParams fp;
};
hipError_t launch_theta_group(int prec, const FFTParams &fp, const ThetaJob *jobs, int n_members, hipStream_t s);
hipError_t launch_phi_group(int prec, const FFTParams &fp, const PhiJob *jobs, int n_members, hipStream_t s);

struct GatherParams {
    int32_t nft, nfp;
    int32_t tile_t, tile_p;
    int32_t nbins_phi;
    int64_t nbins;
    int32_t w;
    double beta;
    int32_t n_fields;
    int32_t fields_per_pass;   // fields staged in LDS together (1..4)
    int32_t tile_pitch;        // LDS row pitch of a staged patch, in elements (>= tile_p + w - 1)
    int64_t n_pts;
    int32_t real_output;
    int32_t real_grid;         // 1: the fine grid is real (Hermitian plans); the output is real
    // The tap weights as polynomials in the point's centred offset, lowest
    // degree first: FP32 plans with w >= kPolyMinW, FP32 table
    // [w][kPolyCoefs]; FP64 plans with w >= kPolyMinW64, FP64 table
    // [w][kPolyCoefs64] whose edge rows (taps 0 and w - 1, evaluated
    // directly) are unused.  nullptr: direct evaluation.
    const void *wpoly;
    // vector rotation: the (p, q) pair of each sorted point (plan
    // precision) and the fields (u, v) it rotates, in one gather pass;
    // pq == nullptr: none
    const void *pq;
    int32_t rot_u, rot_v;
};
constexpr int kPolyCoefs = 9;
constexpr int kPolyMinW = 7;
constexpr int kPolyCoefs64 = 15;
constexpr int kPolyMinW64 = 7;

// binlist holds the non-empty bins in increasing order and their number in
// entry nbins; after it (16-byte aligned, see bin_items) one int4 per
// non-empty bin in the same order: {bin, first record, record count, 0}.
// Gather workgroups are dealt to the 8 XCDs round-robin; workgroup blk
// takes entry (blk & 7) * per + (blk >> 3), per = ceil(n / 8) for n
// non-empty bins, so each XCD runs a contiguous eighth of them in bin
// order.  bin_dealt then holds one int4 per workgroup: the entry it takes,
// or all zero, so the gather finds its bin with one load instead of two.
// The scan writes it from LDS for plans of at most kDealtMaxBins bins (one
// pass), the scatter's threads for larger plans.
hipError_t launch_gather(int prec, const GatherParams &gp, const void *grid, const void *rec,
                         const int32_t *perm, const int32_t *binlist, void *out, hipStream_t s);

// One member of a group class for the gather (device memory).  Members of a
// class share every GatherParams field except n_pts.
struct GatherJob {
    const void *grid, *rec;
    const int32_t *perm, *binlist;
    void *out;
    GatherParams gp;
};
hipError_t launch_gather_group(int prec, const GatherParams &gp, const GatherJob *jobs, int n_members,
                               hipStream_t s);

// Rotation of a vector field (u, v) at departure points into the arrival
// frame (section 3, matrix Q), in place; comps = 2 for complex values, 1 for
// real; u and v point at the fields' [n] values.
hipError_t launch_rotate_uv(int prec, void *u, void *v, int comps, int64_t n, const double *phi_a,
                            const double *theta_a, const double *phi_d, const double *theta_d, hipStream_t s);

// DFS analysis of fields on Grid [0] (J latitudes, 2J longitudes, J a power
// of two, 16 <= J <= 2048): vals [F][J][2J] real -> A [F][J][2J-1] (phi
// modes) -> out [F][2J-1][2J-1] exp-form coefficients.  tws: twiddle tables
// of the 2J-point transform; phase: [2J-1] complex e^{-i n pi/(2J)} / (2J)^2.
struct AnalysisParams {
    int32_t J, log_len;  // log_len = log2(2J)
    int32_t n_fields;
    const int32_t *zonal_cut;  // [J] kept |m| per row (device), or nullptr: no zonal filter
    int32_t m_major;           // 1: output [F][K][K] with mode m outer (nufft2_exec's m-major layout)
};
hipError_t launch_analysis(int prec, const AnalysisParams &ap, const void *vals, const void *tws, const void *phase,
                           void *A, void *out, hipStream_t s);
// The phi step alone: A[f][i][m + J - 1] = sum_k vals[f][i][k] e^{-i m pi k / J}
// (unnormalised), |m| <= J - 1, with the zonal filter when ap.zonal_cut is set.
hipError_t launch_analysis_rows(int prec, const AnalysisParams &ap, const void *vals, const void *tws, void *A,
                                hipStream_t s);

// Gauss-Legendre latitude step: for each field and each parity p of m, the
// coefficient columns inv[p] (J x J, row-major: coefficient index x sample)
// times the phi-step samples A[f][j][m + J - 1] of the m of parity p, scaled
// by 1/(2J) and written in exp form to out[f][n + J][m + J - 1]
// ([F][2J+1][2J-1] complex): even m -> cos(n theta), n = 0..J-1; odd m ->
// sin(n theta), n = 1..J.
hipError_t launch_gl_latitude(int prec, int J, int n_fields, const void *inv, const void *A, void *out,
                              hipStream_t s);

}  // namespace nufft2
