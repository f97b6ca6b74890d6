// Plan state shared by the host sources of the library (not part of the C ABI).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "nufft2.h"
#include "nufft2_internal.hpp"

struct nufft2_plan_s {
    int prec = 0;
    int64_t Kt = 0, Kp = 0;
    int F = 0;
    int w = 0;
    double beta = 0;
    int nft = 0, nfp = 0;
    int tile_t = 0, tile_p = 0;
    int nbins_t = 0, nbins_p = 0;
    int64_t nbins = 0;
    int real_output = 0;
    int hermitian = 0;      // real-field plan: m >= 0 half, real fine grid
    int64_t ncols = 0;      // columns through the theta pass (Kp, or Kp / 2 + 1)
    int fields_per_pass = 1;
    int tile_pitch = 0;  // gather patch row pitch in LDS (elements)
    hipStream_t stream = nullptr;
    int device = 0;
    size_t csize = 0;  // bytes per complex
    size_t rsize = 0;  // bytes per real
    size_t gsize = 0;  // bytes per fine-grid element (complex, or real for real-field plans)
    nufft2::FFTParams fp{};

    // device workspaces
    void *corr_t = nullptr, *corr_p = nullptr;
    void *tw_t = nullptr, *tw_p = nullptr;  // two-level twiddle tables
    void *twist_t = nullptr;                // [2][Kt]: corr_t[a], corr_t[a] e^{2 pi i n / nft}
    void *S = nullptr, *grid = nullptr;
    void *c2r = nullptr;    // real-field plans: e^{2 pi i k / nfp}, k < ncols
    float *wpoly = nullptr; // tap-weight polynomials (FP32 w >= kPolyMinW, FP64 w >= kPolyMinW64)
    int32_t *bincount = nullptr, *binstart = nullptr;
    int32_t *binlist = nullptr;  // non-empty bins in order, their number last
    uint8_t *rowmark = nullptr, *rowtouched = nullptr;
    int32_t *flags = nullptr;
    int4 *stage = nullptr;    // side-by-side scan passes (more bins than one pass)
    int2 *passtot = nullptr;
    int32_t *lstart = nullptr;
    // point workspaces (grown by setpts)
    int64_t pts_cap = 0;
    int2 *keyrank = nullptr;
    void *rec = nullptr;
    int32_t *perm = nullptr;
    // vector rotation (nufft2_setpts_vector): the (p, q) pair of each sorted
    // point (plan precision, pq_cap points) and the rotated fields (u, v);
    // rot_u < 0: no rotation (plain nufft2_setpts, group setpts)
    void *pq = nullptr;
    int64_t pq_cap = 0;
    int32_t rot_u = -1, rot_v = -1;

    int64_t n_pts = -1;
    size_t ws_bytes = 0;
    hipError_t last_err = hipSuccess;

    // stage timing
    uint32_t prof_mask = 0;
    struct Bracket { int stage; hipEvent_t a, b; };
    std::vector<Bracket> prof_pending;
    std::vector<hipEvent_t> prof_pool;
};

namespace nufft2 {

// Grow the plan's point workspaces to hold n points (waits for the plan's
// stream before freeing smaller ones).  NUFFT2_OK, ERR_ALLOC or ERR_HIP.
nufft2_status plan_reserve_points(nufft2_plan_s *p, int64_t n);
// Kernel parameters of the plan's setpts for n points and of its gather.
SetptsParams plan_setpts_params(const nufft2_plan_s *p, int64_t n);
GatherParams plan_gather_params(const nufft2_plan_s *p);
// Elements per thread and phi-pass rows per workgroup (fp's theta_ept,
// phi_ept, phi_batch, log_phi_batch) for `members` plans of p's shape
// launched at once; fp's other fields are p's.
void fft_launch_shape(const nufft2_plan_s *p, int64_t members, nufft2::FFTParams &fp);

}  // namespace nufft2
