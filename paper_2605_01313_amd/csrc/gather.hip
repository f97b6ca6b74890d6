// ES gather launches for FP32 plans, and the vector rotation; the kernels
// are in gather_kernels.hpp (FP64 launches in gather_f64.hip, a separate
// translation unit so that the two precisions compile in parallel).
#include "gather_kernels.hpp"

namespace nufft2 {

hipError_t launch_gather_f64(const GatherParams &gp, const void *grid, const void *rec, const int32_t *perm,
                             const int32_t *binlist, void *out, const GatherJob *jobs, int n_members, hipStream_t s);

hipError_t launch_gather(int prec, const GatherParams &gp, const void *grid, const void *rec,
                         const int32_t *perm, const int32_t *binlist, void *out, hipStream_t s)
{
    if (gp.n_pts == 0) return hipSuccess;
    if (prec == 1) return launch_prec<float>(gp, grid, rec, perm, binlist, out, nullptr, 0, s);
    return launch_gather_f64(gp, grid, rec, perm, binlist, out, nullptr, 0, s);
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
    if (prec == 1) return launch_prec<float>(gp, nullptr, nullptr, nullptr, nullptr, nullptr, jobs, n_members, s);
    return launch_gather_f64(gp, nullptr, nullptr, nullptr, nullptr, nullptr, jobs, n_members, s);
}

}  // namespace nufft2
