// ES gather launches for FP64 plans (kernels in gather_kernels.hpp).
#include "gather_kernels.hpp"

namespace nufft2 {

hipError_t launch_gather_f64(const GatherParams &gp, const void *grid, const void *rec, const int32_t *perm,
                             const int32_t *binlist, void *out, const GatherJob *jobs, int n_members, hipStream_t s)
{
    return launch_prec<double>(gp, grid, rec, perm, binlist, out, jobs, n_members, s);
}

}  // namespace nufft2
