"""Type-2 NUFFT interpolation of double-Fourier-sphere fields to departure points,
for one AMD Instinct MI355X (gfx950).

The computation lives in libnufft2.so (HIP kernels behind the C ABI of
include/nufft2.h); `nufft2` is its Python binding.
"""
from .nufft2 import (NUFFT2_FP32, NUFFT2_FP64, Analysis, GLAnalysis, Group, Nufft2Error,  # noqa: F401
                     PartialRegularity, Plan, Server,
                     autotune,
                     nufft2_autotune, nufft2_check,
                     nufft2_debug_buffer, nufft2_destroy, nufft2_exec, nufft2_get_info,
                     nufft2_kernel_correction, nufft2_kernel_params, nufft2_plan,
                     nufft2_profile_enable, nufft2_profile_read, nufft2_set_stream,
                     nufft2_setpts, nufft2_strerror, nufft2_group_create, nufft2_group_setpts,
                     nufft2_group_exec, nufft2_group_destroy, nufft2_group_get_info)
