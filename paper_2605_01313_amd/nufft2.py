"""Python binding of libnufft2.so: the C ABI of include/nufft2.h, same names.

Argument marshalling only: every step of the interpolation runs in the HIP
kernels behind the C ABI.  PyTorch is used for device memory and the current
stream in the `Plan` convenience class; the `nufft2_*` functions take raw
device pointers (ints) like the C functions do.

If the library has not been built this module raises on import; there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libnufft2.so")

NUFFT2_OK = 0
NUFFT2_ERR_ARG = 1
NUFFT2_ERR_EPS_RANGE = 2
NUFFT2_ERR_ALLOC = 3
NUFFT2_ERR_NO_POINTS = 4
NUFFT2_ERR_NONFINITE = 5
NUFFT2_ERR_HIP = 6

NUFFT2_FP32 = 1
NUFFT2_FP64 = 2

EXPORTED = (
    "nufft2_plan", "nufft2_setpts", "nufft2_setpts_vector", "nufft2_exec", "nufft2_destroy", "nufft2_strerror",
    "nufft2_get_info", "nufft2_check", "nufft2_set_stream", "nufft2_kernel_params",
    "nufft2_kernel_correction", "nufft2_debug_buffer", "nufft2_profile_enable",
    "nufft2_profile_read", "nufft2_group_create", "nufft2_group_setpts", "nufft2_group_exec", "nufft2_group_run",
    "nufft2_group_destroy", "nufft2_group_get_info", "nufft2_autotune", "nufft2_autotune_group",
    "nufft2_server_create",
    "nufft2_server_clock", "nufft2_server_submit", "nufft2_server_wait", "nufft2_server_drain",
    "nufft2_server_stats", "nufft2_server_destroy", "nufft2_analysis_plan", "nufft2_analysis_exec",
    "nufft2_analysis_destroy", "nufft2_rotate_uv", "nufft2_analysis_set_zonal_filter", "nufft2_analysis_set_layout", "nufft2_pr_plan",
    "nufft2_pr_project", "nufft2_pr_synthesize", "nufft2_pr_destroy", "nufft2_gl_nodes", "nufft2_gl_plan",
    "nufft2_gl_exec", "nufft2_gl_destroy", "nufft2_exec_noalloc", "nufft2_noalloc_capacity",
)
NUFFT2_N_STAGES = 4
STAGE_NAMES = ("setpts", "theta_pass", "phi_pass", "gather")


class nufft2_opts(ctypes.Structure):
    _fields_ = [("w", ctypes.c_int32), ("beta_over_w", ctypes.c_double),
                ("tile_theta", ctypes.c_int32), ("tile_phi", ctypes.c_int32),
                ("real_output", ctypes.c_int32), ("hermitian", ctypes.c_int32),
                ("m_major", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class nufft2_info(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("w", ctypes.c_int32), ("beta", ctypes.c_double),
                ("n_modes_theta", ctypes.c_int64), ("n_modes_phi", ctypes.c_int64),
                ("nf_theta", ctypes.c_int64), ("nf_phi", ctypes.c_int64),
                ("n_fields", ctypes.c_int32), ("real_output", ctypes.c_int32),
                ("tile_theta", ctypes.c_int32), ("tile_phi", ctypes.c_int32),
                ("n_bins", ctypes.c_int64), ("n_pts", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_uint64), ("last_hip_error", ctypes.c_int32),
                ("device", ctypes.c_int32), ("hermitian", ctypes.c_int32), ("fields_per_pass", ctypes.c_int32),
                ("m_major", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class nufft2_group_info(ctypes.Structure):
    _fields_ = [("n_members", ctypes.c_int32), ("n_classes", ctypes.c_int32),
                ("setpts_kernels", ctypes.c_int32), ("exec_kernels", ctypes.c_int32),
                ("table_bytes", ctypes.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class nufft2_tune_result(ctypes.Structure):
    _fields_ = [("w", ctypes.c_int32), ("tile_theta", ctypes.c_int32), ("tile_phi", ctypes.c_int32),
                ("from_cache", ctypes.c_int32), ("err", ctypes.c_double), ("ms", ctypes.c_double),
                ("n_timed", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class nufft2_server_opts(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("max_inflight", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class nufft2_request(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("n_fields", ctypes.c_int32),
                ("n_modes_theta", ctypes.c_int64), ("n_modes_phi", ctypes.c_int64),
                ("eps", ctypes.c_double), ("n_pts", ctypes.c_int64),
                ("coeffs_host", ctypes.c_void_p), ("phi_host", ctypes.c_void_p),
                ("theta_host", ctypes.c_void_p), ("out_host", ctypes.c_void_p),
                ("t_arrival", ctypes.c_double)]


class nufft2_server_stats_t(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("points_fields", ctypes.c_int64), ("latency_p50", ctypes.c_double),
                ("latency_p99", ctypes.c_double), ("latency_max", ctypes.c_double),
                ("first_arrival", ctypes.c_double), ("last_completion", ctypes.c_double),
                ("plans_created", ctypes.c_int64), ("plans_evicted", ctypes.c_int64),
                ("hbm_high_water", ctypes.c_uint64), ("max_inflight_seen", ctypes.c_int32),
                ("reserved", ctypes.c_int32),
                ("queue_p50", ctypes.c_double), ("queue_p99", ctypes.c_double),
                ("h2d_p50", ctypes.c_double), ("h2d_p99", ctypes.c_double),
                ("kernel_p50", ctypes.c_double), ("kernel_p99", ctypes.c_double),
                ("d2h_p50", ctypes.c_double), ("d2h_p99", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'`"
            " (there is no non-HIP fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    H = ctypes.c_void_p
    sigs = {
        "nufft2_plan": [i32, i64, i64, i32, dbl, ctypes.POINTER(nufft2_opts), vp, ctypes.POINTER(H)],
        "nufft2_setpts": [H, i64, vp, vp],
        "nufft2_exec": [H, vp, vp],
        "nufft2_destroy": [H],
        "nufft2_get_info": [H, ctypes.POINTER(nufft2_info)],
        "nufft2_check": [H],
        "nufft2_set_stream": [H, vp],
        "nufft2_kernel_params": [i32, dbl, ctypes.POINTER(i32), ctypes.POINTER(dbl)],
        "nufft2_kernel_correction": [i64, i64, i32, dbl, vp],
        "nufft2_debug_buffer": [H, i32, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_uint64)],
        "nufft2_profile_enable": [H, ctypes.c_uint32],
        "nufft2_profile_read": [H, vp, vp],
        "nufft2_group_create": [vp, i32, ctypes.POINTER(H)],
        "nufft2_group_setpts": [H, vp, vp, vp],
        "nufft2_group_exec": [H, vp, vp],
        "nufft2_group_run": [H, vp, vp, vp, vp, vp],
        "nufft2_group_destroy": [H],
        "nufft2_group_get_info": [H, ctypes.POINTER(nufft2_group_info)],
        "nufft2_autotune": [i32, i64, i64, i32, dbl, i64, vp, vp, vp, ctypes.c_char_p,
                            ctypes.POINTER(nufft2_opts), ctypes.POINTER(nufft2_tune_result)],
        "nufft2_autotune_group": [i32, i64, i64, i32, dbl, i32, i64, vp, vp, vp, ctypes.c_char_p,
                                  ctypes.POINTER(nufft2_opts), ctypes.POINTER(nufft2_tune_result)],
        "nufft2_server_create": [ctypes.POINTER(nufft2_server_opts), ctypes.POINTER(H)],
        "nufft2_server_submit": [H, ctypes.POINTER(nufft2_request), ctypes.POINTER(ctypes.c_uint64)],
        "nufft2_server_wait": [H, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(dbl)],
        "nufft2_server_drain": [H],
        "nufft2_server_stats": [H, ctypes.POINTER(nufft2_server_stats_t)],
        "nufft2_server_destroy": [H],
        "nufft2_analysis_plan": [i32, i64, i32, vp, ctypes.POINTER(H)],
        "nufft2_analysis_exec": [H, vp, vp],
        "nufft2_analysis_destroy": [H],
        "nufft2_rotate_uv": [H, vp, i32, i32, vp, vp, vp, vp],
        "nufft2_setpts_vector": [H, i64, vp, vp, vp, vp, i32, i32],
        "nufft2_analysis_set_zonal_filter": [H, i32],
        "nufft2_analysis_set_layout": [H, i32],
        "nufft2_pr_plan": [i32, i64, i64, i32, vp, ctypes.POINTER(H)],
        "nufft2_pr_project": [H, vp, vp],
        "nufft2_pr_synthesize": [H, vp, vp],
        "nufft2_pr_destroy": [H],
        "nufft2_gl_nodes": [i64, vp],
        "nufft2_gl_plan": [i32, i64, i32, vp, ctypes.POINTER(H)],
        "nufft2_gl_exec": [H, vp, vp],
        "nufft2_gl_destroy": [H],
        "nufft2_exec_noalloc": [i32, i64, i64, i32, dbl, ctypes.POINTER(nufft2_opts), i64, vp, vp, vp, vp, vp],
        "nufft2_noalloc_capacity": [ctypes.POINTER(ctypes.c_uint64)],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.nufft2_server_clock.argtypes = [H]
    lib.nufft2_server_clock.restype = ctypes.c_double
    lib.nufft2_strerror.argtypes = [ctypes.c_int]
    lib.nufft2_strerror.restype = ctypes.c_char_p
    return lib


_lib = _load()


class Nufft2Error(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {nufft2_strerror(status)} (status {status})")


def _check(status, where):
    if status != NUFFT2_OK:
        raise Nufft2Error(status, where)


# ---- the C ABI, one function each ------------------------------------------
def nufft2_strerror(status: int) -> str:
    return _lib.nufft2_strerror(int(status)).decode()


def nufft2_plan(prec, n_modes_theta, n_modes_phi, n_fields, eps, opts=None, stream=0):
    """Returns (status, handle)."""
    h = ctypes.c_void_p()
    po = ctypes.byref(opts) if opts is not None else None
    st = _lib.nufft2_plan(int(prec), int(n_modes_theta), int(n_modes_phi), int(n_fields),
                          float(eps), po, ctypes.c_void_p(stream or None), ctypes.byref(h))
    return st, h


def nufft2_setpts(handle, n_pts, phi_ptr, theta_ptr):
    return _lib.nufft2_setpts(handle, int(n_pts), ctypes.c_void_p(phi_ptr or None),
                              ctypes.c_void_p(theta_ptr or None))


def nufft2_setpts_vector(handle, n_pts, phi_ptr, theta_ptr, phi_a_ptr, theta_a_ptr, field_u, field_v):
    P = lambda x: ctypes.c_void_p(x or None)
    return _lib.nufft2_setpts_vector(handle, int(n_pts), P(phi_ptr), P(theta_ptr), P(phi_a_ptr), P(theta_a_ptr),
                                     int(field_u), int(field_v))


def nufft2_exec(handle, coeffs_ptr, out_ptr):
    return _lib.nufft2_exec(handle, ctypes.c_void_p(coeffs_ptr or None),
                            ctypes.c_void_p(out_ptr or None))


def nufft2_destroy(handle):
    return _lib.nufft2_destroy(handle)


def nufft2_get_info(handle):
    info = nufft2_info()
    st = _lib.nufft2_get_info(handle, ctypes.byref(info))
    return st, info


def nufft2_check(handle):
    return _lib.nufft2_check(handle)


def nufft2_set_stream(handle, stream):
    return _lib.nufft2_set_stream(handle, ctypes.c_void_p(stream or None))


def nufft2_kernel_params(prec, eps):
    w = ctypes.c_int32()
    beta = ctypes.c_double()
    st = _lib.nufft2_kernel_params(int(prec), float(eps), ctypes.byref(w), ctypes.byref(beta))
    return st, w.value, beta.value


def nufft2_kernel_correction(K, nf, w, beta):
    import numpy as np
    out = np.zeros(int(K), dtype=np.float64)
    st = _lib.nufft2_kernel_correction(int(K), int(nf), int(w), float(beta), out.ctypes.data)
    return st, out


def nufft2_debug_buffer(handle, which):
    ptr = ctypes.c_void_p()
    nbytes = ctypes.c_uint64()
    st = _lib.nufft2_debug_buffer(handle, int(which), ctypes.byref(ptr), ctypes.byref(nbytes))
    return st, (ptr.value or 0), nbytes.value


def nufft2_profile_enable(handle, stage_mask):
    return _lib.nufft2_profile_enable(handle, int(stage_mask))


def nufft2_profile_read(handle):
    """Returns (status, total_ms[4], count[4])."""
    import numpy as np
    ms = np.zeros(NUFFT2_N_STAGES, dtype=np.float64)
    cnt = np.zeros(NUFFT2_N_STAGES, dtype=np.int64)
    st = _lib.nufft2_profile_read(handle, ms.ctypes.data, cnt.ctypes.data)
    return st, ms, cnt


def _ptr_array(values):
    arr = (ctypes.c_void_p * len(values))()
    for i, v in enumerate(values):
        arr[i] = v or None
    return arr


def nufft2_group_create(handles):
    """Returns (status, group handle) for a list of plan handles."""
    arr = (ctypes.c_void_p * len(handles))(*[h.value for h in handles])
    g = ctypes.c_void_p()
    st = _lib.nufft2_group_create(arr, len(handles), ctypes.byref(g))
    return st, g


def nufft2_group_setpts(group, n_pts, phi_ptrs, theta_ptrs):
    n = (ctypes.c_int64 * len(n_pts))(*[int(x) for x in n_pts])
    return _lib.nufft2_group_setpts(group, n, _ptr_array(phi_ptrs), _ptr_array(theta_ptrs))


def nufft2_group_exec(group, coeffs_ptrs, out_ptrs):
    return _lib.nufft2_group_exec(group, _ptr_array(coeffs_ptrs), _ptr_array(out_ptrs))


def nufft2_group_run(group, n_pts, phi_ptrs, theta_ptrs, coeffs_ptrs, out_ptrs):
    n = (ctypes.c_int64 * len(n_pts))(*[int(x) for x in n_pts])
    return _lib.nufft2_group_run(group, n, _ptr_array(phi_ptrs), _ptr_array(theta_ptrs), _ptr_array(coeffs_ptrs),
                                 _ptr_array(out_ptrs))


def nufft2_group_destroy(group):
    return _lib.nufft2_group_destroy(group)


def nufft2_group_get_info(group):
    info = nufft2_group_info()
    st = _lib.nufft2_group_get_info(group, ctypes.byref(info))
    return st, info


def nufft2_autotune(prec, n_modes_theta, n_modes_phi, n_fields, eps, n_pts, phi_ptr, theta_ptr,
                    stream=0, cache_path=None, hermitian=False):
    """Returns (status, nufft2_opts, nufft2_tune_result)."""
    opts = nufft2_opts()
    opts.hermitian = int(bool(hermitian))
    res = nufft2_tune_result()
    st = _lib.nufft2_autotune(int(prec), int(n_modes_theta), int(n_modes_phi), int(n_fields), float(eps),
                              int(n_pts), ctypes.c_void_p(phi_ptr or None), ctypes.c_void_p(theta_ptr or None),
                              ctypes.c_void_p(stream or None),
                              cache_path.encode() if cache_path else None, ctypes.byref(opts), ctypes.byref(res))
    return st, opts, res


def nufft2_autotune_group(prec, n_modes_theta, n_modes_phi, n_fields, eps, members, n_pts, phi_ptr, theta_ptr,
                          stream=0, cache_path=None, hermitian=False):
    """Returns (status, nufft2_opts, nufft2_tune_result)."""
    opts = nufft2_opts()
    opts.hermitian = int(bool(hermitian))
    res = nufft2_tune_result()
    st = _lib.nufft2_autotune_group(int(prec), int(n_modes_theta), int(n_modes_phi), int(n_fields), float(eps),
                                    int(members), int(n_pts), ctypes.c_void_p(phi_ptr or None),
                                    ctypes.c_void_p(theta_ptr or None), ctypes.c_void_p(stream or None),
                                    cache_path.encode() if cache_path else None, ctypes.byref(opts),
                                    ctypes.byref(res))
    return st, opts, res


def nufft2_server_create(hbm_budget=0, max_inflight=0):
    """Returns (status, server handle)."""
    o = nufft2_server_opts(int(hbm_budget), int(max_inflight), 0)
    h = ctypes.c_void_p()
    st = _lib.nufft2_server_create(ctypes.byref(o), ctypes.byref(h))
    return st, h


def nufft2_server_clock(server):
    return _lib.nufft2_server_clock(server)


def nufft2_server_submit(server, req):
    """req: nufft2_request.  Returns (status, ticket)."""
    t = ctypes.c_uint64()
    st = _lib.nufft2_server_submit(server, ctypes.byref(req), ctypes.byref(t))
    return st, t.value


def nufft2_server_wait(server, ticket):
    """Returns (status, request status, latency seconds)."""
    rs = ctypes.c_int()
    lat = ctypes.c_double()
    st = _lib.nufft2_server_wait(server, int(ticket), ctypes.byref(rs), ctypes.byref(lat))
    return st, rs.value, lat.value


def nufft2_server_drain(server):
    return _lib.nufft2_server_drain(server)


def nufft2_server_stats(server):
    s = nufft2_server_stats_t()
    st = _lib.nufft2_server_stats(server, ctypes.byref(s))
    return st, s


def nufft2_server_destroy(server):
    return _lib.nufft2_server_destroy(server)


def nufft2_exec_noalloc(prec, n_modes_theta, n_modes_phi, n_fields, eps, opts, n_pts, phi_ptr, theta_ptr,
                        coeffs_ptr, out_ptr, stream=0):
    return _lib.nufft2_exec_noalloc(prec, n_modes_theta, n_modes_phi, n_fields, eps,
                                    ctypes.byref(opts) if opts is not None else None, n_pts, phi_ptr, theta_ptr,
                                    coeffs_ptr, out_ptr, stream)


def nufft2_noalloc_capacity():
    b = ctypes.c_uint64()
    st = _lib.nufft2_noalloc_capacity(ctypes.byref(b))
    return st, b.value


def nufft2_rotate_uv(handle, out_ptr, field_u, field_v, phi_a, theta_a, phi_d, theta_d):
    P = lambda x: ctypes.c_void_p(x or None)
    return _lib.nufft2_rotate_uv(handle, P(out_ptr), int(field_u), int(field_v), P(phi_a), P(theta_a),
                                 P(phi_d), P(theta_d))


def nufft2_analysis_plan(prec, J, n_fields, stream=0):
    """Returns (status, analysis handle)."""
    h = ctypes.c_void_p()
    st = _lib.nufft2_analysis_plan(int(prec), int(J), int(n_fields), ctypes.c_void_p(stream or None),
                                   ctypes.byref(h))
    return st, h


def nufft2_analysis_exec(handle, values_ptr, coeffs_ptr):
    return _lib.nufft2_analysis_exec(handle, ctypes.c_void_p(values_ptr or None), ctypes.c_void_p(coeffs_ptr or None))


def nufft2_analysis_destroy(handle):
    return _lib.nufft2_analysis_destroy(handle)


def nufft2_analysis_set_zonal_filter(handle, M0):
    return _lib.nufft2_analysis_set_zonal_filter(handle, int(M0))


def nufft2_analysis_set_layout(handle, m_major):
    return _lib.nufft2_analysis_set_layout(handle, int(m_major))


def nufft2_pr_plan(prec, N, M, n_fields, stream=0):
    """Returns (status, partial-regularity plan handle)."""
    h = ctypes.c_void_p()
    st = _lib.nufft2_pr_plan(int(prec), int(N), int(M), int(n_fields), ctypes.c_void_p(stream or None),
                             ctypes.byref(h))
    return st, h


def nufft2_pr_project(handle, coeffs_ptr, pr_ptr):
    return _lib.nufft2_pr_project(handle, ctypes.c_void_p(coeffs_ptr or None), ctypes.c_void_p(pr_ptr or None))


def nufft2_pr_synthesize(handle, pr_ptr, coeffs_ptr):
    return _lib.nufft2_pr_synthesize(handle, ctypes.c_void_p(pr_ptr or None), ctypes.c_void_p(coeffs_ptr or None))


def nufft2_pr_destroy(handle):
    return _lib.nufft2_pr_destroy(handle)


def nufft2_gl_nodes(J):
    """Returns (status, numpy array of the J Gauss-Legendre colatitudes)."""
    import numpy as np
    out = np.zeros(max(int(J), 1), dtype=np.float64)
    st = _lib.nufft2_gl_nodes(int(J), out.ctypes.data_as(ctypes.c_void_p))
    return st, out


def nufft2_gl_plan(prec, J, n_fields, stream=0):
    """Returns (status, Gauss-Legendre analysis handle)."""
    h = ctypes.c_void_p()
    st = _lib.nufft2_gl_plan(int(prec), int(J), int(n_fields), ctypes.c_void_p(stream or None), ctypes.byref(h))
    return st, h


def nufft2_gl_exec(handle, values_ptr, coeffs_ptr):
    return _lib.nufft2_gl_exec(handle, ctypes.c_void_p(values_ptr or None), ctypes.c_void_p(coeffs_ptr or None))


def nufft2_gl_destroy(handle):
    return _lib.nufft2_gl_destroy(handle)


# ---- torch convenience -----------------------------------------------------
class Plan:
    """A plan bound to torch tensors on the current device and stream.

    >>> p = Plan("fp32", K, K, n_fields=3, eps=1e-6)
    >>> p.setpts(phi, theta)            # float64 device tensors
    >>> out = p.exec(coeffs)            # complex64 device tensor (F, K, K)

    hermitian=True: coefficients of real fields (c[-n][-m] = conj c[n][m]);
    the plan reads the m >= 0 half, works on a real fine grid and returns
    real values (float32 / float64).
    m_major=True: coefficients given as (F, K_phi, K_theta) (mode m outer),
    the layout Analysis writes with m_major=True.
    """

    def __init__(self, prec, n_modes_theta, n_modes_phi, n_fields=1, eps=1e-6, *, w=0,
                 beta_over_w=0.0, tile_theta=0, tile_phi=0, real_output=False, hermitian=False, m_major=False,
                 stream=None):
        import torch
        self._torch = torch
        self.prec = {"fp32": NUFFT2_FP32, "fp64": NUFFT2_FP64,
                     NUFFT2_FP32: NUFFT2_FP32, NUFFT2_FP64: NUFFT2_FP64}[prec]
        self.cdtype = torch.complex64 if self.prec == NUFFT2_FP32 else torch.complex128
        self.rdtype = torch.float32 if self.prec == NUFFT2_FP32 else torch.float64
        self.m_major = bool(m_major)
        # the coefficient tensor's shape: (F, K_theta, K_phi), or (F, K_phi, K_theta) m-major
        self.shape = ((int(n_fields), int(n_modes_phi), int(n_modes_theta)) if self.m_major
                      else (int(n_fields), int(n_modes_theta), int(n_modes_phi)))
        self.hermitian = bool(hermitian)
        self.real_output = bool(real_output) or self.hermitian
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        opts = nufft2_opts(int(w), float(beta_over_w), int(tile_theta), int(tile_phi),
                           int(bool(real_output)), int(self.hermitian), int(self.m_major), 0)
        st, h = nufft2_plan(self.prec, n_modes_theta, n_modes_phi, n_fields, eps, opts,
                            self.stream.cuda_stream)
        _check(st, "nufft2_plan")
        self.handle = h
        self._pts = None
        self.n_pts = -1

    def info(self):
        st, info = nufft2_get_info(self.handle)
        _check(st, "nufft2_get_info")
        return info.as_dict()

    def _check_points(self, phi, theta):
        t = self._torch
        for x in (phi, theta):
            if x.dtype != t.float64 or not x.is_cuda or not x.is_contiguous():
                raise TypeError("points must be contiguous float64 device tensors")
        if phi.numel() != theta.numel():
            raise ValueError("phi and theta differ in length")
        return phi.numel()

    def _check_coeffs(self, coeffs):
        if coeffs.dtype != self.cdtype or not coeffs.is_cuda or not coeffs.is_contiguous():
            raise TypeError(f"coeffs must be a contiguous {self.cdtype} device tensor")
        if tuple(coeffs.shape) != self.shape and tuple(coeffs.shape) != self.shape[1:]:
            raise ValueError(f"coeffs shape {tuple(coeffs.shape)} != {self.shape}")

    def _check_out(self, out, n_pts):
        """The output tensor the kernels write: dtype, device, contiguity and
        size are checked before any launch (a wrong one would be written out
        of bounds)."""
        F = self.shape[0]
        dt = self.rdtype if self.real_output else self.cdtype
        if out.dtype != dt or not out.is_cuda or not out.is_contiguous() or out.numel() != F * max(n_pts, 0):
            raise ValueError(f"out must be a contiguous {dt} device tensor of {F} x {max(n_pts, 0)} values")
        return out

    def _check_io(self, coeffs, out, n_pts):
        self._check_coeffs(coeffs)
        if out is None:
            dt = self.rdtype if self.real_output else self.cdtype
            return self._torch.empty((self.shape[0], max(n_pts, 0)), dtype=dt, device=coeffs.device)
        return self._check_out(out, n_pts)

    def setpts(self, phi, theta):
        n = self._check_points(phi, theta)
        _check(nufft2_setpts(self.handle, n, phi.data_ptr() if n else 0,
                             theta.data_ptr() if n else 0), "nufft2_setpts")
        self._pts = (phi, theta)   # keep alive until the stream has consumed them
        self.n_pts = n

    def setpts_vector(self, phi, theta, phi_a, theta_a, field_u, field_v):
        """setpts whose following execs return fields (u, v) rotated into each
        point's arrival frame (section 3's matrix Q, inside the gather)."""
        n = self._check_points(phi, theta)
        for x in (phi_a, theta_a):
            if x.dtype != self._torch.float64 or not x.is_cuda or not x.is_contiguous() or x.numel() != n:
                raise TypeError("arrival points must be contiguous float64 device tensors of n_pts entries")
        P = (lambda x: x.data_ptr() if n else 0)
        _check(nufft2_setpts_vector(self.handle, n, P(phi), P(theta), P(phi_a), P(theta_a), field_u, field_v),
               "nufft2_setpts_vector")
        self._pts = (phi, theta)
        self._arrival = (phi_a, theta_a)   # read by this call's kernels
        self.n_pts = n

    def exec(self, coeffs, out=None):
        out = self._check_io(coeffs, out, self.n_pts)
        _check(nufft2_exec(self.handle, coeffs.data_ptr(), out.data_ptr() if out.numel() else 0),
               "nufft2_exec")
        return out

    def check(self):
        st = nufft2_check(self.handle)
        return st

    def rotate_uv(self, out, field_u, field_v, phi_a, theta_a):
        """Rotate fields (u, v) of `out` into the arrival frame (in place); the
        departure points are those of the last setpts."""
        if self._pts is None:
            raise RuntimeError("rotate_uv before setpts")
        phi_d, theta_d = self._pts
        self._check_out(out, self.n_pts)
        for x in (phi_a, theta_a):
            if x.dtype != self._torch.float64 or not x.is_cuda or not x.is_contiguous() or x.numel() != self.n_pts:
                raise TypeError("arrival points must be contiguous float64 device tensors of n_pts entries")
        _check(nufft2_rotate_uv(self.handle, out.data_ptr(), field_u, field_v, phi_a.data_ptr(),
                                theta_a.data_ptr(), phi_d.data_ptr(), theta_d.data_ptr()), "nufft2_rotate_uv")
        return out

    def profile(self, stage_mask):
        _check(nufft2_profile_enable(self.handle, stage_mask), "nufft2_profile_enable")

    def profile_read(self):
        st, ms, cnt = nufft2_profile_read(self.handle)
        _check(st, "nufft2_profile_read")
        return {STAGE_NAMES[i]: (float(ms[i]), int(cnt[i])) for i in range(NUFFT2_N_STAGES)}

    def debug_buffer(self, which):
        st, ptr, nbytes = nufft2_debug_buffer(self.handle, which)
        _check(st, "nufft2_debug_buffer")
        return ptr, nbytes

    def debug_tensor(self, which, dtype, shape):
        """Copy a plan workspace into a new device tensor (stage tests)."""
        t = self._torch
        ptr, nbytes = self.debug_buffer(which)
        out = t.empty(shape, dtype=dtype, device="cuda")
        assert out.numel() * out.element_size() <= nbytes
        import ctypes as _ct
        hip = _ct.CDLL("libamdhip64.so")
        hip.hipMemcpy.argtypes = [_ct.c_void_p, _ct.c_void_p, _ct.c_size_t, _ct.c_int]
        self._torch.cuda.synchronize()
        rc = hip.hipMemcpy(_ct.c_void_p(out.data_ptr()), _ct.c_void_p(ptr),
                           out.numel() * out.element_size(), 3)
        if rc != 0:
            raise RuntimeError(f"hipMemcpy failed ({rc})")
        return out

    def destroy(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            nufft2_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Group:
    """Plans run together (nufft2_group_*).

    >>> g = Group([p0, p1, ...])                 # Plan objects on one stream
    >>> g.setpts([phi0, phi1, ...], [theta0, ...])
    >>> outs = g.exec([c0, c1, ...])             # list of output tensors
    >>> outs = g.run(phis, thetas, coeffs)       # both as one graph launch
    """

    def __init__(self, plans):
        self._torch = plans[0]._torch
        self.plans = list(plans)
        st, g = nufft2_group_create([p.handle for p in self.plans])
        _check(st, "nufft2_group_create")
        self.handle = g
        self._keep = None

    def info(self):
        st, info = nufft2_group_get_info(self.handle)
        _check(st, "nufft2_group_get_info")
        return info.as_dict()

    def _points_args(self, phis, thetas):
        t = self._torch
        if len(phis) != len(self.plans) or len(thetas) != len(self.plans):
            raise ValueError("one (phi, theta) pair per member")
        for x in list(phis) + list(thetas):
            if x.dtype != t.float64 or not x.is_cuda or not x.is_contiguous():
                raise TypeError("points must be contiguous float64 device tensors")
        ns = [x.numel() for x in phis]
        if any(a.numel() != b for a, b in zip(thetas, ns)):
            raise ValueError("phi and theta differ in length")
        return ns, [x.data_ptr() if x.numel() else 0 for x in phis], [x.data_ptr() if x.numel() else 0 for x in thetas]

    def _exec_args(self, coeffs, outs, ns):
        """Checked coefficient tensors and outputs for point counts ns."""
        t = self._torch
        if len(coeffs) != len(self.plans):
            raise ValueError("one coefficient tensor per member")
        for p, c in zip(self.plans, coeffs):
            p._check_coeffs(c)
        if outs is None:
            # one element at least per field, so that every member has a
            # device pointer (the C call takes none null)
            outs = []
            for p, c, n in zip(self.plans, coeffs, ns):
                dt = p.rdtype if p.real_output else p.cdtype
                outs.append(t.empty((p.shape[0], max(n, 1)), dtype=dt, device=c.device))
        else:
            if len(outs) != len(self.plans):
                raise ValueError("one output tensor per member")
            for p, o, n in zip(self.plans, outs, ns):
                if n > 0:
                    p._check_out(o, n)
                elif not o.is_cuda:
                    raise ValueError("outputs must be device tensors")
        return outs

    def setpts(self, phis, thetas):
        ns, pp, tp = self._points_args(phis, thetas)
        _check(nufft2_group_setpts(self.handle, ns, pp, tp), "nufft2_group_setpts")
        for p, n, a, b in zip(self.plans, ns, phis, thetas):
            p.n_pts = n
            p._pts = (a, b)

    def exec(self, coeffs, outs=None):
        ns = [p.n_pts for p in self.plans]
        outs = self._exec_args(coeffs, outs, ns)
        _check(nufft2_group_exec(self.handle, [c.data_ptr() for c in coeffs],
                                 [o.data_ptr() for o in outs]), "nufft2_group_exec")
        self._keep = (coeffs, outs)
        return [o[:, :p.n_pts] for o, p in zip(outs, self.plans)]

    def bind(self, phis, thetas, coeffs, outs=None):
        """Validate one set of per-member tensors and return a callable that
        runs setpts + exec on them (nufft2_group_run) without checking them
        again: for time-stepping loops that update these tensors in place
        every step.  The tensors must keep their storage while bound (no
        resize_, set_ or reallocation); the callable keeps them alive and
        returns the output views.

        >>> step = g.bind(phis, thetas, coeffs)
        >>> for _ in range(n_steps):
        ...     update(phis, thetas, coeffs)   # in place
        ...     outs = step()
        """
        ns, pp, tp = self._points_args(phis, thetas)
        outs = self._exec_args(coeffs, outs, ns)
        n_arr = (ctypes.c_int64 * len(ns))(*ns)
        args = (n_arr, _ptr_array(pp), _ptr_array(tp), _ptr_array([c.data_ptr() for c in coeffs]),
                _ptr_array([o.data_ptr() for o in outs]))
        keep = (list(phis), list(thetas), list(coeffs), list(outs))
        views = [o[:, :n] for o, n in zip(outs, ns)]
        handle, plans = self.handle, self.plans

        def step():
            _check(_lib.nufft2_group_run(handle, *args), "nufft2_group_run")
            return views

        step.keep = keep
        for p, n, a, b in zip(plans, ns, phis, thetas):
            p.n_pts = n
            p._pts = (a, b)
        self._keep = keep
        return step

    def run(self, phis, thetas, coeffs, outs=None):
        """setpts then exec as one graph launch (nufft2_group_run)."""
        ns, pp, tp = self._points_args(phis, thetas)
        outs = self._exec_args(coeffs, outs, ns)
        _check(nufft2_group_run(self.handle, ns, pp, tp, [c.data_ptr() for c in coeffs],
                                [o.data_ptr() for o in outs]), "nufft2_group_run")
        for p, n, a, b in zip(self.plans, ns, phis, thetas):
            p.n_pts = n
            p._pts = (a, b)
        self._keep = (coeffs, outs)
        return [o[:, :n] for o, n in zip(outs, ns)]

    def destroy(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            nufft2_group_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def autotune(prec, n_modes_theta, n_modes_phi, n_fields, eps, phi, theta, cache_path=None, stream=None,
             hermitian=False, members=1):
    """Tune width and tiles on the given points (float64 device tensors).

    members > 1: the tiles are timed on a group of that many plans, each
    with these points (nufft2_autotune_group).
    Returns a dict: w, tile_theta, tile_phi (keyword arguments for Plan) and
    the measurement (err, ms, from_cache, n_timed).
    """
    import torch
    prec_code = {"fp32": NUFFT2_FP32, "fp64": NUFFT2_FP64, NUFFT2_FP32: NUFFT2_FP32,
                 NUFFT2_FP64: NUFFT2_FP64}[prec]
    for x in (phi, theta):
        if x.dtype != torch.float64 or not x.is_cuda or not x.is_contiguous():
            raise TypeError("points must be contiguous float64 device tensors")
    s = stream if stream is not None else torch.cuda.current_stream()
    if members > 1:
        st, opts, res = nufft2_autotune_group(prec_code, n_modes_theta, n_modes_phi, n_fields, eps, members,
                                              phi.numel(), phi.data_ptr(), theta.data_ptr(), s.cuda_stream,
                                              cache_path, hermitian)
    else:
        st, opts, res = nufft2_autotune(prec_code, n_modes_theta, n_modes_phi, n_fields, eps, phi.numel(),
                                        phi.data_ptr(), theta.data_ptr(), s.cuda_stream, cache_path, hermitian)
    _check(st, "nufft2_autotune")
    out = res.as_dict()
    out.update(w=opts.w, tile_theta=opts.tile_theta, tile_phi=opts.tile_phi)
    return out


class Server:
    """Request loop with continuous batching (nufft2_server_*).

    Host tensors (pinned for overlap) stay referenced until their request
    completes.

    >>> srv = Server(hbm_budget=8 << 30, max_inflight=8)
    >>> t = srv.submit("fp32", coeffs, phi, theta, eps=1e-6, out=out)   # CPU tensors
    >>> status, latency = srv.wait(t)
    """

    def __init__(self, hbm_budget=0, max_inflight=0):
        st, h = nufft2_server_create(hbm_budget, max_inflight)
        _check(st, "nufft2_server_create")
        self.handle = h
        self._live = {}

    def clock(self):
        return nufft2_server_clock(self.handle)

    def submit(self, prec, coeffs, phi, theta, eps, out=None, t_arrival=None):
        import torch
        code = {"fp32": NUFFT2_FP32, "fp64": NUFFT2_FP64}[prec]
        cdt = torch.complex64 if code == NUFFT2_FP32 else torch.complex128
        if coeffs.dtype != cdt or coeffs.is_cuda or not coeffs.is_contiguous() or coeffs.dim() != 3:
            raise TypeError(f"coeffs must be a contiguous host {cdt} tensor (F, Kt, Kp)")
        for x in (phi, theta):
            if x.dtype != torch.float64 or x.is_cuda or not x.is_contiguous():
                raise TypeError("points must be contiguous host float64 tensors")
        F, Kt, Kp = coeffs.shape
        n = phi.numel()
        if out is not None and (out.dtype != cdt or out.is_cuda or tuple(out.shape) != (F, n)
                                or not out.is_contiguous()):
            raise TypeError(f"out must be a contiguous host {cdt} tensor ({F}, {n})")
        req = nufft2_request(code, F, Kt, Kp, float(eps), n, coeffs.data_ptr(), phi.data_ptr(),
                             theta.data_ptr(), out.data_ptr() if out is not None else None,
                             self.clock() if t_arrival is None else float(t_arrival))
        st, ticket = nufft2_server_submit(self.handle, req)
        _check(st, "nufft2_server_submit")
        self._live[ticket] = (coeffs, phi, theta, out)
        return ticket

    def wait(self, ticket):
        st, rs, lat = nufft2_server_wait(self.handle, ticket)
        _check(st, "nufft2_server_wait")
        self._live.pop(ticket, None)
        return rs, lat

    def drain(self):
        _check(nufft2_server_drain(self.handle), "nufft2_server_drain")
        self._live.clear()

    def stats(self):
        st, s = nufft2_server_stats(self.handle)
        _check(st, "nufft2_server_stats")
        return s.as_dict()

    def destroy(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            nufft2_server_destroy(self.handle)
            self.handle = ctypes.c_void_p()
            self._live.clear()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Analysis:
    """Grid values on Grid [0] -> exp-form coefficients (nufft2_analysis_*).

    >>> an = Analysis("fp64", J=256, n_fields=3)
    >>> coeffs = an.exec(values)      # (F, J, 2J) real -> (F, 2J-1, 2J-1) complex
    """

    def __init__(self, prec, J, n_fields=1, stream=None):
        import torch
        self._torch = torch
        self.prec = {"fp32": NUFFT2_FP32, "fp64": NUFFT2_FP64}[prec]
        self.rdtype = torch.float32 if self.prec == NUFFT2_FP32 else torch.float64
        self.cdtype = torch.complex64 if self.prec == NUFFT2_FP32 else torch.complex128
        self.J, self.F = int(J), int(n_fields)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        st, h = nufft2_analysis_plan(self.prec, J, n_fields, self.stream.cuda_stream)
        _check(st, "nufft2_analysis_plan")
        self.handle = h

    def set_zonal_filter(self, M0=20):
        """Zonal filter of section 4 on the following execs (M0 < 0: off)."""
        _check(nufft2_analysis_set_zonal_filter(self.handle, M0), "nufft2_analysis_set_zonal_filter")

    def set_layout(self, m_major):
        """m_major=True: write (F, K, K) with the mode m outer (the layout of
        Plan(..., m_major=True)); the same values either way."""
        _check(nufft2_analysis_set_layout(self.handle, int(bool(m_major))), "nufft2_analysis_set_layout")

    def exec(self, values, out=None):
        t = self._torch
        J, F = self.J, self.F
        if values.dtype != self.rdtype or not values.is_cuda or not values.is_contiguous() \
                or tuple(values.shape) not in ((F, J, 2 * J), (J, 2 * J)):
            raise TypeError(f"values must be a contiguous {self.rdtype} device tensor ({F}, {J}, {2 * J})")
        if out is None:
            out = t.empty((F, 2 * J - 1, 2 * J - 1), dtype=self.cdtype, device=values.device)
        _check(nufft2_analysis_exec(self.handle, values.data_ptr(), out.data_ptr()), "nufft2_analysis_exec")
        return out

    def destroy(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            nufft2_analysis_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class PartialRegularity:
    """Partial-regularity DFS expansion (nufft2_pr_*): exp-form coefficients
    <-> pr coefficients.

    >>> pr = PartialRegularity("fp64", N=255, M=255, n_fields=3)
    >>> x = pr.project(coeffs)          # (F, 2N+1, 2M+1) complex -> (F, 2, N+1, M+1) real
    >>> c = pr.synthesize(x)            # back to exp form (the projection of coeffs)
    """

    def __init__(self, prec, N, M, n_fields=1, stream=None):
        import torch
        self._torch = torch
        self.prec = {"fp32": NUFFT2_FP32, "fp64": NUFFT2_FP64}[prec]
        self.rdtype = torch.float32 if self.prec == NUFFT2_FP32 else torch.float64
        self.cdtype = torch.complex64 if self.prec == NUFFT2_FP32 else torch.complex128
        self.N, self.M, self.F = int(N), int(M), int(n_fields)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        st, h = nufft2_pr_plan(self.prec, N, M, n_fields, self.stream.cuda_stream)
        _check(st, "nufft2_pr_plan")
        self.handle = h

    def _want(self, x, dtype, shape, what):
        if x.dtype != dtype or not x.is_cuda or not x.is_contiguous() or tuple(x.shape) != shape:
            raise TypeError(f"{what} must be a contiguous {dtype} device tensor {shape}")

    def project(self, coeffs, out=None):
        N, M, F = self.N, self.M, self.F
        self._want(coeffs, self.cdtype, (F, 2 * N + 1, 2 * M + 1), "coeffs")
        if out is None:
            out = self._torch.empty((F, 2, N + 1, M + 1), dtype=self.rdtype, device=coeffs.device)
        self._want(out, self.rdtype, (F, 2, N + 1, M + 1), "out")
        _check(nufft2_pr_project(self.handle, coeffs.data_ptr(), out.data_ptr()), "nufft2_pr_project")
        return out

    def synthesize(self, pr, out=None):
        N, M, F = self.N, self.M, self.F
        self._want(pr, self.rdtype, (F, 2, N + 1, M + 1), "pr")
        if out is None:
            out = self._torch.empty((F, 2 * N + 1, 2 * M + 1), dtype=self.cdtype, device=pr.device)
        self._want(out, self.cdtype, (F, 2 * N + 1, 2 * M + 1), "out")
        _check(nufft2_pr_synthesize(self.handle, pr.data_ptr(), out.data_ptr()), "nufft2_pr_synthesize")
        return out

    def destroy(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            nufft2_pr_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class GLAnalysis:
    """Samples on the Gauss-Legendre grid -> exp-form coefficients (nufft2_gl_*).

    >>> gl = GLAnalysis("fp64", J=256, n_fields=3)
    >>> coeffs = gl.exec(values)      # (F, J, 2J) real -> (F, 2J+1, 2J-1) complex
    """

    def __init__(self, prec, J, n_fields=1, stream=None):
        import torch
        self._torch = torch
        self.prec = {"fp32": NUFFT2_FP32, "fp64": NUFFT2_FP64}[prec]
        self.rdtype = torch.float32 if self.prec == NUFFT2_FP32 else torch.float64
        self.cdtype = torch.complex64 if self.prec == NUFFT2_FP32 else torch.complex128
        self.J, self.F = int(J), int(n_fields)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        st, h = nufft2_gl_plan(self.prec, J, n_fields, self.stream.cuda_stream)
        _check(st, "nufft2_gl_plan")
        self.handle = h

    def exec(self, values, out=None):
        J, F = self.J, self.F
        if values.dtype != self.rdtype or not values.is_cuda or not values.is_contiguous() \
                or tuple(values.shape) not in ((F, J, 2 * J), (J, 2 * J)):
            raise TypeError(f"values must be a contiguous {self.rdtype} device tensor ({F}, {J}, {2 * J})")
        if out is None:
            out = self._torch.empty((F, 2 * J + 1, 2 * J - 1), dtype=self.cdtype, device=values.device)
        _check(nufft2_gl_exec(self.handle, values.data_ptr(), out.data_ptr()), "nufft2_gl_exec")
        return out

    def destroy(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            nufft2_gl_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
