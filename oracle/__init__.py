"""ORACLE -- test infrastructure only.

Only the tests, the smoke check (`__graft_entry__.smoke`) and the CPU
baseline leg of `bench.py` may import this package.  The product library
(`paper_2605_01313_amd`) never imports, links or calls it, and shares no
code with it.

Contents
  * `dfs_eval`   -- FP64 direct sum of the complex-exponential DFS series
                    (section 5, eq. std_dfs_exp), plain C + OpenMP
                    (`dfs_direct.c`), at arbitrary points.
  * `dfs_eval_ld` -- the same sum in long double, used to certify the FP64
                    oracle's own rounding at the largest sizes.
  * `std_to_exp` -- the map of eq. dfs_fourier_coeffs from standard-DFS
                    cos/sin coefficients to exp-form coefficients.
  * `rotation_pq`, `rotate_uv` -- the rotation Q of section 3 that expresses
                    a vector at the departure point in the arrival point's
                    local (east, north) frame.
  * `dfs_analysis` -- grid values on Grid [0] -> exp-form coefficients, in
                    the paper's order: Fourier transform in phi, cosine /
                    sine transforms in theta (section 4), then `std_to_exp`;
                    the transforms are written as plain sums.
  * `pr_to_std`, `std_to_pr`, `exp_to_std`, `zonal_cutoff`, `zonal_filter`
                 -- the partial-regularity expansion and the zonal filter of
                    section 4 (`partial_regularity.py`).
  * `gl_nodes`, `gl_analysis` -- samples on the Gauss-Legendre grid -> exp-form
                    coefficients (section 5's interpolation for the SHT model,
                    `gl.py`).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dfs_direct.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               "-fno-fast-math", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _open(path):
    lib = ctypes.CDLL(path)
    sig = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
    for name in ("oracle_dfs_eval", "oracle_dfs_eval_ld"):
        fn = getattr(lib, name)
        fn.argtypes = sig
        fn.restype = ctypes.c_int
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = _open(_LIB)
    return _lib


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    _load().oracle_set_num_threads(int(n))


def _eval(fn_name, coeffs, phi, theta, lib=None):
    lib = lib or _load()
    c = np.asarray(coeffs, dtype=np.complex128)
    if c.ndim == 2:
        c = c[None]
    if c.ndim != 3:
        raise ValueError("coeffs must be (K_theta, K_phi) or (F, K_theta, K_phi)")
    c = np.ascontiguousarray(c)
    ph = np.ascontiguousarray(np.asarray(phi, dtype=np.float64).ravel())
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).ravel())
    if ph.shape != th.shape:
        raise ValueError("phi and theta must have the same length")
    F, Kt, Kp = c.shape
    out = np.empty((F, ph.size), dtype=np.complex128)
    rc = getattr(lib, fn_name)(c.ctypes.data, Kt, Kp, F, ph.ctypes.data,
                               th.ctypes.data, ph.size, out.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"{fn_name} failed ({rc})")
    return out


def load_variant(path):
    """Open another build of `dfs_direct.c` (used to check that the pins
    reject planted mistakes); returns an evaluator with `dfs_eval`'s signature."""
    lib = _open(path)
    return lambda coeffs, phi, theta: _eval("oracle_dfs_eval", coeffs, phi, theta, lib)


def dfs_eval(coeffs, phi, theta):
    """f_F(phi_j, theta_j) for every field F and point j, FP64 direct sum.

    coeffs: (K_theta, K_phi) or (F, K_theta, K_phi) complex, centred indices
    (row a <-> n = a - K_theta//2, column b <-> m = b - K_phi//2).
    Returns (F, P) complex128.
    """
    return _eval("oracle_dfs_eval", coeffs, phi, theta)


def dfs_eval_ld(coeffs, phi, theta):
    """As `dfs_eval`, accumulated in long double (certification only)."""
    return _eval("oracle_dfs_eval_ld", coeffs, phi, theta)


def std_to_exp(fc, fs):
    """Standard-DFS cos/sin coefficients -> exp-form coefficients (eq. dfs_fourier_coeffs).

    fc, fs: real arrays (N+1, M+1) indexed [n, m], n = 0..N, m = 0..M, holding
    the coefficients of the standard DFS basis (eq. std_dfs): for even m the
    theta factor is cos(n theta), for odd m it is sin(n theta); fc multiplies
    cos(m phi), fs multiplies sin(m phi).  Entries the basis does not use
    (fs[:, 0]; n = 0 for odd m) are ignored.

    Returns the centred (2N+1, 2M+1) complex array ft[n, m], n, m in
    [-N, N] x [-M, M].  The paper's printed map leaves out the m = 0, n >= 1
    entries and the sine part at n = 0 for even m; both are taken from the
    cos/sin-to-exponential identities: ft[+-n, 0] = fc[n, 0]/2 and
    ft[0, +-m] = (fc[0, m] -+ i fs[0, m])/2.
    """
    fc = np.asarray(fc, dtype=np.float64)
    fs = np.asarray(fs, dtype=np.float64)
    N, M = fc.shape[0] - 1, fc.shape[1] - 1
    ft = np.zeros((2 * N + 1, 2 * M + 1), dtype=np.complex128)

    def put(n, m, v):
        ft[n + N, m + M] += v

    put(0, 0, fc[0, 0])
    for n in range(1, N + 1):                      # m = 0, n >= 1
        put(n, 0, 0.5 * fc[n, 0])
        put(-n, 0, 0.5 * fc[n, 0])
    for m in range(1, M + 1):
        if m % 2 == 0:
            put(0, m, 0.5 * (fc[0, m] - 1j * fs[0, m]))
            put(0, -m, 0.5 * (fc[0, m] + 1j * fs[0, m]))
            for n in range(1, N + 1):
                a = 0.25 * (fc[n, m] - 1j * fs[n, m])
                b = 0.25 * (fc[n, m] + 1j * fs[n, m])
                put(n, m, a)
                put(-n, m, a)
                put(n, -m, b)
                put(-n, -m, b)
        else:
            for n in range(1, N + 1):              # n = 0 term vanishes (sin 0)
                a = -0.25 * (1j * fc[n, m] + fs[n, m])
                b = -0.25 * (1j * fc[n, m] - fs[n, m])
                put(n, m, a)
                put(-n, m, -a)
                put(n, -m, b)
                put(-n, -m, -b)
    return ft


def grid0_nodes(J):
    """Grid [0] of section 3 with J latitudes: theta_i = (i + 1/2) pi / J
    (i < J), phi_k = pi k / J (k < 2J)."""
    theta = (np.arange(J) + 0.5) * np.pi / J
    phi = np.arange(2 * J) * np.pi / J
    return theta, phi


def dfs_analysis(values):
    """Exp-form DFS coefficients of fields sampled on Grid [0] (section 4).

    values: real array [F][J][2J]; row i is colatitude theta_i, column k is
    longitude phi_k (`grid0_nodes`).  Truncation N = M = J - 1.

    Steps, as the paper orders them:
      1. Fourier transform in phi of every row: a_m(theta_i), b_m(theta_i),
         the cos(m phi) and sin(m phi) coefficients, m = 0 .. M.
      2. In theta, for each m: the cosine transform (even m, basis
         cos(n theta), n = 0 .. N) or the sine transform (odd m, basis
         sin(n theta), n = 1 .. N) of a_m and b_m on the half-offset nodes.
         This gives the standard-DFS coefficients fc[n, m], fs[n, m]
         (eq. std_dfs).
      3. `std_to_exp`: the map of eq. dfs_fourier_coeffs.
    Both transforms are the discrete orthogonality sums of their bases on
    these nodes, written out (no FFT).  The trigonometric factors of the node
    angles are taken at exactly reduced arguments: m phi_k = pi (m k mod 2J) / J
    and n theta_i = pi (n (2i + 1) mod 4J) / (2J), so that their rounding does
    not grow with m k or n i.

    Returns complex [F][2J-1][2J-1], centred (row a <-> n = a - (J-1)).
    """
    values = np.asarray(values, dtype=np.float64)
    if values.ndim == 2:
        values = values[None]
    F, J, L = values.shape
    if L != 2 * J:
        raise ValueError("values must be [F][J][2J]")
    N = M = J - 1
    m = np.arange(M + 1)
    n = np.arange(N + 1)
    k = np.arange(2 * J)
    i = np.arange(J)
    # 1. phi: f(phi) = a_0 + sum_{m>=1} a_m cos(m phi) + b_m sin(m phi)
    arg_p = np.pi * (np.outer(k, m) % (2 * J)) / J            # m phi_k, [2J, M+1]
    cos_pm = np.cos(arg_p)
    sin_pm = np.sin(arg_p)
    a = values @ cos_pm / J                      # [F, J, M+1]
    a[..., 0] *= 0.5
    b = values @ sin_pm / J
    # 2. theta: g(theta) = sum_n c_n cos(n theta)  or  sum_{n>=1} s_n sin(n theta)
    w_cos = np.full(N + 1, 2.0 / J)
    w_cos[0] = 1.0 / J
    arg_t = np.pi * (np.outer(n, 2 * i + 1) % (4 * J)) / (2 * J)   # n theta_i, [N+1, J]
    proj_cos = w_cos[:, None] * np.cos(arg_t)
    proj_sin = (2.0 / J) * np.sin(arg_t)
    proj_sin[0] = 0.0
    even = (m % 2 == 0)[None, :]
    out = np.empty((F, 2 * N + 1, 2 * M + 1), dtype=np.complex128)
    for f in range(F):
        fc = np.where(even, proj_cos @ a[f], proj_sin @ a[f])    # [N+1, M+1]
        fs = np.where(even, proj_cos @ b[f], proj_sin @ b[f])
        fs[:, 0] = 0.0
        # 3. eq. dfs_fourier_coeffs
        out[f] = std_to_exp(fc, fs)
    return out


def rotation_pq(phi_a, theta_a, phi_d, theta_d):
    """Entries p, q of the rotation Q = [[p, q], [-q, p]] of section 3 (after
    eq. sslforceb), FP64: phi longitude, theta colatitude, A arrival, D
    departure;

        p = (sin th_A sin th_D + (1 + cos th_A cos th_D) cos(ph_A - ph_D)) / (1 + cos eta)
        q = (cos th_A + cos th_D) sin(ph_A - ph_D) / (1 + cos eta)

    with cos eta = r_A . r_D for the unit position vectors.  Undefined for
    antipodal pairs (1 + cos eta = 0)."""
    pa, ta, pd, td = (np.asarray(x, dtype=np.float64) for x in (phi_a, theta_a, phi_d, theta_d))
    sa, ca, sd, cd = np.sin(ta), np.cos(ta), np.sin(td), np.cos(td)
    dphi = pa - pd
    cos_eta = sa * sd * np.cos(dphi) + ca * cd
    den = 1.0 + cos_eta
    p = (sa * sd + (1.0 + ca * cd) * np.cos(dphi)) / den
    q = (ca + cd) * np.sin(dphi) / den
    return p, q


def rotate_uv(u, v, phi_a, theta_a, phi_d, theta_d):
    """(u, v) at the departure points (east, north components) expressed at
    the arrival points: (p u + q v, -q u + p v)."""
    p, q = rotation_pq(phi_a, theta_a, phi_d, theta_d)
    return p * u + q * v, -q * u + p * v


from .partial_regularity import (  # noqa: E402,F401
    exp_to_std, normal_system, pr_range, pr_to_std, std_to_pr, std_weights,
    zonal_cutoff, zonal_filter, zonal_limit,
)
from .gl import gl_analysis, gl_latitude_matrices, gl_nodes  # noqa: E402,F401
