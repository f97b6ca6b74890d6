"""ORACLE (test infrastructure only) -- the partial-regularity DFS expansion
and the zonal filter of section 4.

The partial-regularity basis (eq. pr_dfs) multiplies cos(m phi) and
sin(m phi) by these theta factors:

    m = 0          cos(n theta)                 n = 0 .. N
    m = 1          sin(theta) cos(n theta)      n = 0 .. N-1
    m >= 2 even    sin(theta) sin(n theta)      n = 1 .. N-1
    m >= 3 odd     sin^2(theta) sin(n theta)    n = 1 .. N-2

Coefficient arrays are real [N+1, M+1] indexed [n, m]: pc multiplies
cos(m phi), ps multiplies sin(m phi); entries outside a column's index range
(and ps[:, 0]) are zero on output and ignored on input.  Standard-DFS
coefficients (eq. std_dfs) use the same layout: fc, fs with cos(n theta) for
even m and sin(n theta) for odd m.

Functions
  * `pr_to_std`   -- the conversion printed after eq. std_dfs, one formula
                     per class of m, with reading R19 (below).
  * `std_to_pr`   -- the least-squares projection: for each m, the
                     orthogonality conditions of the residual against the
                     column's basis (section 4) as a linear system, solved
                     densely.
  * `exp_to_std`  -- exp-form -> standard coefficients: the least-squares
                     inverse of eq. dfs_fourier_coeffs (exact on the image of
                     `std_to_exp`).
  * `zonal_cutoff`, `zonal_filter` -- the filter M_zf(theta) =
                     min(M, M0 + M sin theta), M0 = 20, applied per Grid [0]
                     latitude to the longitudinal Fourier modes.

Reading R19: for even m >= 2 the paper prints the n = 0 standard
coefficient as 0.  Since sin(theta) sin(theta) = (1 - cos(2 theta)) / 2, the
n = 1 basis function has the constant term 1/2, so the standard n = 0
coefficient is f_{1,m} / 2; only this value makes the series vanish at the
poles, the property stated after eq. pr_dfs.  The pins evaluate the basis
functions directly and fail the printed value.
"""
from __future__ import annotations

import numpy as np


def pr_range(m: int, N: int):
    """Index range (lo, hi), inclusive, of the pr theta factors of column m."""
    if m == 0:
        return 0, N
    if m == 1:
        return 0, N - 1
    if m % 2 == 0:
        return 1, N - 1
    return 1, N - 2


def _pr_column_to_std(f, m, N):
    """Standard theta coefficients t[0..N] of one pr column f[0..N] (section 4
    conversion formulas; f_k = 0 outside the column's range)."""
    lo, hi = pr_range(m, N)

    def F(k):
        return f[k] if lo <= k <= hi else 0.0

    t = np.zeros(N + 1)
    if m == 0:
        for n in range(N + 1):
            t[n] = F(n)
    elif m == 1:
        t[1] = 0.5 * (2.0 * F(0) - F(2))
        for n in range(2, N - 1):
            t[n] = 0.5 * (F(n - 1) - F(n + 1))
        for n in (N - 1, N):
            t[n] = 0.5 * F(n - 1)
    elif m % 2 == 0:
        t[0] = 0.5 * F(1)                       # reading R19 (printed: 0)
        t[1] = 0.5 * F(2)
        for n in range(2, N - 1):
            t[n] = 0.5 * (-F(n - 1) + F(n + 1))
        for n in (N - 1, N):
            t[n] = -0.5 * F(n - 1)
    else:
        t[1] = 0.25 * (3.0 * F(1) - F(3))
        t[2] = 0.25 * (2.0 * F(2) - F(4))
        for n in range(3, N - 2):
            t[n] = 0.25 * (-F(n - 2) + 2.0 * F(n) - F(n + 2))
        for n in (N - 2, N - 1):
            t[n] = 0.25 * (-F(n - 2) + 2.0 * F(n))
        t[N] = -0.25 * F(N - 2)
    return t


def _check_shape(a):
    a = np.asarray(a, dtype=np.float64)
    if a.ndim != 2 or a.shape[0] < 6:
        raise ValueError("coefficients must be [N+1, M+1] with N >= 5")
    return a


def pr_to_std(pc, ps):
    """Partial-regularity -> standard DFS coefficients (section 4, the
    conversion after eq. std_dfs).  Returns (fc, fs)."""
    pc, ps = _check_shape(pc), _check_shape(ps)
    N, M = pc.shape[0] - 1, pc.shape[1] - 1
    fc = np.zeros_like(pc)
    fs = np.zeros_like(ps)
    for m in range(M + 1):
        fc[:, m] = _pr_column_to_std(pc[:, m], m, N)
        if m > 0:
            fs[:, m] = _pr_column_to_std(ps[:, m], m, N)
    return fc, fs


def std_weights(m: int, N: int):
    """int_0^pi of the squared standard theta factors: cos(n theta) for even
    m (pi at n = 0, pi/2 otherwise), sin(n theta) for odd m (0 at n = 0,
    pi/2 otherwise)."""
    w = np.full(N + 1, np.pi / 2)
    w[0] = np.pi if m % 2 == 0 else 0.0
    return w


def conversion_matrix(m: int, N: int):
    """A[:, j] = standard coefficients of the j-th pr theta factor of column
    m (j = lo .. hi), from `_pr_column_to_std` on unit vectors."""
    lo, hi = pr_range(m, N)
    A = np.zeros((N + 1, hi - lo + 1))
    for j in range(lo, hi + 1):
        e = np.zeros(N + 1)
        e[j] = 1.0
        A[:, j - lo] = _pr_column_to_std(e, m, N)
    return A


def normal_system(m: int, N: int):
    """Gram matrix G[j, k] = int_0^pi B_j B_k dtheta of the pr theta factors
    of column m and the map b -> rhs[k] = int_0^pi (sum_n b_n T_n) B_k
    dtheta from standard coefficients b (T_n the standard theta factors):
    G = A^T W A, R = A^T W with W = diag(std_weights)."""
    A = conversion_matrix(m, N)
    W = std_weights(m, N)
    return A.T @ (W[:, None] * A), A.T * W[None, :]


def std_to_pr(fc, fs):
    """Least-squares projection of standard DFS coefficients onto the
    partial-regularity basis (section 4): for every m and both the cos(m phi)
    and sin(m phi) parts, the coefficients x of the column's basis B_j solve
    sum_j x_j int B_j B_k = int fbar_m B_k for all k in the column's range
    (the residual is orthogonal to every B_k), which is the minimiser of the
    L2 error E_2.  m = 0 reduces to the identity."""
    fc, fs = _check_shape(fc), _check_shape(fs)
    N, M = fc.shape[0] - 1, fc.shape[1] - 1
    pc = np.zeros_like(fc)
    ps = np.zeros_like(fs)
    # the system depends only on the class of m (0, 1, even >= 2, odd >= 3):
    # one LU factorisation per class, applied to all of its columns
    from scipy.linalg import lu_factor, lu_solve
    classes = {0: [0], 1: [1] if M >= 1 else [], 2: list(range(2, M + 1, 2)), 3: list(range(3, M + 1, 2))}
    for key, ms in classes.items():
        if not ms:
            continue
        G, R = normal_system(ms[0], N)
        lu = lu_factor(G)
        lo, hi = pr_range(ms[0], N)
        pc[lo:hi + 1, ms] = lu_solve(lu, R @ fc[:, ms])
        if key > 0:
            ps[lo:hi + 1, ms] = lu_solve(lu, R @ fs[:, ms])
    return pc, ps


def exp_to_std(ft):
    """Exp-form coefficients [2N+1, 2M+1] (centred) -> standard (fc, fs).

    For each (n, m) with n, m >= 0, the real pair (fc[n, m], fs[n, m]) that
    eq. dfs_fourier_coeffs maps closest (least squares) to the given entries
    at (+-n, +-m).  Writing the entries e(n, m):
      m = 0:          fc[0, 0] = Re e(0, 0);  fc[n, 0] = Re(e(n, 0) + e(-n, 0))
      even m >= 2:    fc[n, m] = Re of the sum of the four entries,
                      fs[n, m] = Im(e(n,-m) + e(-n,-m) - e(n,m) - e(-n,m));
                      n = 0: fc = Re(e(0,m) + e(0,-m)), fs = Im(e(0,-m) - e(0,m))
      odd m:          with S = e(n,m) - e(-n,m) + e(n,-m) - e(-n,-m) and
                      D = e(n,-m) - e(-n,-m) - e(n,m) + e(-n,m):
                      fc[n, m] = -Im S,  fs[n, m] = Re D   (n >= 1)
    """
    ft = np.asarray(ft, dtype=np.complex128)
    N, M = (ft.shape[0] - 1) // 2, (ft.shape[1] - 1) // 2

    def e(n, m):
        return ft[n + N, m + M]

    fc = np.zeros((N + 1, M + 1))
    fs = np.zeros((N + 1, M + 1))
    fc[0, 0] = e(0, 0).real
    for n in range(1, N + 1):
        fc[n, 0] = (e(n, 0) + e(-n, 0)).real
    for m in range(1, M + 1):
        if m % 2 == 0:
            fc[0, m] = (e(0, m) + e(0, -m)).real
            fs[0, m] = (e(0, -m) - e(0, m)).imag
            for n in range(1, N + 1):
                fc[n, m] = (e(n, m) + e(-n, m) + e(n, -m) + e(-n, -m)).real
                fs[n, m] = (e(n, -m) + e(-n, -m) - e(n, m) - e(-n, m)).imag
        else:
            for n in range(1, N + 1):
                S = e(n, m) - e(-n, m) + e(n, -m) - e(-n, -m)
                D = e(n, -m) - e(-n, -m) - e(n, m) + e(-n, m)
                fc[n, m] = -S.imag
                fs[n, m] = D.real
    return fc, fs


def zonal_limit(J: int, M0: float = 20.0):
    """M_zf at the Grid [0] colatitudes theta_i = (i + 1/2) pi / J, with the
    truncation M = J - 1 of the Grid [0] expansion (FP64)."""
    M = J - 1
    theta = (np.arange(J) + 0.5) * np.pi / J
    return np.minimum(float(M), M0 + M * np.sin(theta))


def zonal_cutoff(J: int, M0: float = 20.0):
    """Largest kept longitudinal wavenumber per latitude: m is zeroed when
    m > M_zf, so the kept ones are m <= floor(M_zf)."""
    return np.floor(zonal_limit(J, M0)).astype(np.int64)


def zonal_filter(values, M0: float = 20.0):
    """Zonal filter of section 4 on Grid [0] samples [F][J][2J] (or [J][2J]):
    at each latitude the longitudinal Fourier components with wavenumber
    m > M_zf(theta_i) are removed (numpy's real FFT along phi)."""
    v = np.asarray(values, dtype=np.float64)
    squeeze = v.ndim == 2
    if squeeze:
        v = v[None]
    F, J, L = v.shape
    if L != 2 * J:
        raise ValueError("values must be [F][J][2J]")
    spec = np.fft.rfft(v, axis=2)                    # m = 0 .. J
    m = np.arange(J + 1)
    lim = zonal_limit(J, M0)
    spec[:, m[None, :] > lim[:, None]] = 0.0
    out = np.fft.irfft(spec, n=2 * J, axis=2)
    return out[0] if squeeze else out
