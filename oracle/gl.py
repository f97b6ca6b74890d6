"""ORACLE (test infrastructure only) -- DFS coefficients from samples on the
Gauss-Legendre grid (section 2, eq. GLGrid; section 5, the interpolation for
the SHT model).

Grid: J colatitudes theta_j = arccos(z_j), z_j the roots of the degree-J
Legendre polynomial, in increasing theta (row j); 2J longitudes
phi_k = pi k / J (column k).

Steps, in the paper's order:
  1. the Fourier transform in longitude of every row (numpy's FFT as the
     library step): g_m(theta_j) = (1/2J) sum_k f(phi_k, theta_j) e^{-i m phi_k},
     |m| <= J - 1 (the m = J Nyquist mode is dropped, as on Grid [0]);
  2. in latitude, for each m, the direct inversion of the latitude "DFT"
     matrix with an LU factorisation computed once per parity and applied to
     every m of that parity (scipy.linalg.lu_factor / lu_solve):  even m take the
     cosine basis cos(n theta), n = 0 .. J-1; odd m the sine basis
     sin(n theta), n = 1 .. J (reading R22: the standard DFS parities of
     eq. std_dfs with as many basis functions as latitudes, so that the
     samples are interpolated);
  3. the exp form of eq. std_dfs_exp: cos(n theta) = (e^{in theta} +
     e^{-in theta}) / 2 and sin(n theta) = (e^{in theta} - e^{-in theta}) / (2i).
Output: [F][2J+1][2J-1] complex, centred (row a <-> n = a - J, column
b <-> m = b - (J - 1)).
"""
from __future__ import annotations

import numpy as np


def _legendre_and_derivative(J, z):
    """P_J(z) and P_J'(z) by the three-term recurrence (elementwise)."""
    p0, p1 = np.ones_like(z), z
    for n in range(2, J + 1):
        p0, p1 = p1, ((2 * n - 1) * z * p1 - (n - 1) * p0) / n
    if J == 1:
        p0 = np.ones_like(z)
    return p1, J * (z * p1 - p0) / (z * z - 1)


def _gl_theta_ld(J: int):
    """Colatitudes of the Legendre roots in numpy's long double: numpy's
    Gauss-Legendre nodes as the start, then Newton steps in theta on
    P_J(cos theta) (an FP64 cosine near the poles only fixes theta to
    ~1e-14, because d theta = dz / sin theta)."""
    z, _ = np.polynomial.legendre.leggauss(J)
    th = np.sort(np.arccos(z)).astype(np.longdouble)
    for _ in range(3):
        p, dp = _legendre_and_derivative(J, np.cos(th))
        th = th + p / (np.sin(th) * dp)          # d/dtheta P_J(cos theta) = -sin(theta) P_J'
    return th


def gl_nodes(J: int):
    """(theta [J] increasing, phi [2J]) of the Gauss-Legendre grid, FP64."""
    theta = _gl_theta_ld(J).astype(np.float64)
    phi = np.arange(2 * J) * np.pi / J
    return theta, phi


def gl_latitude_matrices(J: int):
    """C_even[j, n] = cos(n theta_j), n = 0..J-1; C_odd[j, n] = sin((n+1) theta_j),
    evaluated in long double at the long-double nodes and rounded to FP64."""
    th = _gl_theta_ld(J)
    n = np.arange(J, dtype=np.longdouble)
    return (np.cos(np.outer(th, n)).astype(np.float64),
            np.sin(np.outer(th, n + 1)).astype(np.float64))


def gl_analysis(values):
    values = np.asarray(values, dtype=np.float64)
    if values.ndim == 2:
        values = values[None]
    F, J, L = values.shape
    if L != 2 * J:
        raise ValueError("values must be [F][J][2J]")
    from scipy.linalg import lu_factor, lu_solve
    g = np.fft.fft(values, axis=2) / (2 * J)             # [F, J, 2J]: m mod 2J
    Ce, Co = gl_latitude_matrices(J)
    lu = (lu_factor(Ce), lu_factor(Co))
    out = np.zeros((F, 2 * J + 1, 2 * J - 1), dtype=np.complex128)
    n = np.arange(1, J)
    for parity in (0, 1):
        ms = [m for m in range(-(J - 1), J) if m % 2 == parity]
        cols = np.array(ms) + J - 1
        rhs = g[:, :, np.array(ms) % (2 * J)]            # [F, J, #m]
        rhs = np.moveaxis(rhs, 1, 0).reshape(J, -1)      # [J, F * #m]
        x = lu_solve(lu[parity], rhs).reshape(J, F, len(ms))
        if parity == 0:                                  # cos(n theta), n = 0..J-1
            out[:, J, cols] = x[0]
            half = np.moveaxis(x[1:], 0, 1) / 2          # [F, J-1, #m]
            out[:, (J + n)[:, None], cols[None, :]] = half
            out[:, (J - n)[:, None], cols[None, :]] = half
        else:                                            # sin(n theta), n = 1..J
            b = np.moveaxis(x, 0, 1)                     # [F, J, #m], row k <-> n = k + 1
            nn = np.arange(1, J + 1)
            out[:, (J + nn)[:, None], cols[None, :]] = -0.5j * b
            out[:, (J - nn)[:, None], cols[None, :]] = 0.5j * b
    return out
