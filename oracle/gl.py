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
     matrix with an LU factorisation (numpy.linalg.solve):  even m take the
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


def gl_nodes(J: int):
    """(theta [J] increasing, phi [2J]) of the Gauss-Legendre grid."""
    z, _ = np.polynomial.legendre.leggauss(J)
    theta = np.sort(np.arccos(z))
    phi = np.arange(2 * J) * np.pi / J
    return theta, phi


def gl_latitude_matrices(J: int):
    """C_even[j, n] = cos(n theta_j), n = 0..J-1; C_odd[j, n] = sin((n+1) theta_j)."""
    theta, _ = gl_nodes(J)
    n = np.arange(J)
    return np.cos(np.outer(theta, n)), np.sin(np.outer(theta, n + 1))


def gl_analysis(values):
    values = np.asarray(values, dtype=np.float64)
    if values.ndim == 2:
        values = values[None]
    F, J, L = values.shape
    if L != 2 * J:
        raise ValueError("values must be [F][J][2J]")
    g = np.fft.fft(values, axis=2) / (2 * J)             # [F, J, 2J]: m mod 2J
    Ce, Co = gl_latitude_matrices(J)
    out = np.zeros((F, 2 * J + 1, 2 * J - 1), dtype=np.complex128)
    for m in range(-(J - 1), J):
        col = m + J - 1
        rhs = g[:, :, m % (2 * J)].T                     # [J, F]
        if m % 2 == 0:
            a = np.linalg.solve(Ce, rhs)                 # cos(n theta), n = 0..J-1
            out[:, J, col] = a[0]
            for n in range(1, J):
                out[:, J + n, col] = a[n] / 2
                out[:, J - n, col] = a[n] / 2
        else:
            b = np.linalg.solve(Co, rhs)                 # sin(n theta), n = 1..J
            for n in range(1, J + 1):
                out[:, J + n, col] = -0.5j * b[n - 1]
                out[:, J - n, col] = 0.5j * b[n - 1]
    return out
