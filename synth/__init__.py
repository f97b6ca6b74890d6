"""Seeded synthetic inputs for the DFS departure-point interpolation.

This module only draws inputs: coefficient arrays, lat-lon node sets and
departure points.  It holds none of the interpolation arithmetic, so the CPU
oracle and the HIP path can both consume what it produces without sharing any
computation.

Conventions (see the paper, sections 3 and 5):
  * theta is colatitude, phi is longitude; on the doubled torus both are
    2*pi-periodic.
  * A coefficient array has shape (K_theta, K_phi) (or (F, K_theta, K_phi)),
    complex, with centred indices: row a <-> n = a - K_theta//2 (theta mode),
    column b <-> m = b - K_phi//2 (phi mode).
  * Points come as two float64 arrays (phi, theta).
"""
from __future__ import annotations

import numpy as np

EARTH_RADIUS = 6.37122e6          # metres (Williamson test-case radius)
DAY = 86400.0


# --------------------------------------------------------------------------
# Grids (section 3, eq. of the grid types: Grid [0])
# --------------------------------------------------------------------------
def grid0_axes(J: int):
    """Grid [0]: theta_j = (j + 1/2) pi / J, j < J;  phi_k = pi k / J, k < 2J."""
    theta = (np.arange(J, dtype=np.float64) + 0.5) * np.pi / J
    phi = np.arange(2 * J, dtype=np.float64) * np.pi / J
    return theta, phi


def grid0_points(J: int):
    """All N_lat * M_lon = 2 J^2 Grid [0] nodes, theta-major (phi fastest)."""
    theta, phi = grid0_axes(J)
    T, P = np.meshgrid(theta, phi, indexing="ij")
    return P.ravel().copy(), T.ravel().copy()


# --------------------------------------------------------------------------
# Coefficients
# --------------------------------------------------------------------------
def mode_axis(K: int) -> np.ndarray:
    return np.arange(K, dtype=np.int64) - K // 2


def envelope_gauss(K_theta: int, K_phi: int, scale: float = 200.0):
    n = mode_axis(K_theta)[:, None].astype(np.float64)
    m = mode_axis(K_phi)[None, :].astype(np.float64)
    return np.exp(-(n * n + m * m) / scale)


def envelope_algebraic(K_theta: int, K_phi: int, p: float = 1.5):
    n = mode_axis(K_theta)[:, None].astype(np.float64)
    m = mode_axis(K_phi)[None, :].astype(np.float64)
    return (1.0 + n * n + m * m) ** (-p)


def symmetrize_dfs_real(Z: np.ndarray) -> np.ndarray:
    """Project a centred (K, K) array (odd K) onto coefficients of a real DFS field.

    First the glide projection  Y[n,m] = (Z[n,m] + (-1)^m Z[-n,m]) / 2,
    then the Hermitian one      X[n,m] = (Y[n,m] + conj Y[-n,-m]) / 2.
    Both symmetries survive the composition (the glide one commutes with
    the Hermitian one), so X is the exp-form coefficient array of a real
    field that has the DFS parity of section 4.
    """
    Kt, Kp = Z.shape
    if Kt % 2 == 0 or Kp % 2 == 0:
        raise ValueError("symmetrization needs odd mode counts")
    m = mode_axis(Kp)
    sign = np.where(m % 2 == 0, 1.0, -1.0)[None, :]
    Y = 0.5 * (Z + sign * Z[::-1, :])
    X = 0.5 * (Y + np.conj(Y[::-1, ::-1]))
    return X


def random_complex(rng: np.random.Generator, shape):
    """i.i.d. N(0,1) real parts, then i.i.d. N(0,1) imaginary parts."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return re + 1j * im


def dfs_field_coeffs(rng, K_theta, K_phi, envelope):
    """Coefficients of a real band-limited DFS field with the given envelope."""
    Z = random_complex(rng, (K_theta, K_phi))
    return symmetrize_dfs_real(Z) * envelope


# --------------------------------------------------------------------------
# Departure points
# --------------------------------------------------------------------------
def sph_to_cart(phi, theta):
    st = np.sin(theta)
    return np.stack([st * np.cos(phi), st * np.sin(phi), np.cos(theta)], axis=-1)


def cart_to_sph(x):
    r = np.linalg.norm(x, axis=-1)
    theta = np.arccos(np.clip(x[..., 2] / r, -1.0, 1.0))
    phi = np.mod(np.arctan2(x[..., 1], x[..., 0]), 2 * np.pi)
    return phi, theta


def rotate(x, axis, angle):
    """Rodrigues rotation of row vectors x about a unit axis by angle."""
    axis = np.asarray(axis, dtype=np.float64)
    axis = axis / np.linalg.norm(axis)
    c, s = np.cos(angle), np.sin(angle)
    return (x * c + np.cross(axis, x) * s
            + np.outer(x @ axis, axis) * (1.0 - c))


def sbr_axis(alpha: float):
    """Rotation axis of the Williamson solid-body-rotation wind tilted by alpha."""
    return np.array([-np.sin(alpha), 0.0, np.cos(alpha)])


def sbr_departures(phi_a, theta_a, alpha, u0, dt, a=EARTH_RADIUS):
    """Exact departure points of a solid-body rotation: rotate back by u0 dt / a."""
    x = sph_to_cart(phi_a, theta_a)
    xd = rotate(x, sbr_axis(alpha), -(u0 / a) * dt)
    return cart_to_sph(xd)


def _real_sph_harm(l, m, theta, phi, diff):
    """Real spherical harmonic (or its theta/phi derivatives) from scipy's complex one."""
    from scipy.special import sph_harm_y
    res = sph_harm_y(l, abs(m), theta, phi, diff_n=1 if diff else 0)
    if diff:
        y, d = res
        d_theta, d_phi = d[..., 0], d[..., 1]
        pick = (lambda z: z.real) if m >= 0 else (lambda z: z.imag)
        return pick(d_theta), pick(d_phi)
    pick = (lambda z: z.real) if m >= 0 else (lambda z: z.imag)
    return pick(res)


class StreamFunctionWind:
    """Divergence-free wind v = r_hat x grad(psi) of a random low-mode stream function.

    psi = sum_q a_q Y_{l_q m_q}: real spherical harmonics with (l, m) drawn
    without replacement from 1 <= l <= lmax, a_q ~ N(0, 1).  The wind is held
    as a non-dimensional angular displacement per step; `scale` is set so the
    largest displacement over a node set equals a target Courant number.
    """

    def __init__(self, rng, n_modes=8, lmax=4):
        pairs = [(l, m) for l in range(1, lmax + 1) for m in range(-l, l + 1)]
        idx = rng.choice(len(pairs), size=n_modes, replace=False)
        self.modes = [pairs[i] for i in idx]
        self.amps = rng.standard_normal(n_modes)
        self.scale = 1.0

    def tangent_wind(self, phi, theta):
        """(v_theta, v_phi) components of r_hat x grad psi (unit sphere)."""
        g_t = np.zeros_like(theta)
        g_p = np.zeros_like(theta)
        for (l, m), c in zip(self.modes, self.amps):
            dt, dp = _real_sph_harm(l, m, theta, phi, True)
            g_t += c * dt
            g_p += c * dp
        st = np.sin(theta)
        st = np.where(np.abs(st) < 1e-300, 1e-300, st)
        # grad psi = d_theta psi e_theta + (1/sin) d_phi psi e_phi
        # r_hat x e_theta = e_phi, r_hat x e_phi = -e_theta
        v_theta = -(g_p / st)
        v_phi = g_t
        return self.scale * v_theta, self.scale * v_phi

    def cart_wind(self, x):
        phi, theta = cart_to_sph(x)
        vt, vp = self.tangent_wind(phi, theta)
        ct, stt = np.cos(theta), np.sin(theta)
        cp, sp = np.cos(phi), np.sin(phi)
        e_t = np.stack([ct * cp, ct * sp, -stt], axis=-1)
        e_p = np.stack([-sp, cp, np.zeros_like(sp)], axis=-1)
        return vt[:, None] * e_t + vp[:, None] * e_p

    def normalize_courant(self, phi, theta, courant, n_lat):
        """Scale so max |v| over the given nodes equals courant * (pi / n_lat)."""
        self.scale = 1.0
        vt, vp = self.tangent_wind(phi, theta)
        vmax = np.max(np.hypot(vt, vp))
        self.scale = courant * (np.pi / n_lat) / vmax

    def departures(self, phi_a, theta_a, iters=2):
        """Backward trajectory: x_D = x_A - v(midpoint), midpoint fixed-point iteration."""
        xa = sph_to_cart(phi_a, theta_a)
        xd = xa.copy()
        for _ in range(iters):
            mid = xa + xd
            mid /= np.linalg.norm(mid, axis=-1, keepdims=True)
            xd = xa - self.cart_wind(mid)
            xd /= np.linalg.norm(xd, axis=-1, keepdims=True)
        return cart_to_sph(xd)


# --------------------------------------------------------------------------
# Workloads (the five configurations of the benchmark suite)
# --------------------------------------------------------------------------
class Workload:
    """One departure-point set with F coefficient fields, all float64/complex128."""

    def __init__(self, name, J, coeffs, phi, theta, meta=None):
        self.name = name
        self.J = J
        self.coeffs = coeffs            # (F, K, K) complex128
        self.phi = phi                  # (P,) float64
        self.theta = theta              # (P,) float64
        self.meta = meta or {}

    @property
    def n_fields(self):
        return self.coeffs.shape[0]

    @property
    def n_pts(self):
        return self.phi.shape[0]


def workload_small_jitter(J=32, seed=0, amp=0.05):
    """32x64 Grid [0] nodes jittered by U[-amp, amp] rad, one Gaussian-envelope field."""
    K = 2 * J - 1
    rng = np.random.default_rng(seed)
    F = dfs_field_coeffs(rng, K, K, envelope_gauss(K, K))
    phi0, theta0 = grid0_points(J)
    off = rng.uniform(-amp, amp, size=(2, phi0.size))
    phi = phi0 + off[0]
    theta = theta0 + off[1]
    # wrap onto the torus: any real value is a valid torus coordinate
    phi = np.mod(phi, 2 * np.pi)
    theta = np.mod(theta, 2 * np.pi)
    return Workload("grid32x64_jitter_gauss", J, F[None], phi, theta,
                    {"envelope": "gauss200", "seed": seed})


def workload_sbr(J=256, seeds=(1, 2, 3), alpha=np.pi / 4, dt=1200.0):
    """256x512 nodes displaced back along a solid-body rotation; h, u, v fields."""
    K = 2 * J - 1
    env = envelope_algebraic(K, K, 1.5)
    F = np.stack([dfs_field_coeffs(np.random.default_rng(s), K, K, env) for s in seeds])
    phi_a, theta_a = grid0_points(J)
    u0 = 2 * np.pi * EARTH_RADIUS / (12 * DAY)
    phi, theta = sbr_departures(phi_a, theta_a, alpha, u0, dt)
    return Workload(f"grid{J}x{2*J}_sbr", J, F, phi, theta,
                    {"alpha": alpha, "dt": dt, "u0": u0, "seeds": list(seeds)})


def workload_wind(J, field_seeds, wind_seed, courant, p=1.5, name=None):
    """J x 2J nodes displaced by a random 8-mode stream-function wind."""
    K = 2 * J - 1
    env = envelope_algebraic(K, K, p)
    F = np.stack([dfs_field_coeffs(np.random.default_rng(s), K, K, env) for s in field_seeds])
    phi_a, theta_a = grid0_points(J)
    wind = StreamFunctionWind(np.random.default_rng(wind_seed))
    wind.normalize_courant(phi_a, theta_a, courant, J)
    phi, theta = wind.departures(phi_a, theta_a)
    return Workload(name or f"grid{J}x{2*J}_wind", J, F, phi, theta,
                    {"courant": courant, "wind_seed": wind_seed, "p": p,
                     "field_seeds": list(field_seeds)})


def workload_large(J=1024):
    """1024x2048 nodes, 3 fields (seeds 11-13), 8-mode wind (seed 14), max Courant 8."""
    return workload_wind(J, (11, 12, 13), 14, 8.0, name=f"grid{J}x{2*J}_wind_c8")


def sample_indices(n_pts, n_sample, seed=15):
    if n_sample >= n_pts:
        return np.arange(n_pts)
    return np.sort(np.random.default_rng(seed).choice(n_pts, n_sample, replace=False))


def ensemble_members(n_small=64, n_large=16, J_small=128, J_large=256):
    """Member specs of the uneven ensemble: own seed, spectrum exponent and Courant."""
    specs = []
    for i in range(n_small + n_large):
        rng = np.random.default_rng(1000 + i)
        p = rng.uniform(1.0, 2.0)
        c = rng.uniform(2.0, 8.0)
        J = J_small if i < n_small else J_large
        specs.append({"index": i, "J": J, "p": p, "courant": c, "seed": 1000 + i})
    return specs


def ensemble_member(spec, n_fields=3):
    s = spec["seed"]
    return workload_wind(spec["J"], tuple(10 * s + f for f in range(n_fields)),
                         10 * s + 9, spec["courant"], p=spec["p"],
                         name=f"member{spec['index']}_J{spec['J']}")
