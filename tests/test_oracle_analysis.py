"""Pins of the oracle's DFS analysis (grid values on Grid [0] -> exp-form
coefficients, section 4 and eq. dfs_fourier_coeffs).

Each pin reaches the answer by another route than the analysis' own sums:
the synthesis (the pinned direct sum of eq. std_dfs_exp), closed-form single
modes, a least-squares fit of the basis at the nodes, and numpy's FFT over
the glide-doubled torus.
"""
import numpy as np
import pytest

import oracle


def random_std(rng, J):
    """Random standard-DFS coefficients of the basis of eq. std_dfs, N = M = J - 1."""
    N = M = J - 1
    fc = rng.standard_normal((N + 1, M + 1))
    fs = rng.standard_normal((N + 1, M + 1))
    fs[:, 0] = 0.0                     # no sin(0 phi) term
    for m in range(1, M + 1, 2):       # odd m: sin(n theta), n >= 1
        fc[0, m] = fs[0, m] = 0.0
    return fc, fs


def sample(ft, J):
    """Values of the exp-form series at the Grid [0] nodes (pinned direct sum)."""
    th, ph = oracle.grid0_nodes(J)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    v = oracle.dfs_eval(ft[None], PH.ravel(), TH.ravel()).reshape(J, 2 * J)
    assert np.abs(v.imag).max() < 1e-12 * max(1.0, np.abs(v).max())
    return v.real


@pytest.mark.parametrize("J", [1, 2, 3, 6, 16, 33])
def test_analysis_inverts_synthesis_at_the_nodes(J):
    rng = np.random.default_rng(J)
    fc, fs = random_std(rng, J)
    ft = oracle.std_to_exp(fc, fs)
    back = oracle.dfs_analysis(sample(ft, J))[0]
    assert np.abs(back - ft).max() <= 1e-13 * max(1.0, np.abs(ft).max())


def test_single_modes_closed_form():
    J = 8
    th, ph = oracle.grid0_nodes(J)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    N = M = J - 1
    cases = [
        (np.cos(2 * PH) * np.cos(3 * TH), ("c", 3, 2)),
        (np.sin(4 * PH) * np.cos(5 * TH), ("s", 5, 4)),
        (np.cos(3 * PH) * np.sin(2 * TH), ("c", 2, 3)),
        (np.sin(5 * PH) * np.sin(1 * TH), ("s", 1, 5)),
        (np.full_like(TH, 2.5), ("c", 0, 0)),
        (np.cos(4 * TH), ("c", 4, 0)),
    ]
    for vals, (kind, n, m) in cases:
        fc = np.zeros((N + 1, M + 1))
        fs = np.zeros((N + 1, M + 1))
        (fc if kind == "c" else fs)[n, m] = 2.5 if (n, m) == (0, 0) else 1.0
        want = oracle.std_to_exp(fc, fs)
        got = oracle.dfs_analysis(vals)[0]
        assert np.abs(got - want).max() < 1e-14, (kind, n, m)


@pytest.mark.parametrize("J", [3, 4])
def test_least_squares_fit_of_the_basis(J):
    """Brute force: fit the standard basis to the node values by least squares."""
    rng = np.random.default_rng(100 + J)
    vals = rng.standard_normal((J, 2 * J))
    th, ph = oracle.grid0_nodes(J)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    N = M = J - 1
    cols, keys = [], []
    for m in range(M + 1):
        for n in range(N + 1):
            if m % 2 == 0:
                tf = np.cos(n * TH)
            elif n == 0:
                continue
            else:
                tf = np.sin(n * TH)
            cols.append((tf * np.cos(m * PH)).ravel())
            keys.append(("c", n, m))
            if m > 0:
                cols.append((tf * np.sin(m * PH)).ravel())
                keys.append(("s", n, m))
    A = np.stack(cols, axis=1)
    coef = np.linalg.lstsq(A, vals.ravel(), rcond=None)[0]
    fc = np.zeros((N + 1, M + 1))
    fs = np.zeros((N + 1, M + 1))
    for (kind, n, m), c in zip(keys, coef):
        (fc if kind == "c" else fs)[n, m] = c
    # the basis has fewer functions than nodes: compare on its projection
    proj = (A @ coef).reshape(J, 2 * J)
    want = oracle.std_to_exp(fc, fs)
    got = oracle.dfs_analysis(proj)[0]
    assert np.abs(got - want).max() < 1e-12


def test_numpy_fft_of_the_glide_doubled_torus():
    """Library special case: extend the J x 2J samples to the 2J x 2J torus by
    the glide reflection f(phi, 2 pi - theta) = f(phi + pi, theta), take
    numpy's 2-D FFT, undo the half-cell theta offset; the band |n|, |m| <= J-1
    is the exp-form series (band-limited input)."""
    J = 12
    rng = np.random.default_rng(7)
    fc, fs = random_std(rng, J)
    vals = sample(oracle.std_to_exp(fc, fs), J)
    torus = np.empty((2 * J, 2 * J))
    torus[:J] = vals
    shift = np.roll(vals, -J, axis=1)            # phi + pi
    torus[J:] = shift[::-1]                      # theta_{2J-1-i} = 2 pi - theta_i
    G = np.fft.fft2(torus) / (2 * J) ** 2        # G[n, m] = mean f e^{-i(n theta' + m phi)}
    n = np.fft.fftfreq(2 * J, 1.0 / (2 * J)).astype(int)
    G *= np.exp(-1j * n * np.pi / (2 * J))[:, None]   # theta_i = theta'_i + pi / (2J)
    want = np.zeros((2 * J - 1, 2 * J - 1), dtype=complex)
    for a in range(-(J - 1), J):
        for b in range(-(J - 1), J):
            want[a + J - 1, b + J - 1] = G[a % (2 * J), b % (2 * J)]
    got = oracle.dfs_analysis(vals)[0]
    assert np.abs(got - want).max() < 1e-13


# ---- the rotation Q of section 3 ---------------------------------------------
def _frame(phi, th):
    r = np.array([np.sin(th) * np.cos(phi), np.sin(th) * np.sin(phi), np.cos(th)])
    east = np.array([-np.sin(phi), np.cos(phi), 0.0])
    north = np.array([-np.cos(th) * np.cos(phi), -np.cos(th) * np.sin(phi), np.sin(th)])
    return r, east, north


def test_rotation_is_parallel_transport_along_the_great_circle():
    """Geometry, not the formula: rotate the departure point's east and north
    unit vectors about r_D x r_A by the angle between r_D and r_A (Rodrigues)
    and read them in the arrival point's frame."""
    rng = np.random.default_rng(3)
    for _ in range(50):
        pa, pd = rng.uniform(-7, 7, 2)
        ta, td = rng.uniform(0.05, np.pi - 0.05, 2)
        rA, eA, nA = _frame(pa, ta)
        rD, eD, nD = _frame(pd, td)
        axis = np.cross(rD, rA)
        ang = np.arctan2(np.linalg.norm(axis), rD @ rA)
        k = axis / np.linalg.norm(axis)

        def R(x):
            return x * np.cos(ang) + np.cross(k, x) * np.sin(ang) + k * (k @ x) * (1 - np.cos(ang))

        Q = np.array([[eA @ R(eD), eA @ R(nD)], [nA @ R(eD), nA @ R(nD)]])
        p, q = oracle.rotation_pq(pa, ta, pd, td)
        assert np.allclose(Q, [[p, q], [-q, p]], atol=1e-12)


def test_rotation_special_cases():
    rng = np.random.default_rng(4)
    pa, ta = rng.uniform(0, 2 * np.pi, 100), rng.uniform(0.1, 3.0, 100)
    pd, td = pa + rng.uniform(-0.3, 0.3, 100), ta + rng.uniform(-0.3, 0.3, 100)
    p, q = oracle.rotation_pq(pa, ta, pd, td)
    assert np.allclose(p * p + q * q, 1.0, atol=1e-13)      # a rotation
    p0, q0 = oracle.rotation_pq(pa, ta, pa, ta)                # no displacement
    assert np.allclose(p0, 1.0) and np.allclose(q0, 0.0)
    pm, qm = oracle.rotation_pq(pa, ta, pa, td)                # along a meridian
    assert np.allclose(pm, 1.0) and np.allclose(qm, 0.0, atol=1e-15)
    u, v = rng.standard_normal(100), rng.standard_normal(100)
    ur, vr = oracle.rotate_uv(u, v, pa, ta, pd, td)
    assert np.allclose(ur * ur + vr * vr, u * u + v * v)         # lengths kept
