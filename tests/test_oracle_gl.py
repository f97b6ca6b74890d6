"""Pins of the oracle's Gauss-Legendre DFS analysis (section 2, eq. GLGrid;
section 5's interpolation for the SHT model).

Routes other than the oracle's own: Legendre polynomials evaluated by scipy
at the nodes, the direct sum of the exp-form series at the grid nodes
(interpolation), exact recovery of band-limited series, the symmetries of a
real DFS field, and a brute-force least-squares fit of the 2-D basis.
"""
import numpy as np
import pytest
from scipy.special import eval_legendre

import oracle


@pytest.mark.parametrize("J", [4, 16, 64, 256])
def test_nodes_are_legendre_roots(J):
    th, ph = oracle.gl_nodes(J)
    assert th.shape == (J,) and ph.shape == (2 * J,)
    assert np.all(np.diff(th) > 0) and 0 < th[0] and th[-1] < np.pi
    z = np.cos(th)
    dP = J * (z * eval_legendre(J, z) - eval_legendre(J - 1, z)) / (z * z - 1.0)
    assert np.abs(eval_legendre(J, z) / dP).max() < 1e-15          # the Newton step at each root
    assert np.allclose(th, np.pi - th[::-1], atol=1e-14)          # symmetric about the equator


def test_nodes_against_40_digit_newton():
    """Nodes near the poles, where an FP64 arccos of the Legendre root is
    off by ~1e-14: Newton in theta at 40 digits (mpmath)."""
    import mpmath as mpm
    mpm.mp.dps = 40
    J = 1024
    th, _ = oracle.gl_nodes(J)
    for i in (0, 1, 5, 511, 1018, 1023):
        t = mpm.mpf(th[i])
        for _ in range(4):
            h = mpm.mpf("1e-28")
            f = mpm.legendre(J, mpm.cos(t))
            df = (mpm.legendre(J, mpm.cos(t + h)) - mpm.legendre(J, mpm.cos(t - h))) / (2 * h)
            t -= f / df
        assert abs(float(th[i] - t)) <= 2.5e-16, i


def exp_series_values(coeffs, J):
    th, ph = oracle.gl_nodes(J)
    T, P = np.meshgrid(th, ph, indexing="ij")
    v = oracle.dfs_eval(coeffs, P.ravel(), T.ravel())
    return v.reshape(coeffs.shape[0], J, 2 * J)


@pytest.mark.parametrize("J", [3, 8, 16, 40])
def test_interpolates_the_samples(J):
    rng = np.random.default_rng(J)
    vals = rng.standard_normal((2, J, 2 * J))
    e = oracle.gl_analysis(vals)
    back = exp_series_values(e, J)
    # the phi Nyquist mode is dropped: compare with the samples projected off it
    spec = np.fft.rfft(vals, axis=2)
    spec[..., J] = 0.0
    want = np.fft.irfft(spec, n=2 * J, axis=2)
    assert np.abs(back.imag).max() < 1e-12
    assert np.abs(back.real - want).max() < 1e-12


def random_band_limited(rng, J):
    """Exp-form coefficients of a real DFS field in the analysis' basis
    (even m: |n| <= J - 1; odd m: |n| <= J; |m| <= J - 1): random complex
    values projected onto the glide symmetry e(-n, m) = (-1)^m e(n, m) and
    the Hermitian symmetry e(-n, -m) = conj e(n, m)."""
    e = rng.standard_normal((2 * J + 1, 2 * J - 1)) + 1j * rng.standard_normal((2 * J + 1, 2 * J - 1))
    sign = np.where(np.arange(-(J - 1), J) % 2 == 0, 1.0, -1.0)[None, :]
    e = 0.5 * (e + sign * e[::-1, :])
    e = 0.5 * (e + np.conj(e[::-1, ::-1]))
    even = sign[0] > 0
    e[0, even] = 0.0
    e[2 * J, even] = 0.0
    return e


@pytest.mark.parametrize("J", [4, 12, 32])
def test_recovers_band_limited_series(J):
    rng = np.random.default_rng(100 + J)
    e = random_band_limited(rng, J)
    vals = exp_series_values(e[None], J)
    assert np.abs(vals.imag).max() < 1e-10                        # a real field
    got = oracle.gl_analysis(vals.real)[0]
    assert np.abs(got - e).max() < 1e-12 * max(1.0, np.abs(e).max())


def test_real_field_symmetries():
    J = 20
    rng = np.random.default_rng(5)
    e = oracle.gl_analysis(rng.standard_normal((J, 2 * J)))[0]
    n = np.arange(-J, J + 1)[:, None]
    m = np.arange(-(J - 1), J)[None, :]
    # Hermitian: e(-n, -m) = conj e(n, m); glide: e(-n, m) = (-1)^m e(n, m)
    assert np.abs(e[::-1, ::-1] - np.conj(e)).max() < 1e-13
    assert np.abs(e[::-1, :] - np.where(m % 2 == 0, 1, -1) * e).max() < 1e-13
    assert not e[J, (m[0] % 2 != 0)].any()                      # odd m: no n = 0 term
    assert not e[[0, 2 * J]][:, m[0] % 2 == 0].any()            # even m: no |n| = J term
    del n


def test_least_squares_fit_of_the_basis():
    """Brute force at J = 4: fit the 2-D basis (cos or sin in theta by the
    parity of m, e^{i m phi} for |m| <= J - 1) to the 4 x 8 samples by least
    squares; the per-m latitude systems are square, so the fit is the
    analysis."""
    J = 4
    rng = np.random.default_rng(2)
    vals = rng.standard_normal((J, 2 * J))
    th, ph = oracle.gl_nodes(J)
    T, P = np.meshgrid(th, ph, indexing="ij")
    cols, keys = [], []
    for m in range(-(J - 1), J):
        for n in (range(0, J) if m % 2 == 0 else range(1, J + 1)):
            tf = np.cos(n * T) if m % 2 == 0 else np.sin(n * T)
            cols.append((tf * np.exp(1j * m * P)).ravel())
            keys.append((m, n))
    A = np.stack(cols, axis=1)
    coef = np.linalg.lstsq(A, vals.ravel().astype(complex), rcond=None)[0]
    want = np.zeros((2 * J + 1, 2 * J - 1), dtype=complex)
    for (m, n), c in zip(keys, coef):
        if m % 2 == 0:
            if n == 0:
                want[J, m + J - 1] += c
            else:
                want[J + n, m + J - 1] += c / 2
                want[J - n, m + J - 1] += c / 2
        else:
            want[J + n, m + J - 1] += c / 2j
            want[J - n, m + J - 1] -= c / 2j
    got = oracle.gl_analysis(vals)[0]
    assert np.abs(got - want).max() < 1e-12


PLANTS = [
    ("th = np.sort(np.arccos(z)).astype(np.longdouble)", "th = np.arccos(z).astype(np.longdouble)"),  # z order
    ("g = np.fft.fft(values, axis=2) / (2 * J)", "g = np.fft.fft(values, axis=2) / J"),
    ("out[:, (J + nn)[:, None], cols[None, :]] = -0.5j * b", "out[:, (J + nn)[:, None], cols[None, :]] = 0.5j * b"),
    ("np.sin(np.outer(th, n + 1))", "np.sin(np.outer(th, n))"),
    ("lu = (lu_factor(Ce), lu_factor(Co))", "lu = (lu_factor(Co), lu_factor(Ce))"),          # parities swapped
]


def _gl_pins_hold(o):
    J = 8
    rng = np.random.default_rng(31)
    vals = rng.standard_normal((1, J, 2 * J))
    th, ph = oracle.gl_nodes(J)           # the true grid
    T, P = np.meshgrid(th, ph, indexing="ij")
    try:
        e = o["gl_analysis"](vals)
    except Exception:
        return False
    back = oracle.dfs_eval(e, P.ravel(), T.ravel()).reshape(1, J, 2 * J)
    spec = np.fft.rfft(vals, axis=2)
    spec[..., J] = 0.0
    if np.abs(back - np.fft.irfft(spec, n=2 * J, axis=2)).max() > 1e-12:
        return False
    # the glide symmetry of a real DFS field (the interpolant in the wrong
    # parity basis still meets the samples, but not this)
    m = np.arange(-(J - 1), J)[None, :]
    return np.abs(e[0, ::-1, :] - np.where(m % 2 == 0, 1, -1) * e[0]).max() < 1e-12


def test_planted_mistakes_are_caught():
    import oracle.gl as gl
    src = open(gl.__file__).read()
    clean = {}
    exec(compile(src, "gl_clean", "exec"), clean)
    assert _gl_pins_hold(clean)
    import warnings
    for a, b in PLANTS:
        assert a in src, a
        ns = {}
        exec(compile(src.replace(a, b, 1), "gl_planted", "exec"), ns)
        with warnings.catch_warnings():
            warnings.simplefilter("ignore")         # a planted basis can be singular
            assert not _gl_pins_hold(ns), f"planted mistake not caught: {b}"
