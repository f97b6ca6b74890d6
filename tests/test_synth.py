"""Properties of the seeded input generators (no interpolation arithmetic here)."""
import numpy as np

import synth


def test_grid0_counts_and_range():
    for J in (4, 32, 256):
        phi, theta = synth.grid0_points(J)
        assert phi.size == 2 * J * J
        assert np.all((theta > 0) & (theta < np.pi))
        assert np.all((phi >= 0) & (phi < 2 * np.pi))


def test_coefficients_have_glide_and_hermitian_symmetry():
    rng = np.random.default_rng(0)
    K = 15
    F = synth.dfs_field_coeffs(rng, K, K, synth.envelope_gauss(K, K))
    m = synth.mode_axis(K)
    sign = np.where(m % 2 == 0, 1.0, -1.0)[None, :]
    np.testing.assert_allclose(F[::-1, :], sign * F, atol=1e-15)      # F[-n,m] = (-1)^m F[n,m]
    np.testing.assert_allclose(F[::-1, ::-1], np.conj(F), atol=1e-15)  # F[-n,-m] = conj F[n,m]


def test_small_jitter_workload_is_reproducible():
    a = synth.workload_small_jitter()
    b = synth.workload_small_jitter()
    np.testing.assert_array_equal(a.coeffs, b.coeffs)
    np.testing.assert_array_equal(a.phi, b.phi)
    assert a.coeffs.shape == (1, 63, 63) and a.n_pts == 2048
    # offsets of at most 0.05 rad from the nodes, modulo 2 pi
    phi0, theta0 = synth.grid0_points(32)
    d = np.angle(np.exp(1j * (a.theta - theta0)))
    assert np.max(np.abs(d)) <= 0.05 + 1e-12
    # some points cross a pole onto the far half of the torus
    assert np.any(a.theta > np.pi) or np.any(a.theta < 0.05)


def test_sbr_departure_rotates_back_to_arrival():
    J = 16
    phi_a, theta_a = synth.grid0_points(J)
    alpha, dt = np.pi / 4, 1200.0
    u0 = 2 * np.pi * synth.EARTH_RADIUS / (12 * synth.DAY)
    phi_d, theta_d = synth.sbr_departures(phi_a, theta_a, alpha, u0, dt)
    xd = synth.sph_to_cart(phi_d, theta_d)
    xa = synth.rotate(xd, synth.sbr_axis(alpha), (u0 / synth.EARTH_RADIUS) * dt)
    np.testing.assert_allclose(xa, synth.sph_to_cart(phi_a, theta_a), atol=1e-14)
    # one 12-day period is a full turn
    assert abs((u0 / synth.EARTH_RADIUS) * 12 * synth.DAY - 2 * np.pi) < 1e-12


def test_stream_function_wind_courant_and_divergence():
    J = 32
    phi, theta = synth.grid0_points(J)
    w = synth.StreamFunctionWind(np.random.default_rng(14))
    w.normalize_courant(phi, theta, 8.0, J)
    vt, vp = w.tangent_wind(phi, theta)
    np.testing.assert_allclose(np.max(np.hypot(vt, vp)), 8.0 * np.pi / J, rtol=1e-12)
    # surface divergence of r x grad(psi) vanishes: check by central differences
    rng = np.random.default_rng(1)
    th = rng.uniform(0.3, 2.8, 50)
    ph = rng.uniform(0, 2 * np.pi, 50)
    h = 1e-5

    def div(th, ph):
        vt_p, _ = w.tangent_wind(ph, th + h)
        vt_m, _ = w.tangent_wind(ph, th - h)
        _, vp_p = w.tangent_wind(ph + h, th)
        _, vp_m = w.tangent_wind(ph - h, th)
        d_th = (np.sin(th + h) * vt_p - np.sin(th - h) * vt_m) / (2 * h)
        d_ph = (vp_p - vp_m) / (2 * h)
        return (d_th + d_ph) / np.sin(th)

    scale = 8.0 * np.pi / J
    assert np.max(np.abs(div(th, ph))) < 1e-6 * scale
    # departure points stay on the sphere and move by about the wind displacement
    pd, td = w.departures(phi, theta)
    disp = np.arccos(np.clip(np.sum(synth.sph_to_cart(pd, td) * synth.sph_to_cart(phi, theta), -1), -1, 1))
    assert disp.max() <= 8.0 * np.pi / J * 1.05
    assert disp.max() >= 8.0 * np.pi / J * 0.9


def test_sample_indices_are_seeded_and_unique():
    a = synth.sample_indices(100000, 1000)
    b = synth.sample_indices(100000, 1000)
    np.testing.assert_array_equal(a, b)
    assert np.unique(a).size == 1000
