"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each pin is a function of an evaluator with the oracle's signature, so the
same battery also runs against deliberately broken builds of the oracle
source (test_planted_mistakes_are_caught) to show it can fail.
"""
import os
import re
import subprocess
import tempfile

import mpmath
import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# --------------------------------------------------------------------------
# The pins
# --------------------------------------------------------------------------
def pin_single_mode(ev):
    """One nonzero coefficient at (n0, m0) gives e^{i(m0 phi + n0 theta)} (eq. std_dfs_exp)."""
    rng = np.random.default_rng(101)
    Kt, Kp = 9, 13
    phi = rng.uniform(-1.0, 7.5, 24)
    theta = rng.uniform(-1.0, 7.5, 24)
    worst = 0.0
    for (n0, m0) in [(0, 0), (3, -5), (-4, 6), (2, 1), (-1, -6), (4, 0), (0, -3)]:
        F = np.zeros((Kt, Kp), complex)
        F[n0 + Kt // 2, m0 + Kp // 2] = 1.0
        got = ev(F, phi, theta)[0]
        exact = np.array([complex(mpmath.expj(mpmath.mpf(m0) * mpmath.mpf(p)
                                              + mpmath.mpf(n0) * mpmath.mpf(t)))
                          for p, t in zip(phi, theta)])
        worst = max(worst, float(np.max(np.abs(got - exact))))
    return worst < 1e-13, worst


def torus_nodes(J):
    """The 2J x 2J doubled Grid [0] torus: theta_i = (i + 1/2) pi / J, phi_k = pi k / J."""
    th = (np.arange(2 * J) + 0.5) * np.pi / J
    ph = np.arange(2 * J) * np.pi / J
    T, P = np.meshgrid(th, ph, indexing="ij")
    return P.ravel(), T.ravel()


def pin_torus_nodes(ev):
    """At the torus nodes the series is an inverse DFT: numpy.fft reproduces it.

    f(phi_k, theta_i) = sum_n e^{i n pi / 2J} e^{2 pi i n i / 2J} sum_m F[n,m] e^{2 pi i m k / 2J},
    i.e. ifft2 of F (times the half-cell phase in theta) scaled by (2J)^2.
    """
    J = 8
    K = 2 * J - 1
    rng = np.random.default_rng(7)
    F = synth.random_complex(rng, (K, K))
    n = synth.mode_axis(K)
    G = np.zeros((2 * J, 2 * J), complex)
    G[np.ix_(n % (2 * J), n % (2 * J))] = F * np.exp(1j * n * np.pi / (2 * J))[:, None]
    v = np.fft.ifft2(G) * (2 * J) ** 2
    phi, theta = torus_nodes(J)
    got = ev(F, phi, theta)[0].reshape(2 * J, 2 * J)
    err = rel_l2(got, v)
    # The other direction: values on the nodes -> coefficients by fft2 -> back.
    F2 = np.fft.fft2(v) / (2 * J) ** 2
    F2 = F2[np.ix_(n % (2 * J), n % (2 * J))] * np.exp(-1j * n * np.pi / (2 * J))[:, None]
    err2 = rel_l2(F2, F)
    return err < 1e-14 and err2 < 1e-14, max(err, err2)


def pin_bruteforce(ev):
    """40-digit brute force of the double sum on tiny mode counts and random points."""
    rng = np.random.default_rng(11)
    mpmath.mp.dps = 40
    worst = 0.0
    for (Kt, Kp) in [(7, 9), (5, 3), (1, 4), (6, 5)]:
        F = synth.random_complex(rng, (Kt, Kp))
        phi = rng.uniform(-3, 10, 16)
        theta = rng.uniform(-3, 10, 16)
        got = ev(F, phi, theta)[0]
        for j in range(16):
            s = mpmath.mpc(0)
            for a in range(Kt):
                for b in range(Kp):
                    n, m = a - Kt // 2, b - Kp // 2
                    s += mpmath.mpc(F[a, b].real, F[a, b].imag) * mpmath.expj(
                        m * mpmath.mpf(phi[j]) + n * mpmath.mpf(theta[j]))
            scale = float(np.abs(F).sum())
            worst = max(worst, abs(complex(s) - got[j]) / scale)
    mpmath.mp.dps = 15
    return worst < 1e-15, worst


def std_dfs_series(fc, fs, phi, theta):
    """The standard DFS series of section 4 (eq. std_dfs), evaluated term by term."""
    N, M = fc.shape[0] - 1, fc.shape[1] - 1
    out = np.zeros_like(phi)
    for m in range(M + 1):
        for n in range(N + 1):
            if m % 2 == 0:
                tf = np.cos(n * theta)
            else:
                if n == 0:
                    continue
                tf = np.sin(n * theta)
            out += fc[n, m] * tf * np.cos(m * phi)
            if m >= 1:
                out += fs[n, m] * tf * np.sin(m * phi)
    return out


def pin_cos_sin_convention(ev):
    """Exp-form coefficients from eq. dfs_fourier_coeffs reproduce the real cos/sin series."""
    import oracle
    rng = np.random.default_rng(3)
    N, M = 6, 7
    fc = rng.standard_normal((N + 1, M + 1))
    fs = rng.standard_normal((N + 1, M + 1))
    fs[:, 0] = 0.0
    phi = rng.uniform(0, 2 * np.pi, 40)
    theta = rng.uniform(-0.3, np.pi + 0.3, 40)
    want = std_dfs_series(fc, fs, phi, theta)
    got = ev(oracle.std_to_exp(fc, fs), phi, theta)[0]
    err = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
    return err < 1e-13, err


def pin_glide_and_periodicity(ev):
    """DFS parity: f(phi + pi, -theta) = f(phi, theta); 2 pi periodic in both."""
    rng = np.random.default_rng(5)
    K = 21
    F = synth.dfs_field_coeffs(rng, K, K, synth.envelope_algebraic(K, K, 1.0))
    phi = rng.uniform(0, 2 * np.pi, 64)
    theta = rng.uniform(0, np.pi, 64)
    base = ev(F, phi, theta)[0]
    e1 = rel_l2(ev(F, phi + np.pi, -theta)[0], base)
    e2 = rel_l2(ev(F, phi + 2 * np.pi, theta)[0], base)
    e3 = rel_l2(ev(F, phi, theta - 2 * np.pi)[0], base)
    err = max(e1, e2, e3)
    return err < 1e-14, err


def pin_real_field(ev):
    """Hermitian coefficients give a real value at any point."""
    rng = np.random.default_rng(9)
    K = 31
    F = synth.dfs_field_coeffs(rng, K, K, synth.envelope_gauss(K, K))
    phi = rng.uniform(0, 2 * np.pi, 64)
    theta = rng.uniform(0, np.pi, 64)
    v = ev(F, phi, theta)[0]
    err = float(np.max(np.abs(v.imag)) / np.max(np.abs(v.real)))
    return err < 1e-14, err


PINS = [pin_single_mode, pin_torus_nodes, pin_bruteforce, pin_cos_sin_convention,
        pin_glide_and_periodicity, pin_real_field]


# --------------------------------------------------------------------------
# Tests
# --------------------------------------------------------------------------
@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_oracle_pin(oracle_mod, pin):
    ok, err = pin(oracle_mod.dfs_eval)
    assert ok, f"{pin.__name__}: error {err:.3e}"


def test_multifield_is_per_field(oracle_mod):
    rng = np.random.default_rng(12)
    F = synth.random_complex(rng, (3, 11, 9))
    phi, theta = rng.uniform(0, 7, 30), rng.uniform(0, 7, 30)
    allf = oracle_mod.dfs_eval(F, phi, theta)
    for f in range(3):
        np.testing.assert_array_equal(allf[f], oracle_mod.dfs_eval(F[f], phi, theta)[0])


def test_long_double_certifies_fp64_at_largest_size(oracle_mod):
    """At 2047 x 2047 modes the FP64 sum agrees with an extended-precision sum."""
    rng = np.random.default_rng(15)
    K = 2047
    F = synth.random_complex(rng, (K, K)) * synth.envelope_algebraic(K, K, 1.5)
    phi = rng.uniform(0, 2 * np.pi, 3)
    theta = rng.uniform(-0.05, np.pi + 0.05, 3)
    a = oracle_mod.dfs_eval(F, phi, theta)
    b = oracle_mod.dfs_eval_ld(F, phi, theta)
    assert rel_l2(a, b) < 1e-14


def test_grid0_nodes_match_printed_definition():
    """Generator nodes equal the Grid [0] formula (golden fixture, section 3)."""
    rows = [l.split() for l in open(os.path.join(ROOT, "tests", "golden", "grid0_J4.txt"))
            if not l.startswith("#")]
    th = np.array([float(v) for k, i, v in rows if k == "theta"])
    ph = np.array([float(v) for k, i, v in rows if k == "phi"])
    gth, gph = synth.grid0_axes(4)
    np.testing.assert_allclose(gth, th, rtol=0, atol=1e-15)
    np.testing.assert_allclose(gph, ph, rtol=0, atol=1e-15)


# Planted mistakes: each mutation is a plausible slip in the oracle source.
MUTATIONS = {
    "conjugate_phi": (r"ep\[2 \* b \+ 1\] = sin\(arg\);", "ep[2 * b + 1] = -sin(arg);"),
    "conjugate_theta": (r"et\[2 \* a \+ 1\] = sin\(arg\);", "et[2 * a + 1] = -sin(arg);"),
    "swap_coordinates": (r"const double ph = phi\[j\], th = theta\[j\];",
                         "const double ph = theta[j], th = phi[j];"),
    "centre_off_by_one": (r"const int64_t n0 = K_theta / 2, m0 = K_phi / 2;",
                          "const int64_t n0 = K_theta / 2, m0 = K_phi / 2 + 1;"),
    "dropped_imag_term": (r"rr \+= fr \* ep\[2 \* b\] - fi \* ep\[2 \* b \+ 1\];",
                          "rr += fr * ep[2 * b];"),
    "wrong_sign_combine": (r"cr \+= rr \* et\[2 \* a\] - ri \* et\[2 \* a \+ 1\];",
                           "cr += rr * et[2 * a] + ri * et[2 * a + 1];"),
    "dropped_last_mode": (r"for \(int64_t b = 0; b < K_phi; \+\+b\) \{\n\s+const double fr",
                          "for (int64_t b = 0; b < K_phi - 1; ++b) {\n const double fr"),
    "transposed_coeffs": (r"const double \*row = Ff \+ \(size_t\)2 \* a \* K_phi;",
                          "const double *row = Ff + (size_t)2 * a;"),
}


def _build_mutant(src, pattern, repl, out_path):
    new, count = re.subn(pattern, repl, src, count=1)
    assert count == 1, f"mutation pattern not found: {pattern}"
    if "transposed_coeffs" in out_path:
        new = new.replace("const double fr = row[2 * b], fi = row[2 * b + 1];",
                          "const double fr = row[2 * b * K_theta], fi = row[2 * b * K_theta + 1];", 1)
    c_path = out_path[:-3] + ".c"
    with open(c_path, "w") as fh:
        fh.write(new)
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", c_path, "-o", out_path, "-lm"],
                   check=True)


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistakes_are_caught(name):
    """Every planted slip makes at least one pin fail (the pins can fail)."""
    import oracle
    src = open(os.path.join(ROOT, "oracle", "dfs_direct.c")).read()
    pattern, repl = MUTATIONS[name]
    with tempfile.TemporaryDirectory() as d:
        so = os.path.join(d, f"mut_{name}.so")
        _build_mutant(src, pattern, repl, so)
        ev = oracle.load_variant(so)
        results = {p.__name__: p(ev)[0] for p in PINS if p is not pin_bruteforce}
    assert not all(results.values()), f"mutation {name} passed every pin: {results}"
