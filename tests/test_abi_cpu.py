"""C-ABI checks that need no GPU: exports, host-side kernel parameters,
deconvolution factors, and argument validation that fails before any HIP call."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nufft2.h")


@pytest.fixture(scope="module")
def nf():
    from paper_2605_01313_amd import nufft2
    return nufft2


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nufft2_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol(nf):
    lib = ctypes.CDLL(nf.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 11
    for name in names:
        assert hasattr(lib, name), f"{name} declared in nufft2.h but not exported"
    assert set(names) == set(nf.EXPORTED)


def test_only_abi_symbols_are_exported(nf):
    out = os.popen(f"nm -D --defined-only {nf.LIB_PATH}").read().split("\n")
    funcs = [l.split()[-1] for l in out if " T " in l]
    stray = [f for f in funcs if not f.startswith("nufft2_") and not f.startswith("_")]
    assert not stray, stray


def test_kernel_width_rule(nf):
    assert nf.nufft2_kernel_params(nf.NUFFT2_FP64, 1e-12)[:2] == (0, 13)
    assert nf.nufft2_kernel_params(nf.NUFFT2_FP32, 1e-6)[:2] == (0, 7)
    assert nf.nufft2_kernel_params(nf.NUFFT2_FP64, 1e-14)[:2] == (0, 15)
    st, w, beta = nf.nufft2_kernel_params(nf.NUFFT2_FP64, 1e-12)
    assert abs(beta - 2.30 * 13) < 1e-12
    assert nf.nufft2_kernel_params(nf.NUFFT2_FP32, 1e-8)[0] == nf.NUFFT2_ERR_EPS_RANGE
    assert nf.nufft2_kernel_params(nf.NUFFT2_FP64, 1e-16)[0] == nf.NUFFT2_ERR_EPS_RANGE
    assert nf.nufft2_kernel_params(nf.NUFFT2_FP64, -1.0)[0] == nf.NUFFT2_ERR_ARG
    assert nf.nufft2_kernel_params(nf.NUFFT2_FP64, float("nan"))[0] == nf.NUFFT2_ERR_ARG
    assert nf.nufft2_kernel_params(7, 1e-6)[0] == nf.NUFFT2_ERR_ARG


def test_deconvolution_factors_against_adaptive_quadrature(nf):
    """corr(k) = 2 / (w Phi(pi w k / nf)); Phi checked with scipy's adaptive quad."""
    from scipy.integrate import quad
    for (K, nfine, w) in [(63, 128, 13), (511, 1024, 7), (31, 64, 7)]:
        beta = 2.30 * w
        st, c = nf.nufft2_kernel_correction(K, nfine, w, beta)
        assert st == 0
        for a in [0, 1, K // 4, K // 2, K - 1]:
            k = a - K // 2
            xi = np.pi * w * k / nfine
            phi_hat, _ = quad(lambda z: np.exp(beta * (np.sqrt(1 - z * z) - 1)) * np.cos(xi * z),
                              -1, 1, epsabs=0, epsrel=2e-14, limit=400)
            assert abs(c[a] - 2.0 / (w * phi_hat)) <= 1e-12 * abs(c[a])
        assert np.allclose(c, c[::-1], rtol=1e-15, atol=0)       # even in k for odd K


def _emulate_method(corr_t, corr_p, coeffs, phi, theta, w, beta, nft, nfp):
    """numpy re-statement of the three stages, for checking the host parameters."""
    Kt, Kp = coeffs.shape
    n = np.arange(Kt) - Kt // 2
    m = np.arange(Kp) - Kp // 2
    G = np.zeros((nft, nfp), complex)
    G[np.ix_(n % nft, m % nfp)] = coeffs * corr_t[:, None] * corr_p[None, :]
    b = np.fft.ifft2(G) * nft * nfp
    out = np.zeros(phi.size, complex)
    for j in range(phi.size):
        tt = np.mod(theta[j], 2 * np.pi) * nft / (2 * np.pi)
        tp = np.mod(phi[j], 2 * np.pi) * nfp / (2 * np.pi)
        it, ip = int(np.ceil(tt - w / 2)), int(np.ceil(tp - w / 2))
        a = np.arange(w)
        zt = (it + a - tt) / (w / 2)
        zp = (ip + a - tp) / (w / 2)
        kt = np.exp(beta * (np.sqrt(np.maximum(1 - zt * zt, 0)) - 1))
        kp = np.exp(beta * (np.sqrt(np.maximum(1 - zp * zp, 0)) - 1))
        out[j] = kt @ b[np.ix_((it + a) % nft, (ip + a) % nfp)] @ kp
    return out


@pytest.mark.parametrize("eps", [1e-6, 1e-12])
def test_host_parameters_reach_tolerance(nf, oracle_mod, eps):
    """With the library's w, beta and factors the method reaches eps (numpy stages)."""
    import synth
    J = 16
    K = 2 * J - 1
    rng = np.random.default_rng(4)
    F = synth.dfs_field_coeffs(rng, K, K, synth.envelope_algebraic(K, K, 1.5))
    phi = rng.uniform(0, 2 * np.pi, 300)
    theta = rng.uniform(-0.2, np.pi + 0.2, 300)
    st, w, beta = nf.nufft2_kernel_params(nf.NUFFT2_FP64, eps)
    nfine = 4 * J
    _, c = nf.nufft2_kernel_correction(K, nfine, w, beta)
    got = _emulate_method(c, c, F, phi, theta, w, beta, nfine, nfine)
    ref = oracle_mod.dfs_eval(F, phi, theta)[0]
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < eps


def test_plan_argument_errors_before_device_work(nf):
    P = nf.nufft2_plan
    assert P(3, 63, 63, 1, 1e-12)[0] == nf.NUFFT2_ERR_ARG          # bad precision
    assert P(nf.NUFFT2_FP64, 0, 63, 1, 1e-12)[0] == nf.NUFFT2_ERR_ARG
    assert P(nf.NUFFT2_FP64, 63, -1, 1, 1e-12)[0] == nf.NUFFT2_ERR_ARG
    assert P(nf.NUFFT2_FP64, 63, 63, 0, 1e-12)[0] == nf.NUFFT2_ERR_ARG
    assert P(nf.NUFFT2_FP64, 4097, 63, 1, 1e-12)[0] == nf.NUFFT2_ERR_ARG  # grid above 4096
    assert P(nf.NUFFT2_FP32, 63, 63, 1, 1e-9)[0] == nf.NUFFT2_ERR_EPS_RANGE
    assert P(nf.NUFFT2_FP64, 63, 63, 1, 1e-17)[0] == nf.NUFFT2_ERR_EPS_RANGE
    bad_tile = nf.nufft2_opts(0, 0.0, 24, 32, 0, 0)
    assert P(nf.NUFFT2_FP64, 63, 63, 1, 1e-12, bad_tile)[0] == nf.NUFFT2_ERR_ARG
    big_tile = nf.nufft2_opts(16, 0.0, 128, 128, 0, 0)              # LDS patch too large
    assert P(nf.NUFFT2_FP64, 511, 511, 1, 1e-12, big_tile)[0] == nf.NUFFT2_ERR_ARG
    bad_flag = nf.nufft2_opts(0, 0.0, 0, 0, 0, 2)
    assert P(nf.NUFFT2_FP64, 63, 63, 1, 1e-12, bad_flag)[0] == nf.NUFFT2_ERR_ARG
    bad_layout = nf.nufft2_opts(0, 0.0, 0, 0, 0, 0, 2, 0)
    assert P(nf.NUFFT2_FP64, 63, 63, 1, 1e-12, bad_layout)[0] == nf.NUFFT2_ERR_ARG
    bad_reserved = nf.nufft2_opts(0, 0.0, 0, 0, 0, 0, 0, 1)
    assert P(nf.NUFFT2_FP64, 63, 63, 1, 1e-12, bad_reserved)[0] == nf.NUFFT2_ERR_ARG
    # real-field plans need mode ranges symmetric about zero (odd counts)
    herm = nf.nufft2_opts(0, 0.0, 0, 0, 0, 1)
    assert P(nf.NUFFT2_FP64, 64, 63, 1, 1e-12, herm)[0] == nf.NUFFT2_ERR_ARG
    assert P(nf.NUFFT2_FP32, 63, 62, 1, 1e-6, herm)[0] == nf.NUFFT2_ERR_ARG
    null = ctypes.c_void_p()
    assert nf.nufft2_setpts(null, 10, 0, 0) == nf.NUFFT2_ERR_ARG
    assert nf.nufft2_exec(null, 0, 0) == nf.NUFFT2_ERR_ARG
    assert nf.nufft2_check(null) == nf.NUFFT2_ERR_ARG
    assert nf.nufft2_destroy(null) == nf.NUFFT2_OK
    assert nf.nufft2_get_info(null)[0] == nf.NUFFT2_ERR_ARG
    assert nf.nufft2_strerror(nf.NUFFT2_ERR_NO_POINTS) == "exec before setpts"
    # groups: empty or null member lists, null group handles
    assert nf.nufft2_group_create([])[0] == nf.NUFFT2_ERR_ARG
    assert nf.nufft2_group_create([null])[0] == nf.NUFFT2_ERR_ARG
    assert nf.nufft2_group_setpts(null, [1], [0], [0]) == nf.NUFFT2_ERR_ARG
    assert nf.nufft2_group_exec(null, [0], [0]) == nf.NUFFT2_ERR_ARG
    assert nf.nufft2_group_get_info(null)[0] == nf.NUFFT2_ERR_ARG
    assert nf.nufft2_group_destroy(null) == nf.NUFFT2_OK


def test_binding_has_no_fallback_path():
    """The product package never reaches the oracle or a CPU implementation."""
    pkg = os.path.join(ROOT, "paper_2605_01313_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "numpy.fft" not in text and "np.fft" not in text, f


@pytest.mark.parametrize("J", [1, 2, 7, 16, 256, 1024])
def test_gl_nodes_are_the_gauss_legendre_colatitudes(nf, oracle_mod, J):
    """Host helper, no device work: the library's Newton iteration (long
    double) against numpy's Gauss-Legendre nodes used by the oracle."""
    st, th = nf.nufft2_gl_nodes(J)
    assert st == nf.NUFFT2_OK
    want, _ = oracle_mod.gl_nodes(J)
    assert np.abs(th - want).max() < 4e-16


def test_gl_and_pr_argument_errors_before_device_work(nf):
    assert nf.nufft2_gl_nodes(0)[0] == nf.NUFFT2_ERR_ARG
    assert nf.nufft2_gl_plan(1, 24, 1)[0] == nf.NUFFT2_ERR_ARG       # not a power of two
    assert nf.nufft2_gl_plan(1, 8, 1)[0] == nf.NUFFT2_ERR_ARG        # below 16
    assert nf.nufft2_gl_plan(1, 2048, 1)[0] == nf.NUFFT2_ERR_ARG     # above 1024
    assert nf.nufft2_gl_plan(2, 64, 0)[0] == nf.NUFFT2_ERR_ARG       # no fields
    assert nf.nufft2_gl_exec(None, 0, 0) == nf.NUFFT2_ERR_ARG
    assert nf.nufft2_gl_destroy(None) == nf.NUFFT2_OK
    assert nf.nufft2_pr_plan(1, 4, 10, 1)[0] == nf.NUFFT2_ERR_ARG
    assert nf.nufft2_pr_destroy(None) == nf.NUFFT2_OK
