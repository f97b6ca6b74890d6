"""Real-field (Hermitian) plans against the FP64 oracle.

The coefficients of a real DFS field satisfy c[-n][-m] = conj(c[n][m])
(section 5, eq. dfs_fourier_coeffs and the symmetries after it); a plan
created with hermitian=True reads the m >= 0 half only, runs the theta pass
on those columns, a complex-to-real phi pass and the gather on a real fine
grid, and returns real values.  For such coefficients the exact result is
the real series, i.e. the real part of the oracle's direct sum.  For other
coefficients the plan's definition (include/nufft2.h) is the real part of
the series of the m >= 0 half with the m > 0 terms doubled, which the
oracle evaluates directly on those coefficients.

Tolerances as in the complex parity tests: eps = 1e-12 (FP64) and 1e-6
(FP32) on the workloads' decaying spectra; 3 eps on flat (white) spectra,
where the width rule realises about 2 eps.
"""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2605_01313_amd import nufft2  # noqa: F401  (fails loudly if not built)
    return torch, torch.device("cuda:0")


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def run_real(torch_dev, prec, coeffs, phi, theta, eps, **kw):
    torch, dev = torch_dev
    from paper_2605_01313_amd import Plan
    F, Kt, Kp = coeffs.shape
    plan = Plan(prec, Kt, Kp, n_fields=F, eps=eps, hermitian=True, **kw)
    cdt = np.complex64 if prec == "fp32" else np.complex128
    plan.setpts(torch.from_numpy(np.ascontiguousarray(phi)).to(dev),
                torch.from_numpy(np.ascontiguousarray(theta)).to(dev))
    out = plan.exec(torch.from_numpy(coeffs.astype(cdt)).to(dev))
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert got.dtype == (np.float32 if prec == "fp32" else np.float64)
    return plan, got


def half_series(coeffs):
    """Coefficients whose full series is the m >= 0 half with the m > 0
    terms doubled (the real-field plan's definition for any input)."""
    F, Kt, Kp = coeffs.shape
    h = np.zeros_like(coeffs)
    c0 = Kp // 2
    h[:, :, c0] = coeffs[:, :, c0]
    h[:, :, c0 + 1:] = 2.0 * coeffs[:, :, c0 + 1:]
    return h


def real_errors(got, ref):
    return [rel_l2(got[f], ref[f].real) for f in range(ref.shape[0])]


@pytest.mark.parametrize("prec,eps,tol", [("fp64", 1e-12, 1e-12), ("fp32", 1e-6, 1e-6)])
def test_real_small_workload_full(torch_dev, oracle_mod, prec, eps, tol):
    """32 x 64 grid, 2048 jittered points, every output."""
    wl = synth.workload_small_jitter()
    say(f"case real small_workload prec={prec}")
    plan, got = run_real(torch_dev, prec, wl.coeffs, wl.phi, wl.theta, eps)
    assert plan.check() == 0 and plan.info()["hermitian"] == 1
    ref = oracle_mod.dfs_eval(wl.coeffs, wl.phi, wl.theta)
    # the coefficients are those of a real field: the exact sum is real
    assert np.abs(ref.imag).max() <= 1e-13 * np.abs(ref.real).max()
    errs = real_errors(got, ref)
    say(f"  rel l2 {errs}")
    assert max(errs) <= tol


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_real_fft_stage_matches_numpy(torch_dev, prec):
    """Theta-pass output (m >= 0 columns) and the real fine grid on reached
    rows against numpy's ifft of the deconvolved, zero-padded coefficients."""
    torch, dev = torch_dev
    from paper_2605_01313_amd import nufft2
    rng = np.random.default_rng(23)
    Kt, Kp, F = 45, 61, 2
    coeffs = np.stack([synth.dfs_field_coeffs(rng, Kt, Kp, synth.envelope_algebraic(Kt, Kp, 1.0))
                       for _ in range(F)])
    phi = rng.uniform(0, 2 * np.pi, 500)
    theta = rng.uniform(0.3, 2.0, 500)
    say(f"case real fft_stage prec={prec}")
    eps = 1e-12 if prec == "fp64" else 1e-6
    plan, _ = run_real(torch_dev, prec, coeffs, phi, theta, eps)
    info = plan.info()
    nft, nfp, w, beta = info["nf_theta"], info["nf_phi"], info["w"], info["beta"]
    rdt = torch.float64 if prec == "fp64" else torch.float32
    cdt = torch.complex128 if prec == "fp64" else torch.complex64
    M = Kp // 2
    grid = plan.debug_tensor(0, rdt, (F, nft, nfp)).cpu().numpy()
    S = plan.debug_tensor(5, cdt, (F, nft, M + 1)).cpu().numpy()
    touched = plan.debug_tensor(4, torch.uint8, (nft,)).cpu().numpy().astype(bool)
    _, ct = nufft2.nufft2_kernel_correction(Kt, nft, w, beta)
    _, cp = nufft2.nufft2_kernel_correction(Kp, nfp, w, beta)
    n = np.arange(Kt) - Kt // 2
    m = np.arange(Kp) - Kp // 2
    tol = 1e-13 if prec == "fp64" else 2e-6
    assert touched.any() and not touched.all()
    for f in range(F):
        G = np.zeros((nft, nfp), complex)
        G[np.ix_(n % nft, m % nfp)] = coeffs[f] * ct[:, None] * cp[None, :]
        Sref = np.fft.ifft(G, axis=0) * nft
        err_s = rel_l2(S[f][touched], Sref[touched][:, :M + 1])
        ref = np.fft.ifft2(G) * nft * nfp
        assert np.abs(ref.imag).max() <= 1e-12 * np.abs(ref.real).max()
        err = rel_l2(grid[f][touched], ref.real[touched])
        say(f"  field {f} S rel l2 {err_s:.2e}, grid rel l2 {err:.2e}")
        assert err_s < tol and err < tol


@pytest.mark.parametrize("prec,eps,tol", [("fp64", 1e-12, 1e-12), ("fp32", 1e-6, 1e-6)])
def test_real_sbr_workload_full(torch_dev, sbr_full_ref, prec, eps, tol):
    """256 x 512 grid, all 131,072 solid-body-rotation departure points, 3 fields."""
    wl, ref = sbr_full_ref
    say(f"case real sbr prec={prec} (all points)")
    plan, got = run_real(torch_dev, prec, wl.coeffs, wl.phi, wl.theta, eps)
    assert plan.check() == 0
    errs = real_errors(got, ref)
    say(f"  rel l2 per field {errs}")
    assert max(errs) <= tol


@pytest.mark.parametrize("prec,eps,tol", [("fp32", 1e-6, 1e-6), ("fp64", 1e-12, 1e-12)])
def test_real_wind_1024x2048_full_size(torch_dev, wind_large_ref, prec, eps, tol):
    """The 1024 x 2048 workload at full size (2,097,152 wind departure
    points, 2047 x 2047 modes, 3 fields) in the configuration the bench
    times, on the 10^4 outputs per field that default_rng(15) samples."""
    wl, idx, ref = wind_large_ref
    say(f"case real wind1024 full size prec={prec}")
    plan, got = run_real(torch_dev, prec, wl.coeffs, wl.phi, wl.theta, eps)
    info = plan.info()
    assert plan.check() == 0 and info["n_pts"] == wl.n_pts and info["n_bins"] > 8192
    errs = real_errors(got[:, idx], ref)
    say(f"  rel l2 {errs}")
    assert max(errs) <= tol
    plan.destroy()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-6)])
def test_real_plan_agrees_with_the_complex_plan(torch_dev, prec, tol):
    """On coefficients of real fields the real-field plan and the complex
    plan compute the same values (different roundings, within tolerance)."""
    torch, dev = torch_dev
    from paper_2605_01313_amd import Plan
    rng = np.random.default_rng(91)
    K, F, P = 255, 3, 20000
    coeffs = np.stack([synth.dfs_field_coeffs(rng, K, K, synth.envelope_algebraic(K, K, 1.5)) for _ in range(F)])
    phi = rng.uniform(-1.0, 7.0, P)
    theta = rng.uniform(-0.4, np.pi + 0.4, P)
    say(f"case real_vs_complex prec={prec}")
    eps = 1e-12 if prec == "fp64" else 1e-6
    _, got = run_real(torch_dev, prec, coeffs, phi, theta, eps)
    cplan = Plan(prec, K, K, n_fields=F, eps=eps)
    cdt = torch.complex64 if prec == "fp32" else torch.complex128
    cplan.setpts(torch.from_numpy(phi).to(dev), torch.from_numpy(theta).to(dev))
    cout = cplan.exec(torch.from_numpy(coeffs).to(dev).to(cdt)).cpu().numpy()
    for f in range(F):
        err = rel_l2(got[f], cout[f].real)
        say(f"  field {f} rel l2 {err:.2e}")
        assert err <= tol
    cplan.destroy()


@pytest.mark.parametrize("prec,eps,tol", [("fp64", 1e-12, 3e-12), ("fp32", 1e-6, 3e-6)])
def test_real_plan_on_other_coefficients(torch_dev, oracle_mod, prec, eps, tol):
    """Coefficients that are not Hermitian: the result is the real part of
    the series of the m >= 0 half with m > 0 doubled (the columns m < 0 are
    never read: they hold NaN here)."""
    rng = np.random.default_rng(57)
    Kt, Kp, F, P = 31, 41, 2, 3000
    coeffs = synth.random_complex(rng, (F, Kt, Kp))
    phi = rng.uniform(-7, 14, P)
    theta = rng.uniform(-7, 14, P)
    say(f"case real_other_coeffs prec={prec}")
    poisoned = coeffs.copy()
    poisoned[:, :, :Kp // 2] = np.nan
    plan, got = run_real(torch_dev, prec, poisoned, phi, theta, eps)
    errs = real_errors(got, oracle_mod.dfs_eval(half_series(coeffs), phi, theta))
    say(f"  rel l2 {errs}")
    assert max(errs) <= tol


@pytest.mark.parametrize("Kt,Kp,P,F", [(3, 3, 1, 1), (7, 9, 37, 2), (63, 33, 1000, 3), (101, 257, 4097, 1),
                                       (255, 255, 3000, 4), (511, 15, 2000, 2)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_real_ragged_shapes(torch_dev, oracle_mod, Kt, Kp, P, F, prec):
    """Odd mode counts of every size class (down to 3 x 3, where the C2R
    transform has length 16), one point, point counts off the tile, 1-4
    fields, points all around the torus; flat-spectrum fields (3 eps)."""
    rng = np.random.default_rng(Kt * 1000 + Kp + P + 7)
    coeffs = np.stack([synth.dfs_field_coeffs(rng, Kt, Kp, np.ones((Kt, Kp))) for _ in range(F)])
    phi = rng.uniform(-7, 14, P)
    theta = rng.uniform(-7, 14, P)
    say(f"case real ragged K=({Kt},{Kp}) P={P} F={F} prec={prec}")
    eps, tol = (1e-12, 3e-12) if prec == "fp64" else (1e-6, 3e-6)
    plan, got = run_real(torch_dev, prec, coeffs, phi, theta, eps)
    assert plan.check() == 0
    errs = real_errors(got, oracle_mod.dfs_eval(coeffs, phi, theta))
    say(f"  rel l2 {errs}")
    assert max(errs) <= tol


@pytest.mark.parametrize("w", [4, 5, 6, 7, 8, 9])
def test_real_fp32_widths_converge(torch_dev, oracle_mod, w):
    """FP32 kernel weights by the direct formula (w < 7) and by the per-tap
    polynomials (w >= 7): the error falls with the width down to the FP32
    floor, on a decaying spectrum."""
    rng = np.random.default_rng(300 + w)
    K, P = 127, 4000
    coeffs = synth.dfs_field_coeffs(rng, K, K, synth.envelope_algebraic(K, K, 1.5))[None]
    phi = rng.uniform(0, 2 * np.pi, P)
    theta = rng.uniform(-0.1, np.pi + 0.1, P)
    say(f"case real fp32 w={w}")
    plan, got = run_real(torch_dev, "fp32", coeffs, phi, theta, 1e-6, w=w)
    assert plan.info()["w"] == w
    err = real_errors(got, oracle_mod.dfs_eval(coeffs, phi, theta))[0]
    # the FP64 plan of the same width: the FP32 result adds only rounding
    _, got64 = run_real(torch_dev, "fp64", coeffs, phi, theta, 1e-12, w=w)
    err64 = real_errors(got64, oracle_mod.dfs_eval(coeffs, phi, theta))[0]
    say(f"  rel l2 fp32 {err:.2e}, fp64 {err64:.2e}")
    assert err <= max(1.5 * err64, err64 + 6e-7)


def test_real_zero_and_one_point(torch_dev, oracle_mod):
    torch, dev = torch_dev
    from paper_2605_01313_amd import Plan
    say("case real zero/one point")
    rng = np.random.default_rng(5)
    K = 31
    coeffs = synth.dfs_field_coeffs(rng, K, K, synth.envelope_algebraic(K, K, 1.5))[None]
    plan = Plan("fp64", K, K, n_fields=1, eps=1e-12, hermitian=True)
    c = torch.from_numpy(coeffs).to(dev)
    e = torch.empty(0, dtype=torch.float64, device=dev)
    plan.setpts(e, e)
    assert plan.exec(c).shape == (1, 0)
    phi, theta = np.array([2.5]), np.array([-0.3])
    plan.setpts(torch.from_numpy(phi).to(dev), torch.from_numpy(theta).to(dev))
    got = plan.exec(c).cpu().numpy()
    assert plan.check() == 0
    ref = oracle_mod.dfs_eval(coeffs, phi, theta)
    assert abs(got[0, 0] - ref[0, 0].real) <= 1e-12 * abs(ref[0, 0])
    plan.destroy()


def test_real_members_in_a_group_match_single_plans(torch_dev, oracle_mod):
    """A group mixing real-field and complex members: every member's output
    is bit-identical to its plan run alone, and meets the oracle."""
    torch, dev = torch_dev
    from paper_2605_01313_amd import Group, Plan
    rng = np.random.default_rng(19)
    spec = [("fp32", 127, 3, 5000, True), ("fp32", 127, 3, 7000, True), ("fp64", 63, 2, 3000, True),
            ("fp32", 127, 1, 4000, False), ("fp32", 255, 2, 0, True)]
    plans, cs, phis, thetas, host = [], [], [], [], []
    for prec, K, F, n, herm in spec:
        coeffs = np.stack([synth.dfs_field_coeffs(rng, K, K, synth.envelope_algebraic(K, K, 1.5))
                           for _ in range(F)])
        phi = rng.uniform(-1.0, 7.3, n)
        theta = rng.uniform(-0.3, np.pi + 0.3, n)
        eps = 1e-6 if prec == "fp32" else 1e-12
        plans.append(Plan(prec, K, K, n_fields=F, eps=eps, hermitian=herm))
        cdt = torch.complex64 if prec == "fp32" else torch.complex128
        cs.append(torch.from_numpy(coeffs).to(dev).to(cdt))
        phis.append(torch.from_numpy(phi).to(dev))
        thetas.append(torch.from_numpy(theta).to(dev))
        host.append((coeffs, phi, theta, eps))
    say("case real group")
    g = Group(plans)
    g.setpts(phis, thetas)
    outs = [o.cpu().numpy() for o in g.exec(cs)]
    for i, p in enumerate(plans):
        p.setpts(phis[i], thetas[i])
        alone = p.exec(cs[i]).cpu().numpy()
        assert np.array_equal(alone, outs[i]), i
        coeffs, phi, theta, eps = host[i]
        if phi.size:
            ref = oracle_mod.dfs_eval(coeffs, phi, theta)
            errs = real_errors(outs[i], ref) if spec[i][4] else [rel_l2(outs[i][f], ref[f]) for f in range(ref.shape[0])]
            say(f"  member {i} rel l2 {max(errs):.2e}")
            assert max(errs) <= eps
    g.destroy()
    for p in plans:
        p.destroy()
