"""Gauss-Legendre DFS analysis on the GPU (nufft2_gl_*: FFT in longitude,
the latitude inversion on the matrix cores) against the oracle
(eq. GLGrid; section 5's interpolation for the SHT model).

Tolerance: the latitude matrices have condition numbers below 5 for every
supported J, so the coefficients carry a few units of rounding of the plan
precision, growing like the square root of the length of the J-term
latitude product (rounding errors of random sign): 1e-13 (FP64) and
2e-6 max(1, sqrt(J / 256)) (FP32, on FP32-rounded samples), relative to the
largest coefficient.
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


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 2e-6)])
@pytest.mark.parametrize("J,F", [(16, 1), (64, 3), (256, 2), (512, 1), (1024, 1)])
def test_gl_analysis_matches_oracle(torch_dev, oracle_mod, prec, tol, J, F):
    torch, dev = torch_dev
    from paper_2605_01313_amd import GLAnalysis
    say(f"case gl J={J} F={F} {prec}")
    rng = np.random.default_rng(J + 10 * F)
    vals = rng.standard_normal((F, J, 2 * J))
    if prec == "fp32":
        vals = vals.astype(np.float32).astype(np.float64)
    rdt = torch.float32 if prec == "fp32" else torch.float64
    gl = GLAnalysis(prec, J, n_fields=F)
    got = gl.exec(torch.from_numpy(vals).to(rdt).to(dev)).cpu().numpy()
    want = oracle_mod.gl_analysis(vals)
    err = np.abs(got - want).max() / np.abs(want).max()
    if prec == "fp32":
        tol *= max(1.0, np.sqrt(J / 256))
    say(f"  max err / max coeff {err:.2e} (tol {tol:.1e})")
    assert err <= tol
    # every entry is written: a second call into a buffer of NaNs gives the same
    cdt = torch.complex64 if prec == "fp32" else torch.complex128
    out = torch.full((F, 2 * J + 1, 2 * J - 1), float("nan"), dtype=cdt, device=dev)
    again = gl.exec(torch.from_numpy(vals).to(rdt).to(dev), out=out).cpu().numpy()
    assert np.array_equal(again, got)
    gl.destroy()


@pytest.mark.parametrize("prec,eps", [("fp64", 1e-12), ("fp32", 1e-6)])
def test_gl_then_exec_at_departure_points(torch_dev, oracle_mod, prec, eps):
    """A band-limited field sampled on the GL grid -> GPU analysis -> NUFFT
    at departure points of an 8-mode wind, against the oracle's direct sum of
    the original series."""
    torch, dev = torch_dev
    from paper_2605_01313_amd import GLAnalysis, Plan
    J, F = 128, 3
    say(f"case gl_chain {prec}")
    wl = synth.ensemble_member(synth.ensemble_members(n_small=1, n_large=0, J_small=J)[0], n_fields=F)
    K = 2 * J - 1
    th, ph = oracle_mod.gl_nodes(J)
    T, P = np.meshgrid(th, ph, indexing="ij")
    vals = oracle_mod.dfs_eval(wl.coeffs, P.ravel(), T.ravel()).real.reshape(F, J, 2 * J)
    rdt = torch.float32 if prec == "fp32" else torch.float64
    gl = GLAnalysis(prec, J, n_fields=F)
    coeffs = gl.exec(torch.from_numpy(vals).to(rdt).to(dev))
    # the original (2J-1)^2 series sits inside the (2J+1) x (2J-1) result
    c = coeffs.cpu().numpy()
    inner = c[:, 1:-1, :]
    rel = np.abs(inner - wl.coeffs).max() / np.abs(wl.coeffs).max()
    say(f"  coefficient recovery {rel:.2e}")
    assert rel <= (1e-12 if prec == "fp64" else 2e-6)
    assert np.abs(c[:, [0, -1], :]).max() <= (1e-12 if prec == "fp64" else 2e-6) * np.abs(wl.coeffs).max()
    plan = Plan(prec, 2 * J + 1, K, n_fields=F, eps=eps)
    plan.setpts(torch.from_numpy(wl.phi).to(dev), torch.from_numpy(wl.theta).to(dev))
    out = plan.exec(coeffs).cpu().numpy()
    sel = synth.sample_indices(wl.n_pts, 3000)
    ref = oracle_mod.dfs_eval(wl.coeffs, wl.phi[sel], wl.theta[sel])
    err = max(float(np.linalg.norm(out[f, sel] - ref[f]) / np.linalg.norm(ref[f])) for f in range(F))
    say(f"  rel l2 at departure points {err:.2e}")
    assert err <= eps
    gl.destroy()
    plan.destroy()


def test_gl_argument_errors(torch_dev):
    from paper_2605_01313_amd import nufft2
    st, h = nufft2.nufft2_gl_plan(2, 64, 1)
    assert st == nufft2.NUFFT2_OK
    assert nufft2.nufft2_gl_exec(h, 0, 0) == nufft2.NUFFT2_ERR_ARG
    assert nufft2.nufft2_gl_destroy(h) == nufft2.NUFFT2_OK
