"""Vector rotation at the departure points (nufft2_rotate_uv, section 3's
matrix Q) against the oracle: interpolate (u, v) with the plan, rotate on
the GPU, compare with the oracle's direct sum rotated by the oracle's Q."""
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


@pytest.mark.parametrize("prec,eps", [("fp64", 1e-12), ("fp32", 1e-6)])
def test_rotate_uv_matches_oracle(torch_dev, oracle_mod, prec, eps):
    torch, dev = torch_dev
    from paper_2605_01313_amd import Plan
    say(f"case rotate_uv {prec}")
    wl = synth.workload_wind(32, (5, 6, 7), 8, 6.0)        # h, u, v on a 32 x 64 grid, Courant 6
    phi_a, theta_a = synth.grid0_points(32)
    F, K, _ = wl.coeffs.shape
    cdt = torch.complex64 if prec == "fp32" else torch.complex128
    plan = Plan(prec, K, K, n_fields=F, eps=eps)
    plan.setpts(torch.from_numpy(wl.phi).to(dev), torch.from_numpy(wl.theta).to(dev))
    out = plan.exec(torch.from_numpy(wl.coeffs).to(dev).to(cdt))
    plan.rotate_uv(out, 1, 2, torch.from_numpy(phi_a).to(dev), torch.from_numpy(theta_a).to(dev))
    got = out.cpu().numpy()
    ref = oracle_mod.dfs_eval(wl.coeffs, wl.phi, wl.theta)
    ur, vr = oracle_mod.rotate_uv(ref[1], ref[2], phi_a, theta_a, wl.phi, wl.theta)
    assert np.array_equal(got[0], plan.exec(torch.from_numpy(wl.coeffs).to(dev).to(cdt)).cpu().numpy()[0])
    num = np.sqrt(np.linalg.norm(got[1] - ur) ** 2 + np.linalg.norm(got[2] - vr) ** 2)
    err = float(num / np.sqrt(np.linalg.norm(ur) ** 2 + np.linalg.norm(vr) ** 2))
    say(f"  rotated (u, v) rel l2 {err:.2e}")
    assert err <= eps
    plan.destroy()


def test_rotate_uv_identity_without_displacement(torch_dev):
    torch, dev = torch_dev
    from paper_2605_01313_amd import Plan
    rng = np.random.default_rng(1)
    K = 31
    c = synth.random_complex(rng, (2, K, K))
    phi = torch.from_numpy(rng.uniform(0, 2 * np.pi, 700)).to(dev)
    theta = torch.from_numpy(rng.uniform(0.1, 3.0, 700)).to(dev)
    plan = Plan("fp64", K, K, n_fields=2, eps=1e-12)
    plan.setpts(phi, theta)
    out = plan.exec(torch.from_numpy(c).to(dev))
    before = out.cpu().numpy().copy()
    plan.rotate_uv(out, 0, 1, phi, theta)                  # arrival == departure: p = 1, q = 0
    # to rounding: p is (s^2 + 1 + c^2) / (1 + s^2 + c^2) in FP64
    assert np.abs(out.cpu().numpy() - before).max() <= 1e-15 * np.abs(before).max()
    plan.destroy()


def test_rotate_uv_argument_errors(torch_dev):
    torch, dev = torch_dev
    from paper_2605_01313_amd import Plan, nufft2
    plan = Plan("fp32", 15, 15, n_fields=2, eps=1e-6)
    x = torch.zeros(4, dtype=torch.float64, device=dev)
    assert nufft2.nufft2_rotate_uv(plan.handle, x.data_ptr(), 0, 1, x.data_ptr(), x.data_ptr(), x.data_ptr(),
                                   x.data_ptr()) == nufft2.NUFFT2_ERR_NO_POINTS
    plan.setpts(x, x)
    for fu, fv in ((0, 0), (0, 2), (-1, 1)):
        assert nufft2.nufft2_rotate_uv(plan.handle, x.data_ptr(), fu, fv, x.data_ptr(), x.data_ptr(),
                                       x.data_ptr(), x.data_ptr()) == nufft2.NUFFT2_ERR_ARG
    assert nufft2.nufft2_rotate_uv(plan.handle, x.data_ptr(), 0, 1, 0, x.data_ptr(), x.data_ptr(),
                                   x.data_ptr()) == nufft2.NUFFT2_ERR_ARG
    plan.destroy()
