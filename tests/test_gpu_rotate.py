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


# ---- the rotation inside the gather (nufft2_setpts_vector) -----------------

def rel_uv(got_u, got_v, ur, vr):
    num = np.sqrt(np.linalg.norm(got_u - ur) ** 2 + np.linalg.norm(got_v - vr) ** 2)
    return float(num / np.sqrt(np.linalg.norm(ur) ** 2 + np.linalg.norm(vr) ** 2))


# J = 32: small plan (fused scan + scatter); J = 512: one scan pass with the
# scatter kernel; both precisions, real-field and complex plans
@pytest.mark.parametrize("J", [32, 512])
@pytest.mark.parametrize("prec,eps,herm", [("fp64", 1e-12, False), ("fp32", 1e-6, False),
                                           ("fp64", 1e-12, True), ("fp32", 1e-6, True)])
def test_setpts_vector_rotates_inside_exec(torch_dev, oracle_mod, J, prec, eps, herm):
    """Fields (u, v) = (1, 2) come out rotated into the arrival frame; field 0
    is untouched; at sampled points both meet the oracle's direct sum (rotated
    by the oracle's Q) at the plan tolerance, and the result agrees with the
    separate rotation pass to about the FP32 trigonometric error."""
    torch, dev = torch_dev
    from paper_2605_01313_amd import Plan
    say(f"case setpts_vector J={J} {prec} {'real-field' if herm else 'complex'}")
    wl = synth.workload_wind(J, (5, 6, 7), 8, 6.0)
    phi_a, theta_a = synth.grid0_points(J)
    F, K, _ = wl.coeffs.shape
    cdt = torch.complex64 if prec == "fp32" else torch.complex128
    plan = Plan(prec, K, K, n_fields=F, eps=eps, hermitian=herm)
    info = plan.info()
    assert 1 // info["fields_per_pass"] == 2 // info["fields_per_pass"]     # u, v in one gather pass
    c = torch.from_numpy(wl.coeffs).to(dev).to(cdt)
    phi, theta = torch.from_numpy(wl.phi).to(dev), torch.from_numpy(wl.theta).to(dev)
    pa, ta = torch.from_numpy(phi_a).to(dev), torch.from_numpy(theta_a).to(dev)
    plan.setpts(phi, theta)
    plain = plan.exec(c).clone()
    plan.rotate_uv(plain, 1, 2, pa, ta)                    # the separate pass
    plan.setpts_vector(phi, theta, pa, ta, 1, 2)
    fused = plan.exec(c)
    torch.cuda.synchronize()
    got, sep = fused.cpu().numpy(), plain.cpu().numpy()
    assert np.array_equal(got[0], sep[0])
    sel = synth.sample_indices(wl.n_pts, 2000, seed=J)
    ref = oracle_mod.dfs_eval(wl.coeffs, wl.phi[sel], wl.theta[sel])
    if herm:
        ref = ref.real
    ur, vr = oracle_mod.rotate_uv(ref[1], ref[2], phi_a[sel], theta_a[sel], wl.phi[sel], wl.theta[sel])
    err = rel_uv(got[1][sel], got[2][sel], ur, vr)
    e0 = float(np.linalg.norm(got[0][sel] - ref[0]) / np.linalg.norm(ref[0]))
    d = rel_uv(got[1], got[2], sep[1], sep[2])
    say(f"  rotated (u, v) rel l2 {err:.2e}; field 0 {e0:.2e}; fused vs separate pass {d:.2e}")
    assert err <= eps and e0 <= eps
    assert d <= (1e-14 if prec == "fp64" else 3e-7)
    # a plain setpts drops the rotation
    plan.setpts(phi, theta)
    again = plan.exec(c).cpu().numpy()
    plan.rotate_uv(plan.exec(c), 1, 2, pa, ta)
    assert not np.array_equal(again[1], got[1])
    plan.destroy()


def test_setpts_vector_at_the_wind_workload(torch_dev, wind_large_ref):
    """1024 x 2048 wind workload (several scan passes), real-field FP32 plan:
    the rotated (u, v) at the 10^4 sampled points within 1e-6 of the oracle."""
    torch, dev = torch_dev
    from paper_2605_01313_amd import Plan
    import oracle
    say("case setpts_vector wind1024 fp32 real-field")
    wl, idx, ref = wind_large_ref
    phi_a, theta_a = synth.grid0_points(wl.J)
    F, K, _ = wl.coeffs.shape
    plan = Plan("fp32", K, K, n_fields=F, eps=1e-6, hermitian=True)
    assert plan.info()["n_bins"] > 8192
    plan.setpts_vector(torch.from_numpy(wl.phi).to(dev), torch.from_numpy(wl.theta).to(dev),
                       torch.from_numpy(phi_a).to(dev), torch.from_numpy(theta_a).to(dev), 1, 2)
    out = plan.exec(torch.from_numpy(wl.coeffs).to(dev).to(torch.complex64))
    got = out[:, torch.from_numpy(idx).to(dev)].cpu().numpy()
    ur, vr = oracle.rotate_uv(ref[1].real, ref[2].real, phi_a[idx], theta_a[idx], wl.phi[idx], wl.theta[idx])
    err = rel_uv(got[1], got[2], ur, vr)
    say(f"  rotated (u, v) rel l2 on 10^4 points {err:.2e}")
    assert err <= 1e-6
    plan.destroy()


def test_setpts_vector_argument_errors(torch_dev):
    torch, dev = torch_dev
    from paper_2605_01313_amd import Plan, nufft2
    plan = Plan("fp32", 15, 15, n_fields=3, eps=1e-6)
    x = torch.zeros(4, dtype=torch.float64, device=dev)
    p = x.data_ptr()
    for fu, fv in ((0, 0), (0, 3), (-1, 1)):
        assert nufft2.nufft2_setpts_vector(plan.handle, 4, p, p, p, p, fu, fv) == nufft2.NUFFT2_ERR_ARG
    assert nufft2.nufft2_setpts_vector(plan.handle, 4, p, p, 0, p, 1, 2) == nufft2.NUFFT2_ERR_ARG
    assert nufft2.nufft2_setpts_vector(plan.handle, 4, p, p, p, p, 1, 2) == nufft2.NUFFT2_OK
    plan.destroy()
    # fields in different gather passes: a plan that stages one field at a time
    big = Plan("fp64", 511, 511, n_fields=2, eps=1e-12, tile_theta=32, tile_phi=64)
    fpp = big.info()["fields_per_pass"]
    say(f"  fp64 32x64 tiles: {fpp} field(s) per pass")
    assert fpp == 1
    assert nufft2.nufft2_setpts_vector(big.handle, 4, p, p, p, p, 0, 1) == nufft2.NUFFT2_ERR_ARG
    big.destroy()
