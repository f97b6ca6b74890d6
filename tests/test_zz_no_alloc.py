"""nufft2_exec_noalloc (setpts + exec without a plan and without device
allocation, every workspace in the library's static device array) against
the plan path: the same kernels run, so the outputs are bit-identical;
checked on two calls in a row, the second with a smaller input, and for a
size beyond the array (rejected before anything is enqueued)."""
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


def plan_path(torch, dev, prec, coeffs, phi, theta, eps, hermitian):
    from paper_2605_01313_amd import Plan
    F, Kt, Kp = coeffs.shape
    p = Plan(prec, Kt, Kp, n_fields=F, eps=eps, hermitian=hermitian)
    p.setpts(phi, theta)
    out = p.exec(coeffs).clone()
    torch.cuda.synchronize()
    p.destroy()
    return out


def noalloc_path(torch, dev, prec, coeffs, phi, theta, eps, hermitian):
    from paper_2605_01313_amd import nufft2
    F, Kt, Kp = coeffs.shape
    rdt = torch.float32 if prec == "fp32" else torch.float64
    out = torch.empty((F, phi.numel()), dtype=rdt if hermitian else coeffs.dtype, device=dev)
    opts = nufft2.nufft2_opts(0, 0.0, 0, 0, 0, int(hermitian))
    code = nufft2.NUFFT2_FP32 if prec == "fp32" else nufft2.NUFFT2_FP64
    s = torch.cuda.current_stream()
    st = nufft2.nufft2_exec_noalloc(code, Kt, Kp, F, eps, opts, phi.numel(), phi.data_ptr(), theta.data_ptr(),
                                    coeffs.data_ptr(), out.data_ptr(), s.cuda_stream)
    assert st == nufft2.NUFFT2_OK, nufft2.nufft2_strerror(st)
    torch.cuda.synchronize()
    return out


def inputs(torch, dev, prec, K, F, P, seed):
    rng = np.random.default_rng(seed)
    coeffs = np.stack([synth.dfs_field_coeffs(rng, K, K, synth.envelope_algebraic(K, K, 1.5)) for _ in range(F)])
    phi = rng.uniform(-1.0, 7.3, P)
    theta = rng.uniform(-0.3, np.pi + 0.3, P)
    cdt = torch.complex64 if prec == "fp32" else torch.complex128
    return (coeffs, phi, theta,
            torch.from_numpy(coeffs).to(dev).to(cdt), torch.from_numpy(phi).to(dev), torch.from_numpy(theta).to(dev))


@pytest.mark.parametrize("prec,eps,hermitian", [("fp32", 1e-6, True), ("fp32", 1e-6, False),
                                                ("fp64", 1e-12, True), ("fp64", 1e-12, False)])
def test_noalloc_matches_the_plan_path(torch_dev, oracle_mod, prec, eps, hermitian):
    torch, dev = torch_dev
    # two calls in a row, the second with a smaller input (fewer modes,
    # fields and points); then the first again (its tables are re-uploaded)
    for K, F, P, seed in ((255, 3, 40000, 1), (63, 2, 3000, 2), (255, 3, 40000, 1)):
        say(f"case noalloc prec={prec} hermitian={hermitian} K={K} F={F} P={P}")
        coeffs, phi, theta, c, ph, th = inputs(torch, dev, prec, K, F, P, seed)
        got = noalloc_path(torch, dev, prec, c, ph, th, eps, hermitian).cpu().numpy()
        want = plan_path(torch, dev, prec, c, ph, th, eps, hermitian).cpu().numpy()
        assert np.array_equal(got, want)
        sel = synth.sample_indices(P, 300, seed=3)
        ref = oracle_mod.dfs_eval(coeffs, phi[sel], theta[sel])
        if hermitian:
            ref = ref.real
        err = max(float(np.linalg.norm(got[f, sel] - ref[f]) / np.linalg.norm(ref[f])) for f in range(F))
        say(f"  bit-identical to the plan path; rel l2 {err:.2e}")
        assert err <= eps


def test_noalloc_rejects_what_does_not_fit(torch_dev):
    """1024 x 2048 grids (2047 x 2047 modes) need more than the static
    array: ERR_ARG before anything is enqueued (the output is untouched)."""
    torch, dev = torch_dev
    from paper_2605_01313_amd import nufft2
    st, cap = nufft2.nufft2_noalloc_capacity()
    assert st == nufft2.NUFFT2_OK and cap == 128 << 20
    say("case noalloc too large")
    K = 2047
    c = torch.zeros((1, K, K), dtype=torch.complex64, device=dev)
    ph = torch.zeros(16, dtype=torch.float64, device=dev)
    out = torch.full((1, 16), 7.0, dtype=torch.complex64, device=dev)
    st = nufft2.nufft2_exec_noalloc(nufft2.NUFFT2_FP32, K, K, 1, 1e-6, None, 16, ph.data_ptr(), ph.data_ptr(),
                                    c.data_ptr(), out.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert st == nufft2.NUFFT2_ERR_ARG
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
    # nothing enqueued for zero points, and argument errors before any work
    assert nufft2.nufft2_exec_noalloc(nufft2.NUFFT2_FP32, 63, 63, 1, 1e-6, None, 0, 0, 0, 0, 0, 0) == nufft2.NUFFT2_OK
    assert nufft2.nufft2_exec_noalloc(nufft2.NUFFT2_FP32, 63, 63, 1, 1e-6, None, 5, 0, 0, 0, 0, 0) == \
        nufft2.NUFFT2_ERR_ARG
    assert nufft2.nufft2_exec_noalloc(nufft2.NUFFT2_FP32, 63, 63, 1, 1e-9, None, 5, ph.data_ptr(), ph.data_ptr(),
                                      c.data_ptr(), out.data_ptr(), 0) == nufft2.NUFFT2_ERR_EPS_RANGE
