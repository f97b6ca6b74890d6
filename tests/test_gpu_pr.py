"""Partial-regularity expansion and zonal filter on the GPU (nufft2_pr_*,
nufft2_analysis_set_zonal_filter) against the oracle (section 4).

Tolerances.  pr coefficients solve normal equations whose matrices have
condition numbers kappa up to ~5e9 (odd m, N = 1023): both the oracle and the
GPU path are backward stable, so their pr coefficients may differ by about
kappa * 2^-52 relative to the largest one; the test computes kappa from the
oracle's matrices and allows 64 kappa 2^-52 (FP64 path; the FP32 path adds
the rounding of the output, 2^-23).  What the NUFFT consumes -- the
projection converted back to exp form -- is well conditioned and is held to
1e-12 (FP64) and 1e-6 (FP32) relative to its largest entry.
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


def real_field_exp(oracle_mod, rng, N, M, F, p=1.5):
    """Exp-form coefficients of F real DFS fields with an algebraic spectrum."""
    out = []
    for _ in range(F):
        fc = rng.standard_normal((N + 1, M + 1))
        fs = rng.standard_normal((N + 1, M + 1))
        n = np.arange(N + 1)[:, None]
        m = np.arange(M + 1)[None, :]
        env = (1.0 + n * n + m * m) ** (-p / 2)
        fc *= env
        fs *= env
        fs[:, 0] = 0.0
        fc[0, 1::2] = fs[0, 1::2] = 0.0
        out.append(oracle_mod.std_to_exp(fc, fs))
    return np.stack(out)


def oracle_project(oracle_mod, e):
    res = []
    for f in range(e.shape[0]):
        pc, ps = oracle_mod.std_to_pr(*oracle_mod.exp_to_std(e[f]))
        res.append(np.stack([pc, ps]))
    return np.stack(res)


def oracle_synth(oracle_mod, pr):
    return np.stack([oracle_mod.std_to_exp(*oracle_mod.pr_to_std(pr[f, 0], pr[f, 1])) for f in range(pr.shape[0])])


def kappa_max(oracle_mod, N):
    return max(np.linalg.cond(oracle_mod.normal_system(m, N)[0]) for m in (1, 2, 3))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("N,M,F", [(15, 15, 1), (63, 63, 3), (100, 37, 2), (255, 255, 1), (1023, 1023, 1)])
def test_project_and_synthesize_match_oracle(torch_dev, oracle_mod, prec, N, M, F):
    torch, dev = torch_dev
    from paper_2605_01313_amd import PartialRegularity
    say(f"case pr N={N} M={M} F={F} {prec}")
    rng = np.random.default_rng(N * 7 + M + F)
    e = real_field_exp(oracle_mod, rng, N, M, F)
    cdt = torch.complex64 if prec == "fp32" else torch.complex128
    if prec == "fp32":
        e = e.astype(np.complex64).astype(np.complex128)
    h = PartialRegularity(prec, N, M, n_fields=F)
    x = h.project(torch.from_numpy(e).to(cdt).to(dev))
    back = h.synthesize(x)
    x = x.cpu().numpy().astype(np.float64)
    back = back.cpu().numpy().astype(np.complex128)
    want_x = oracle_project(oracle_mod, e)
    kap = kappa_max(oracle_mod, N)
    tol_x = 64 * kap * 2.0 ** -52 + (2.0 ** -23 if prec == "fp32" else 0.0)
    err_x = np.abs(x - want_x).max() / np.abs(want_x).max()
    # zero outside each column's range, exactly
    for m in range(M + 1):
        lo, hi = oracle_mod.pr_range(m, N)
        mask = np.ones(N + 1, bool)
        mask[lo:hi + 1] = False
        assert not x[:, :, mask, m].any()
    assert not x[:, 1, :, 0].any()
    # the projection in exp form: GPU synthesis of GPU pr vs oracle chain
    want_back = oracle_synth(oracle_mod, want_x)
    err_b = np.abs(back - want_back).max() / np.abs(want_back).max()
    say(f"  kappa {kap:.2e}: pr err {err_x:.2e} (tol {tol_x:.1e}), projection err {err_b:.2e}")
    assert err_x <= tol_x
    assert err_b <= (1e-12 if prec == "fp64" else 1e-6)
    h.destroy()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_synthesize_matches_oracle_on_random_pr(torch_dev, oracle_mod, prec):
    torch, dev = torch_dev
    from paper_2605_01313_amd import PartialRegularity
    N, M, F = 40, 29, 2
    say(f"case pr_synth {prec}")
    rng = np.random.default_rng(5)
    pr = rng.standard_normal((F, 2, N + 1, M + 1))
    if prec == "fp32":
        pr = pr.astype(np.float32).astype(np.float64)
    rdt = torch.float32 if prec == "fp32" else torch.float64
    h = PartialRegularity(prec, N, M, n_fields=F)
    got = h.synthesize(torch.from_numpy(pr).to(rdt).to(dev)).cpu().numpy().astype(np.complex128)
    # entries outside the ranges are ignored: the oracle sees them zeroed
    clean = pr.copy()
    for m in range(M + 1):
        lo, hi = oracle_mod.pr_range(m, N)
        clean[:, :, :lo, m] = 0.0
        clean[:, :, hi + 1:, m] = 0.0
    clean[:, 1, :, 0] = 0.0
    want = oracle_synth(oracle_mod, clean)
    err = np.abs(got - want).max() / np.abs(want).max()
    say(f"  err {err:.2e}")
    assert err <= (1e-15 if prec == "fp64" else 2e-7)
    h.destroy()


def test_projection_is_idempotent_on_the_gpu(torch_dev, oracle_mod):
    torch, dev = torch_dev
    from paper_2605_01313_amd import PartialRegularity
    N = M = 127
    say("case pr_idempotent")
    rng = np.random.default_rng(8)
    e = torch.from_numpy(real_field_exp(oracle_mod, rng, N, M, 1)).to(dev)
    h = PartialRegularity("fp64", N, M)
    p1 = h.synthesize(h.project(e))
    p2 = h.synthesize(h.project(p1))
    err = float((p2 - p1).abs().max() / p1.abs().max())
    say(f"  err {err:.2e}")
    assert err <= 1e-12
    h.destroy()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 2e-6)])
@pytest.mark.parametrize("J", [64, 256])
def test_zonal_filtered_analysis_matches_oracle(torch_dev, oracle_mod, prec, tol, J):
    torch, dev = torch_dev
    from paper_2605_01313_amd import Analysis
    say(f"case zonal J={J} {prec}")
    rng = np.random.default_rng(J)
    vals = rng.standard_normal((2, J, 2 * J))
    if prec == "fp32":
        vals = vals.astype(np.float32).astype(np.float64)
    rdt = torch.float32 if prec == "fp32" else torch.float64
    an = Analysis(prec, J, n_fields=2)
    an.set_zonal_filter(20)
    v = torch.from_numpy(vals).to(rdt).to(dev)
    got = an.exec(v).cpu().numpy()
    want = oracle_mod.dfs_analysis(oracle_mod.zonal_filter(vals, 20))
    err = np.abs(got - want).max() / np.abs(want).max()
    say(f"  filtered err {err:.2e}")
    assert err <= tol
    an.set_zonal_filter(-1)
    got = an.exec(v).cpu().numpy()
    want = oracle_mod.dfs_analysis(vals)
    assert np.abs(got - want).max() / np.abs(want).max() <= tol
    an.destroy()


@pytest.mark.parametrize("prec,eps", [("fp64", 1e-12), ("fp32", 1e-6)])
def test_grid_to_departure_points_through_the_pr_basis(torch_dev, oracle_mod, prec, eps):
    """The model's chain (section 5): Grid [0] samples -> zonal filter and
    analysis -> pr projection -> exp form -> NUFFT at departure points,
    against the oracle's chain ending in the direct sum."""
    torch, dev = torch_dev
    from paper_2605_01313_amd import Analysis, PartialRegularity, Plan
    J, F = 64, 3
    N = M = J - 1
    say(f"case pr_chain {prec}")
    wl = synth.ensemble_member(synth.ensemble_members(n_small=1, n_large=0, J_small=J)[0], n_fields=F)
    th, ph = oracle_mod.grid0_nodes(J)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    vals = np.stack([oracle_mod.dfs_eval(wl.coeffs[f:f + 1], PH.ravel(), TH.ravel()).real.reshape(J, 2 * J)
                     for f in range(F)])
    if prec == "fp32":
        vals = vals.astype(np.float32).astype(np.float64)
    rdt = torch.float32 if prec == "fp32" else torch.float64
    an = Analysis(prec, J, n_fields=F)
    an.set_zonal_filter(20)
    h = PartialRegularity(prec, N, M, n_fields=F)
    plan = Plan(prec, 2 * N + 1, 2 * M + 1, n_fields=F, eps=eps)
    phi = torch.from_numpy(wl.phi).to(dev)
    theta = torch.from_numpy(wl.theta).to(dev)
    plan.setpts(phi, theta)
    coeffs = h.synthesize(h.project(an.exec(torch.from_numpy(vals).to(rdt).to(dev))))
    out = plan.exec(coeffs).cpu().numpy()
    ref_c = oracle_synth(oracle_mod, oracle_project(oracle_mod, oracle_mod.dfs_analysis(
        oracle_mod.zonal_filter(vals, 20))))
    sel = synth.sample_indices(wl.n_pts, 3000)
    ref = oracle_mod.dfs_eval(ref_c, wl.phi[sel], wl.theta[sel])
    err = max(float(np.linalg.norm(out[f, sel] - ref[f]) / np.linalg.norm(ref[f])) for f in range(F))
    say(f"  rel l2 {err:.2e}")
    assert err <= eps
    for o in (an, h, plan):
        o.destroy()


def test_pr_argument_errors(torch_dev):
    from paper_2605_01313_amd import nufft2
    assert nufft2.nufft2_pr_plan(1, 4, 10, 1)[0] == nufft2.NUFFT2_ERR_ARG       # N below 5
    assert nufft2.nufft2_pr_plan(1, 10, 2048, 1)[0] == nufft2.NUFFT2_ERR_ARG    # M above 2047
    assert nufft2.nufft2_pr_plan(3, 10, 10, 1)[0] == nufft2.NUFFT2_ERR_ARG      # precision
    assert nufft2.nufft2_pr_plan(2, 10, 10, 0)[0] == nufft2.NUFFT2_ERR_ARG      # no fields
    st, h = nufft2.nufft2_pr_plan(2, 10, 10, 1)
    assert st == nufft2.NUFFT2_OK
    assert nufft2.nufft2_pr_project(h, 0, 0) == nufft2.NUFFT2_ERR_ARG
    assert nufft2.nufft2_pr_synthesize(h, 0, 0) == nufft2.NUFFT2_ERR_ARG
    assert nufft2.nufft2_pr_destroy(h) == nufft2.NUFFT2_OK
    assert nufft2.nufft2_analysis_set_zonal_filter(None, 20) == nufft2.NUFFT2_ERR_ARG
