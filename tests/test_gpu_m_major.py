"""The m-major coefficient layout (opts.m_major, nufft2_analysis_set_layout).

A plan created with m_major = 1 takes the coefficients as [F][K_phi][K_theta];
its theta pass loads the same values from other addresses and runs the same
arithmetic, so its outputs must be bit-identical to those of the plan taking
[F][K_theta][K_phi] (which the other tests hold against the oracle).  The
analysis written m-major must be the transpose of the analysis written
row-major, bit for bit.
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


def workload(J):
    if J == 1024:
        return synth.workload_large()
    return synth.workload_wind(J, (21, 22, 23), 24, 4.0)


# J = 32: fused setpts; 256: one scan pass; 1024: the 1024 x 2048 wind
# workload (theta batches of 4 / 2 columns at compile time)
@pytest.mark.parametrize("J", [32, 256, 1024])
@pytest.mark.parametrize("prec,eps,herm", [("fp32", 1e-6, True), ("fp64", 1e-12, True), ("fp32", 1e-6, False),
                                           ("fp64", 1e-12, False)])
def test_m_major_plan_is_bit_identical(torch_dev, oracle_mod, J, prec, eps, herm):
    torch, dev = torch_dev
    from paper_2605_01313_amd import Plan
    say(f"case m_major J={J} {prec} {'real-field' if herm else 'complex'}")
    wl = workload(J)
    F, K, _ = wl.coeffs.shape
    cdt = torch.complex64 if prec == "fp32" else torch.complex128
    phi, theta = torch.from_numpy(wl.phi).to(dev), torch.from_numpy(wl.theta).to(dev)
    c = torch.from_numpy(wl.coeffs).to(dev).to(cdt).contiguous()
    ct = c.transpose(1, 2).contiguous()                     # [F][K_phi][K_theta]
    a = Plan(prec, K, K, n_fields=F, eps=eps, hermitian=herm)
    b = Plan(prec, K, K, n_fields=F, eps=eps, hermitian=herm, m_major=True)
    assert b.info()["m_major"] == 1 and a.info()["m_major"] == 0
    a.setpts(phi, theta)
    b.setpts(phi, theta)
    ra = a.exec(c).cpu().numpy()
    rb = b.exec(ct).cpu().numpy()
    assert np.array_equal(ra, rb)
    if J == 32:                                            # and against the oracle
        ref = oracle_mod.dfs_eval(wl.coeffs, wl.phi, wl.theta)
        if herm:
            ref = ref.real
        err = max(float(np.linalg.norm(rb[f] - ref[f]) / np.linalg.norm(ref[f])) for f in range(F))
        say(f"  rel l2 {err:.2e}")
        assert err <= eps
    a.destroy()
    b.destroy()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("J", [16, 256, 1024])
def test_analysis_m_major_is_the_transpose(torch_dev, prec, J):
    torch, dev = torch_dev
    from paper_2605_01313_amd import Analysis
    say(f"case analysis m_major J={J} {prec}")
    rng = np.random.default_rng(J)
    rdt = torch.float32 if prec == "fp32" else torch.float64
    vals = torch.from_numpy(rng.standard_normal((2, J, 2 * J))).to(dev).to(rdt)
    an = Analysis(prec, J, n_fields=2)
    rows = an.exec(vals).clone()
    an.set_layout(True)
    cols = an.exec(vals)
    assert torch.equal(cols, rows.transpose(1, 2).contiguous())
    an.set_layout(False)
    assert torch.equal(an.exec(vals), rows)
    an.destroy()


def test_m_major_group_and_analysis_chain(torch_dev, oracle_mod):
    """Grid values -> analysis written m-major -> a group of m-major plans:
    bit-identical to the row-major chain, and the group to single plans."""
    torch, dev = torch_dev
    from paper_2605_01313_amd import Analysis, Group, Plan
    say("case m_major chain")
    J = 64
    K = 2 * J - 1
    rng = np.random.default_rng(3)
    coeffs = synth.random_complex(rng, (2, K, K)) * synth.envelope_algebraic(K, K, 1.5)[None]
    phi_a, theta_a = synth.grid0_points(J)
    vals = oracle_mod.dfs_eval(coeffs, phi_a, theta_a).real.reshape(2, J, 2 * J)
    an = Analysis("fp64", J, n_fields=2)
    an.set_layout(True)
    cm = an.exec(torch.from_numpy(vals).to(dev)).clone()
    an.set_layout(False)
    cr = an.exec(torch.from_numpy(vals).to(dev)).clone()
    an.destroy()
    pts = [(torch.from_numpy(rng.uniform(0, 2 * np.pi, n)).to(dev), torch.from_numpy(rng.uniform(0, np.pi, n)).to(dev))
           for n in (3000, 5000)]
    pm = [Plan("fp64", K, K, n_fields=2, eps=1e-12, m_major=True) for _ in pts]
    pr = [Plan("fp64", K, K, n_fields=2, eps=1e-12) for _ in pts]
    g = Group(pm)
    g.setpts([p for p, _ in pts], [t for _, t in pts])
    outs = [o.clone() for o in g.exec([cm, cm])]
    for (phi, theta), p_r, o in zip(pts, pr, outs):
        p_r.setpts(phi, theta)
        assert torch.equal(p_r.exec(cr), o)
    g.destroy()
    for p in pm + pr:
        p.destroy()
