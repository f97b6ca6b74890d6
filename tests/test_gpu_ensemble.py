"""The uneven ensemble at full shape: 64 members on 128 x 256 grids and 16 on
256 x 512 grids, 3 fields each, every member with its own seed, spectrum
exponent and 8-mode wind (Courant number 2..8), run as one group (FP32,
eps 1e-6): each member meets the oracle on 128 sampled points per field.
"""
import multiprocessing as mp
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _member(spec):
    return synth.ensemble_member(spec)


@pytest.fixture(scope="module")
def members():
    specs = synth.ensemble_members()
    # spawned workers import numpy and scipy only, never the GPU runtime
    with ProcessPoolExecutor(max_workers=min(16, len(specs)), mp_context=mp.get_context("spawn")) as ex:
        out = list(ex.map(_member, specs))
    say(f"built {len(out)} members")
    return out


@pytest.mark.parametrize("herm", [False, True])
def test_full_ensemble_group_meets_oracle_per_member(members, oracle_mod, herm):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2605_01313_amd import Group, Plan
    dev = torch.device("cuda:0")
    assert len(members) == 80
    assert [m.coeffs.shape[-1] for m in members] == [255] * 64 + [511] * 16
    say(f"case ensemble_full 64 x 255^2 + 16 x 511^2 modes, 3 fields, fp32 eps 1e-6, "
        f"{'real-field' if herm else 'complex'} plans")
    plans, coeffs, phis, thetas, outs = [], [], [], [], []
    for m in members:
        F, Kt, Kp = m.coeffs.shape
        plans.append(Plan("fp32", Kt, Kp, n_fields=F, eps=1e-6, hermitian=herm))
        coeffs.append(torch.from_numpy(m.coeffs).to(dev).to(torch.complex64).contiguous())
        phis.append(torch.from_numpy(m.phi).to(dev))
        thetas.append(torch.from_numpy(m.theta).to(dev))
        outs.append(torch.empty((F, m.n_pts), dtype=torch.float32 if herm else torch.complex64, device=dev))
    g = Group(plans)
    info = g.info()
    say(f"  group: {info['n_members']} members, {info['n_classes']} classes")
    assert info["n_members"] == 80 and info["n_classes"] == 2
    g.setpts(phis, thetas)
    g.exec(coeffs, outs)
    torch.cuda.synchronize()
    for p in plans:
        assert p.check() == 0
    worst = 0.0
    for i, m in enumerate(members):
        sel = synth.sample_indices(m.n_pts, 128, seed=300 + i)
        ref = oracle_mod.dfs_eval(m.coeffs, m.phi[sel], m.theta[sel])
        if herm:
            ref = ref.real
        got = outs[i][:, torch.from_numpy(sel).to(dev)].cpu().numpy()
        err = max(float(np.linalg.norm(got[f] - ref[f]) / np.linalg.norm(ref[f])) for f in range(ref.shape[0]))
        worst = max(worst, err)
        assert err <= 1e-6, (i, err)
    say(f"  worst member rel l2 on 128 points x 3 fields: {worst:.2e}")
    g.destroy()
    for p in plans:
        p.destroy()
