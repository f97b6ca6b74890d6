"""Autotuner (nufft2_autotune): width by measured accuracy, tiles by time,
JSON cache; the tuned plan meets the oracle at the requested tolerance."""
import json
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

TILES = {(8, 32), (16, 32), (32, 16), (16, 64), (32, 32), (8, 64), (32, 64), (8, 128)}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2605_01313_amd import nufft2  # noqa: F401  (fails loudly if not built)
    return torch, torch.device("cuda:0")


@pytest.mark.parametrize("prec,eps,J,F,herm", [("fp32", 1e-6, 128, 3, False), ("fp64", 1e-12, 32, 1, False),
                                               ("fp32", 1e-6, 128, 3, True)])
def test_autotune_choice_cache_and_accuracy(torch_dev, oracle_mod, tmp_path, prec, eps, J, F, herm):
    torch, dev = torch_dev
    from paper_2605_01313_amd import Plan, autotune, nufft2_kernel_params
    say(f"case autotune prec={prec} J={J} {'real-field' if herm else 'complex'}")
    spec = synth.ensemble_members(n_small=1, n_large=0, J_small=J)[0]
    wl = synth.ensemble_member(spec, n_fields=F)
    K = wl.coeffs.shape[-1]
    phi = torch.from_numpy(wl.phi).to(dev)
    theta = torch.from_numpy(wl.theta).to(dev)
    cache = str(tmp_path / "tune.json")
    code = 1 if prec == "fp32" else 2
    _, w0, _ = nufft2_kernel_params(code, eps)
    r = autotune(prec, K, K, F, eps, phi, theta, cache_path=cache, hermitian=herm)
    say(f"  tuned {r}")
    assert w0 - 1 <= r["w"] <= w0 + 2
    assert (r["tile_theta"], r["tile_phi"]) in TILES
    assert r["from_cache"] == 0 and r["n_timed"] >= 3 and r["ms"] > 0
    assert r["err"] <= eps
    # the cache answers the same question without measuring
    r2 = autotune(prec, K, K, F, eps, phi, theta, cache_path=cache, hermitian=herm)
    assert r2["from_cache"] == 1
    assert (r2["w"], r2["tile_theta"], r2["tile_phi"]) == (r["w"], r["tile_theta"], r["tile_phi"])
    with open(cache) as f:
        entries = json.load(f)["nufft2_autotune"]
    assert len(entries) == 1 and entries[0]["w"] == r["w"]
    # the tuned plan meets the oracle on sampled points of this workload
    plan = Plan(prec, K, K, n_fields=F, eps=eps, w=r["w"], tile_theta=r["tile_theta"],
                tile_phi=r["tile_phi"], hermitian=herm)
    plan.setpts(phi, theta)
    cdt = torch.complex64 if prec == "fp32" else torch.complex128
    out = plan.exec(torch.from_numpy(wl.coeffs).to(dev).to(cdt)).cpu().numpy()
    sel = synth.sample_indices(wl.n_pts, 2000)
    ref = oracle_mod.dfs_eval(wl.coeffs, wl.phi[sel], wl.theta[sel])
    if herm:
        ref = ref.real
    err = max(float(np.linalg.norm(out[f, sel] - ref[f]) / np.linalg.norm(ref[f])) for f in range(F))
    say(f"  tuned plan rel l2 {err:.2e}")
    assert err <= eps
    plan.destroy()


def test_autotune_argument_errors(torch_dev):
    torch, dev = torch_dev
    from paper_2605_01313_amd import nufft2
    x = torch.zeros(8, dtype=torch.float64, device=dev)
    st, _, _ = nufft2.nufft2_autotune(1, 63, 63, 1, 1e-6, 0, x.data_ptr(), x.data_ptr())
    assert st == nufft2.NUFFT2_ERR_ARG                  # no points
    st, _, _ = nufft2.nufft2_autotune(1, 63, 63, 1, 1e-9, 8, x.data_ptr(), x.data_ptr())
    assert st == nufft2.NUFFT2_ERR_EPS_RANGE
    st, _, _ = nufft2.nufft2_autotune(1, 63, 63, 1, 1e-6, 8, 0, x.data_ptr())
    assert st == nufft2.NUFFT2_ERR_ARG


def test_autotune_at_the_fp32_floor_meets_eps_or_says_it_cannot(torch_dev, tmp_path):
    """eps 1e-7 in FP32 (the floor) on a flat-spectrum probe: the tuner either
    returns a width whose measured error is within eps, or ERR_EPS_RANGE with
    the closest width and error, and then writes no cache entry."""
    torch, dev = torch_dev
    import os

    from paper_2605_01313_amd import nufft2
    say("case autotune fp32 eps 1e-7")
    rng = np.random.default_rng(3)
    n = 20000
    phi = torch.from_numpy(rng.uniform(0, 2 * np.pi, n)).to(dev)
    theta = torch.from_numpy(rng.uniform(0, np.pi, n)).to(dev)
    cache = str(tmp_path / "tune.json")
    st, opts, res = nufft2.nufft2_autotune(nufft2.NUFFT2_FP32, 127, 127, 1, 1e-7, n, phi.data_ptr(),
                                           theta.data_ptr(), torch.cuda.current_stream().cuda_stream, cache)
    say(f"  status {st}, w {res.w}, err {res.err:.3e}")
    if st == nufft2.NUFFT2_OK:
        assert res.err <= 1e-7 and opts.w == res.w
        assert os.path.exists(cache)
    else:
        assert st == nufft2.NUFFT2_ERR_EPS_RANGE
        assert res.err > 1e-7 and res.w >= 8
        assert not os.path.exists(cache) or "eps1.000e-07" not in open(cache).read()


def test_autotune_group_times_tiles_on_a_group(torch_dev, oracle_mod, tmp_path):
    """nufft2_autotune_group: the same width as the single-plan tuner (the
    width search does not depend on members), a tile from the candidate
    list timed on a group of 6 plans, a cache entry of its own (key with
    _m6), and a group of plans with the tuned options meets the oracle."""
    torch, dev = torch_dev
    from paper_2605_01313_amd import Group, Plan, autotune, nufft2
    say("case autotune_group fp32 J=64 members=6 real-field")
    spec = synth.ensemble_members(n_small=1, n_large=0, J_small=64)[0]
    wl = synth.ensemble_member(spec, n_fields=3)
    K = wl.coeffs.shape[-1]
    phi = torch.from_numpy(wl.phi).to(dev)
    theta = torch.from_numpy(wl.theta).to(dev)
    cache = str(tmp_path / "tune.json")
    r1 = autotune("fp32", K, K, 3, 1e-6, phi, theta, cache_path=cache, hermitian=True)
    rg = autotune("fp32", K, K, 3, 1e-6, phi, theta, cache_path=cache, hermitian=True, members=6)
    say(f"  single {r1}\n  group  {rg}")
    assert rg["w"] == r1["w"] and rg["err"] == r1["err"]
    assert (rg["tile_theta"], rg["tile_phi"]) in TILES
    assert rg["from_cache"] == 0 and rg["n_timed"] >= 3 and rg["ms"] > 0
    with open(cache) as f:
        keys = [e["key"] for e in json.load(f)["nufft2_autotune"]]
    assert len(keys) == 2 and sum("_m6_" in k for k in keys) == 1
    rg2 = autotune("fp32", K, K, 3, 1e-6, phi, theta, cache_path=cache, hermitian=True, members=6)
    assert rg2["from_cache"] == 1 and (rg2["tile_theta"], rg2["tile_phi"]) == (rg["tile_theta"], rg["tile_phi"])
    plans = [Plan("fp32", K, K, n_fields=3, eps=1e-6, w=rg["w"], tile_theta=rg["tile_theta"],
                  tile_phi=rg["tile_phi"], hermitian=True) for _ in range(2)]
    g = Group(plans)
    g.setpts([phi, phi], [theta, theta])
    c = torch.from_numpy(wl.coeffs).to(dev).to(torch.complex64)
    outs = [o.cpu().numpy() for o in g.exec([c, c])]
    sel = synth.sample_indices(wl.n_pts, 1000)
    ref = oracle_mod.dfs_eval(wl.coeffs, wl.phi[sel], wl.theta[sel]).real
    for o in outs:
        err = max(float(np.linalg.norm(o[f, sel] - ref[f]) / np.linalg.norm(ref[f])) for f in range(3))
        assert err <= 1e-6, err
    g.destroy()
    for p in plans:
        p.destroy()
    # argument checks (before any device work)
    x = torch.zeros(8, dtype=torch.float64, device=dev)
    for members, n in ((0, 8), (4097, 8), (2, 1 << 30)):
        st, _, _ = nufft2.nufft2_autotune_group(1, 63, 63, 1, 1e-6, members, n, x.data_ptr(), x.data_ptr())
        assert st == nufft2.NUFFT2_ERR_ARG, (members, n)
