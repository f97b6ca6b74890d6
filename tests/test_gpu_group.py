"""Groups of plans (nufft2_group_*): segmented launches in HIP graphs.

A group runs the same kernel bodies as single plans, so every member's
output must be bit-identical to running its plan alone; on top of that the
outputs meet the oracle at the plan tolerance.
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


# (prec, K, F, n_pts, eps): uneven sizes, both precisions, a member without
# points, and two members of the same class
MEMBERS = [
    ("fp32", 63, 1, 3000, 1e-6),
    ("fp32", 127, 3, 9000, 1e-6),
    ("fp32", 63, 1, 2500, 1e-6),
    ("fp64", 31, 2, 1500, 1e-12),
    ("fp32", 255, 2, 0, 1e-6),
    ("fp64", 63, 1, 4000, 1e-12),
]


def make_inputs(seed):
    rng = np.random.default_rng(seed)
    data = []
    for prec, K, F, n, eps in MEMBERS:
        coeffs = synth.random_complex(rng, (F, K, K)) * synth.envelope_algebraic(K, K, 1.5)[None]
        phi = rng.uniform(-1.0, 2 * np.pi + 1.0, n)
        theta = rng.uniform(-0.3, np.pi + 0.3, n)
        data.append((coeffs, phi, theta))
    return data


def to_dev(torch, dev, prec, coeffs, phi, theta):
    cdt = torch.complex64 if prec == "fp32" else torch.complex128
    return (torch.from_numpy(coeffs).to(dev).to(cdt), torch.from_numpy(phi).to(dev),
            torch.from_numpy(theta).to(dev))


def build(torch_dev):
    from paper_2605_01313_amd import Group, Plan
    plans = [Plan(prec, K, K, n_fields=F, eps=eps) for prec, K, F, n, eps in MEMBERS]
    return plans, Group(plans)


def test_group_info_classes(torch_dev):
    plans, g = build(torch_dev)
    info = g.info()
    say(f"case group_info {info}")
    # classes: fp32 K63 F1 (2 members), fp32 K127 F3, fp64 K31 F2, fp32 K255 F2, fp64 K63 F1
    assert info["n_members"] == len(MEMBERS) and info["n_classes"] == 5
    assert info["exec_kernels"] == 15 and info["setpts_kernels"] == 6
    g.destroy()


def test_group_bit_identical_to_single_and_meets_oracle(torch_dev, oracle_mod):
    torch, dev = torch_dev
    say("case group_vs_single")
    data = make_inputs(7)
    plans, g = build(torch_dev)
    devin = [to_dev(torch, dev, m[0], *d) for m, d in zip(MEMBERS, data)]
    g.setpts([x[1] for x in devin], [x[2] for x in devin])
    outs = [o.clone() for o in g.exec([x[0] for x in devin])]
    torch.cuda.synchronize()
    for p in plans:
        assert p.check() == 0
    # the same plans run one by one
    for i, (p, x) in enumerate(zip(plans, devin)):
        p.setpts(x[1], x[2])
        single = p.exec(x[0])
        torch.cuda.synchronize()
        a, b = outs[i].cpu().numpy(), single.cpu().numpy()
        assert a.shape == b.shape
        assert np.array_equal(a, b), f"member {i} differs from its single run"
    # oracle on every member with points
    for i, ((prec, K, F, n, eps), (coeffs, phi, theta)) in enumerate(zip(MEMBERS, data)):
        if n == 0:
            continue
        ref = oracle_mod.dfs_eval(coeffs, phi, theta)
        got = outs[i].cpu().numpy()
        errs = [float(np.linalg.norm(got[f] - ref[f]) / np.linalg.norm(ref[f])) for f in range(F)]
        say(f"  member {i} {prec} K={K} F={F} n={n}: rel l2 {max(errs):.2e}")
        assert max(errs) <= eps
    g.destroy()


def test_group_graph_replays_with_eager_work_between(torch_dev):
    """Replaying the captured graphs gives the first result every time, with
    other eager work and synchronisations in between."""
    torch, dev = torch_dev
    say("case group_replays")
    data = make_inputs(8)
    plans, g = build(torch_dev)
    devin = [to_dev(torch, dev, m[0], *d) for m, d in zip(MEMBERS, data)]
    phis, thetas, coeffs = [x[1] for x in devin], [x[2] for x in devin], [x[0] for x in devin]
    outs = [torch.empty((F, max(n, 1)), dtype=c.dtype, device=dev)
            for (prec, K, F, n, eps), c in zip(MEMBERS, coeffs)]
    g.setpts(phis, thetas)
    g.exec(coeffs, outs)
    torch.cuda.synchronize()
    # members without points write nothing: compare the written columns
    ns = [m[3] for m in MEMBERS]
    first = [o[:, :n].cpu().numpy().copy() for o, n in zip(outs, ns)]
    scratch = torch.randn(1 << 20, device=dev)
    for rep in range(4):
        scratch.mul_(1.0001).add_(0.5)          # unrelated eager work
        for o in outs:
            o.zero_()
        g.setpts(phis, thetas)
        g.exec(coeffs, outs)
        torch.cuda.synchronize()
        for i, o in enumerate(outs):
            assert np.array_equal(o[:, :ns[i]].cpu().numpy(), first[i]), f"replay {rep} member {i}"
    g.destroy()


def test_group_pointer_and_count_changes(torch_dev, oracle_mod):
    """New output buffers, new coefficient buffers and new point counts are
    picked up (table rewrite, setpts graph recapture)."""
    torch, dev = torch_dev
    say("case group_changes")
    plans, g = build(torch_dev)
    for seed, scale in ((9, 1.0), (10, 0.5)):
        data = make_inputs(seed)
        if scale != 1.0:   # different point counts on the second round
            data = [(c, p[: int(len(p) * scale)], t[: int(len(t) * scale)]) for c, p, t in data]
        devin = [to_dev(torch, dev, m[0], *d) for m, d in zip(MEMBERS, data)]
        g.setpts([x[1] for x in devin], [x[2] for x in devin])
        outs = g.exec([x[0] for x in devin])
        torch.cuda.synchronize()
        for i, ((prec, K, F, n, eps), (coeffs, phi, theta)) in enumerate(zip(MEMBERS, data)):
            if len(phi) == 0:
                continue
            sel = np.arange(0, len(phi), max(1, len(phi) // 200))
            ref = oracle_mod.dfs_eval(coeffs, phi[sel], theta[sel])
            got = outs[i].cpu().numpy()[:, sel]
            err = max(float(np.linalg.norm(got[f] - ref[f]) / np.linalg.norm(ref[f])) for f in range(F))
            assert err <= 3 * eps, (seed, i, err)
    g.destroy()


def test_group_argument_errors(torch_dev):
    torch, dev = torch_dev
    from paper_2605_01313_amd import Group, Nufft2Error, Plan, nufft2
    say("case group_errors")
    p0 = Plan("fp32", 31, 31, n_fields=1, eps=1e-6)
    p1 = Plan("fp32", 31, 31, n_fields=1, eps=1e-6, stream=torch.cuda.Stream())
    with pytest.raises(Nufft2Error):
        Group([p0, p1])                      # mixed streams
    with pytest.raises(Nufft2Error):
        Group([p0, p0])                      # repeated plan
    p2 = Plan("fp32", 31, 31, n_fields=1, eps=1e-6)
    g = Group([p0, p2])
    c = torch.zeros((1, 31, 31), dtype=torch.complex64, device=dev)
    st = nufft2.nufft2_group_exec(g.handle, [c.data_ptr(), c.data_ptr()], [c.data_ptr(), c.data_ptr()])
    assert st == nufft2.NUFFT2_ERR_NO_POINTS
    phi = torch.zeros(4, dtype=torch.float64, device=dev)
    st = nufft2.nufft2_group_setpts(g.handle, [4, 4], [phi.data_ptr(), 0], [phi.data_ptr(), phi.data_ptr()])
    assert st == nufft2.NUFFT2_ERR_ARG
    g.setpts([phi, phi], [phi, phi])
    st = nufft2.nufft2_group_exec(g.handle, [c.data_ptr(), 0], [c.data_ptr(), c.data_ptr()])
    assert st == nufft2.NUFFT2_ERR_ARG
    g.destroy()


def test_large_member_emptied_and_refilled(torch_dev, oracle_mod):
    """A member with more bins than one scan pass (its gather table is written
    by the scatter, not the scan) runs with points, then without points (its
    table is not rewritten; its gather must find nothing), then with other
    points; the small member beside it is right every time."""
    torch, dev = torch_dev
    from paper_2605_01313_amd import Group, Plan
    say("case group_large_member")
    rng = np.random.default_rng(41)
    big = Plan("fp32", 1025, 1025, n_fields=1, eps=1e-6)
    small = Plan("fp32", 63, 63, n_fields=1, eps=1e-6)
    assert big.info()["n_bins"] > 8192 and small.info()["n_bins"] <= 8192
    g = Group([big, small])
    cb = synth.random_complex(rng, (1, 1025, 1025)) * synth.envelope_algebraic(1025, 1025, 1.5)[None]
    cs = synth.random_complex(rng, (1, 63, 63)) * synth.envelope_algebraic(63, 63, 1.5)[None]
    cbd = torch.from_numpy(cb).to(dev).to(torch.complex64)
    csd = torch.from_numpy(cs).to(dev).to(torch.complex64)
    for round_, nb in enumerate((40000, 0, 25000)):
        ns = 3000 + 500 * round_
        pts = [(rng.uniform(0, 2 * np.pi, n), rng.uniform(0.0, np.pi, n)) for n in (nb, ns)]
        g.setpts([torch.from_numpy(p).to(dev) for p, _ in pts], [torch.from_numpy(t).to(dev) for _, t in pts])
        outs = g.exec([cbd, csd])
        torch.cuda.synchronize()
        assert outs[0].shape == (1, nb) and outs[1].shape == (1, ns)
        for out, c, (phi, theta) in zip(outs, (cb, cs), pts):
            if len(phi) == 0:
                continue
            sel = synth.sample_indices(len(phi), 300)
            ref = oracle_mod.dfs_eval(c, phi[sel], theta[sel])
            err = float(np.linalg.norm(out.cpu().numpy()[0, sel] - ref[0]) / np.linalg.norm(ref[0]))
            say(f"  round {round_} n {len(phi)} rel l2 {err:.2e}")
            assert err <= 1e-6
    g.destroy()
    big.destroy()
    small.destroy()


def test_group_run_one_graph_equals_setpts_then_exec(torch_dev):
    """nufft2_group_run (setpts + exec in one graph launch) gives the
    outputs of the two calls bit for bit: first call, replays with eager
    work between them, a change of point counts (the combined graph is
    captured again) and the separate calls interleaved with it."""
    torch, dev = torch_dev
    say("case group_run")
    plans, g = build(torch_dev)
    for seed, scale in ((21, 1.0), (22, 1.0), (23, 0.6)):
        data = make_inputs(seed)
        if scale != 1.0:
            data = [(c, p[: int(len(p) * scale)], t[: int(len(t) * scale)]) for c, p, t in data]
        devin = [to_dev(torch, dev, m[0], *d) for m, d in zip(MEMBERS, data)]
        phis, thetas, coeffs = [x[1] for x in devin], [x[2] for x in devin], [x[0] for x in devin]
        ns = [len(d[1]) for d in data]
        g.setpts(phis, thetas)
        ref = [o.clone() for o in g.exec(coeffs)]
        torch.cuda.synchronize()
        scratch = torch.randn(1 << 20, device=dev)
        outs = [torch.empty((F, max(n, 1)), dtype=c.dtype, device=dev)
                for (prec, K, F, _, eps), c, n in zip(MEMBERS, coeffs, ns)]
        for rep in range(3):
            scratch.mul_(1.0001).add_(0.5)          # unrelated eager work
            for o in outs:
                o.zero_()
            got = g.run(phis, thetas, coeffs, outs)
            torch.cuda.synchronize()
            for i, (a, b) in enumerate(zip(got, ref)):
                assert a.shape == b.shape == (MEMBERS[i][2], ns[i])
                assert np.array_equal(a.cpu().numpy(), b.cpu().numpy()), (seed, rep, i)
            assert all(p.n_pts == n for p, n in zip(plans, ns))
    # errors leave nothing launched: a null coefficient pointer
    from paper_2605_01313_amd import nufft2
    n_pts = [p.n_pts for p in plans]
    st = nufft2.nufft2_group_run(g.handle, n_pts, [x.data_ptr() for x in phis], [x.data_ptr() for x in thetas],
                                 [0] * len(plans), [o.data_ptr() for o in outs])
    assert st == nufft2.NUFFT2_ERR_ARG
    g.destroy()


def test_group_bind_steps_with_buffers_updated_in_place(torch_dev):
    """Group.bind validates the member tensors once; each call of the bound
    step runs nufft2_group_run on them.  With new points and coefficients
    copied into the bound tensors before each step, every step gives what
    Group.run gives on the same values, bit for bit."""
    torch, dev = torch_dev
    say("case group_bind")
    plans, g = build(torch_dev)
    data = make_inputs(31)
    devin = [to_dev(torch, dev, m[0], *d) for m, d in zip(MEMBERS, data)]
    phis, thetas, coeffs = [x[1].clone() for x in devin], [x[2].clone() for x in devin], [x[0].clone() for x in devin]
    step = g.bind(phis, thetas, coeffs)
    ns = [m[3] for m in MEMBERS]
    for seed in (32, 33, 34):
        new = [to_dev(torch, dev, m[0], *d) for m, d in zip(MEMBERS, make_inputs(seed))]
        for i, x in enumerate(new):          # in place, same storage
            phis[i].copy_(x[1])
            thetas[i].copy_(x[2])
            coeffs[i].copy_(x[0])
        got = [o.clone() for o in step()]
        ref = g.run([x[1] for x in new], [x[2] for x in new], [x[0] for x in new])
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(got, ref)):
            assert a.shape == b.shape == (MEMBERS[i][2], ns[i])
            assert np.array_equal(a.cpu().numpy(), b.cpu().numpy()), (seed, i)
    g.destroy()
