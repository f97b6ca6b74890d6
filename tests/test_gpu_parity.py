"""HIP path against the FP64 oracle and against numpy restatements of each stage.

Tolerances: FP64 plans at eps = 1e-12 must reach relative l2 <= 1e-12 per
field; FP32 plans at eps = 1e-6 must reach <= 1e-6 (both as the method
defines eps: relative l2 over the evaluated points).
"""
import ctypes
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


def run_plan(torch_dev, prec, coeffs, phi, theta, eps, **kw):
    torch, dev = torch_dev
    from paper_2605_01313_amd import Plan
    F, Kt, Kp = coeffs.shape
    plan = Plan(prec, Kt, Kp, n_fields=F, eps=eps, **kw)
    cdt = np.complex64 if prec == "fp32" else np.complex128
    plan.setpts(torch.from_numpy(np.ascontiguousarray(phi)).to(dev),
                torch.from_numpy(np.ascontiguousarray(theta)).to(dev))
    out = plan.exec(torch.from_numpy(coeffs.astype(cdt)).to(dev))
    torch.cuda.synchronize()
    return plan, out.cpu().numpy()


def field_errors(got, ref):
    return [rel_l2(got[f], ref[f]) for f in range(ref.shape[0])]


# --------------------------------------------------------------------------
# End to end on the small workload (32 x 64 grid, 2048 jittered points)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("prec,eps,tol", [("fp64", 1e-12, 1e-12), ("fp32", 1e-6, 1e-6)])
def test_small_workload_full(torch_dev, oracle_mod, prec, eps, tol):
    wl = synth.workload_small_jitter()
    say(f"case small_workload prec={prec} P={wl.n_pts}")
    plan, got = run_plan(torch_dev, prec, wl.coeffs, wl.phi, wl.theta, eps)
    assert plan.check() == 0
    ref = oracle_mod.dfs_eval(wl.coeffs, wl.phi, wl.theta)
    errs = field_errors(got, ref)
    say(f"  rel l2 {errs}")
    assert max(errs) <= tol


# --------------------------------------------------------------------------
# Stage checks
# --------------------------------------------------------------------------
def test_setpts_records_and_sort(torch_dev):
    """Bin counts, starts and permutation form a valid counting sort; each
    record's cell index equals the FP64 split done here in numpy."""
    torch, dev = torch_dev
    wl = synth.workload_small_jitter()
    rng = np.random.default_rng(2)
    phi = np.concatenate([wl.phi, rng.uniform(-20, 20, 300), [0.0, 2 * np.pi, -1e-18, 6.283185307179586]])
    theta = np.concatenate([wl.theta, rng.uniform(-20, 20, 300), [0.0, 2 * np.pi, 1e-300, -np.pi]])
    say(f"case setpts_sort P={phi.size}")
    coeffs = wl.coeffs
    plan, _ = run_plan(torch_dev, "fp64", coeffs, phi, theta, 1e-12)
    info = plan.info()
    P, nb = phi.size, info["n_bins"]
    perm = plan.debug_tensor(2, torch.int32, (P,)).cpu().numpy()
    starts_all = plan.debug_tensor(3, torch.int32, (nb + 1,)).cpu().numpy()
    counts = np.diff(starts_all)
    starts = starts_all[:-1]
    recs = plan.debug_tensor(1, torch.float64, (P, 3)).cpu().numpy()  # {int32,int32}, vt, vp
    idx = recs[:, 0].copy().view(np.int32).reshape(P, 2)
    assert np.array_equal(np.sort(perm), np.arange(P))
    assert counts.sum() == P and starts_all[0] == 0 and starts_all[-1] == P
    assert np.all(counts >= 0)
    w, nft, nfp = info["w"], info["nf_theta"], info["nf_phi"]

    def split(x, nf):
        t = x * (nf / (2 * np.pi))
        t = t - nf * np.floor(t / nf)
        t = np.where(t >= nf, t - nf, t)
        c = np.ceil(t - 0.5 * w)
        return (c.astype(np.int64) % nf), (t - c) - (w // 2)

    it, vt = split(theta[perm], nft)
    ip, vp = split(phi[perm], nfp)
    assert np.array_equal(idx[:, 0], it)
    assert np.array_equal(idx[:, 1], ip)
    assert np.array_equal(recs[:, 1], vt)
    assert np.array_equal(recs[:, 2], vp)
    tt, tp = info["tile_theta"], info["tile_phi"]
    bins = (it // tt) * (nfp // tp) + ip // tp
    assert np.all(np.diff(bins) >= 0)
    for b in np.unique(bins)[:50]:
        assert counts[b] == np.sum(bins == b)
    assert np.all(np.abs(vt) <= 1.0) and np.all(np.abs(vp) <= 1.0)
    touched = plan.debug_tensor(4, torch.uint8, (nft,)).cpu().numpy()
    want = np.zeros(nft, np.uint8)
    for a in range(w):
        want[(it + a) % nft] = 1
    assert np.array_equal(touched, want)
    check_binlist(plan, torch, starts_all)


def check_binlist(plan, torch, starts_all):
    """The compacted list of non-empty bins equals the bins with a record."""
    nb = starts_all.size - 1
    binlist = plan.debug_tensor(6, torch.int32, (nb + 1,)).cpu().numpy()
    nonempty = np.flatnonzero(np.diff(starts_all) > 0)
    assert binlist[nb] == nonempty.size
    assert np.array_equal(binlist[:nonempty.size], nonempty)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fft_stage_matches_numpy(torch_dev, prec):
    """Fine grid on reached rows == ifft2 of the deconvolved, zero-padded coefficients."""
    torch, dev = torch_dev
    from paper_2605_01313_amd import nufft2
    rng = np.random.default_rng(21)
    Kt, Kp = 45, 61
    F = 2
    coeffs = synth.random_complex(rng, (F, Kt, Kp))
    phi = rng.uniform(0, 2 * np.pi, 500)
    theta = rng.uniform(0.3, 2.0, 500)
    say(f"case fft_stage prec={prec} K=({Kt},{Kp})")
    eps = 1e-12 if prec == "fp64" else 1e-6
    plan, _ = run_plan(torch_dev, prec, coeffs, phi, theta, eps)
    info = plan.info()
    nft, nfp, w, beta = info["nf_theta"], info["nf_phi"], info["w"], info["beta"]
    cdt = torch.complex128 if prec == "fp64" else torch.complex64
    grid = plan.debug_tensor(0, cdt, (F, nft, nfp)).cpu().numpy()
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
        ref = np.fft.ifft2(G) * nft * nfp
        err = rel_l2(grid[f][touched], ref[touched])
        say(f"  field {f} grid rel l2 {err:.2e}")
        assert err < tol


# --------------------------------------------------------------------------
# Moderate resolution (256 x 512, solid-body rotation), sampled points
# --------------------------------------------------------------------------
@pytest.mark.parametrize("prec,eps,tol", [("fp64", 1e-12, 1e-12), ("fp32", 1e-6, 1e-6)])
def test_sbr_workload_full(torch_dev, sbr_full_ref, prec, eps, tol):
    """Every one of the 131,072 points of the 256 x 512 workload, 3 fields."""
    wl, ref = sbr_full_ref
    say(f"case sbr prec={prec} P={wl.n_pts} F={wl.n_fields} (all points)")
    plan, got = run_plan(torch_dev, prec, wl.coeffs, wl.phi, wl.theta, eps)
    assert plan.check() == 0
    errs = field_errors(got, ref)
    say(f"  rel l2 per field {errs}")
    assert max(errs) <= tol


# --------------------------------------------------------------------------
# Shapes and edge cases
# --------------------------------------------------------------------------
@pytest.mark.parametrize("Kt,Kp,P,F", [(7, 9, 1, 1), (16, 10, 37, 2), (63, 33, 1000, 3),
                                       (100, 257, 4097, 1), (255, 255, 3000, 2)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_ragged_shapes(torch_dev, oracle_mod, Kt, Kp, P, F, prec):
    rng = np.random.default_rng(Kt * 1000 + Kp + P)
    coeffs = synth.random_complex(rng, (F, Kt, Kp))
    phi = rng.uniform(-7, 14, P)
    theta = rng.uniform(-7, 14, P)
    say(f"case ragged K=({Kt},{Kp}) P={P} F={F} prec={prec}")
    # Unstructured random coefficients have a white spectrum, the hardest case
    # for the kernel: at sigma = 2 the width rule realises about 2 eps there
    # (1.5e-12 .. 2.3e-12 at w = 13, 1.1e-6 .. 1.4e-6 at w = 7), while the
    # decaying spectra of the workloads meet eps itself.
    eps, tol = (1e-12, 3e-12) if prec == "fp64" else (1e-6, 3e-6)
    plan, got = run_plan(torch_dev, prec, coeffs, phi, theta, eps)
    ref = oracle_mod.dfs_eval(coeffs, phi, theta)
    errs = field_errors(got, ref)
    say(f"  rel l2 {errs}")
    assert max(errs) <= tol


@pytest.mark.parametrize("eps", [1e-5, 1e-6, 1e-8, 1e-10, 1e-13, 1e-14])
def test_fp64_widths_across_the_weight_polynomial_threshold(torch_dev, oracle_mod, eps):
    """FP64 plans of width 6 (every weight evaluated directly) through 15
    (interior tap weights from degree-14 polynomials, edge taps direct) meet
    the header's contract for a white spectrum: within 2.5 eps at eps >=
    1e-12 (3 eps asserted, as in the other white-spectrum cases) and 3.5 eps
    below, where the ratio grows with the width (2.8 at w = 14, 3.35 at
    w = 15, with direct or polynomial weights alike)."""
    rng = np.random.default_rng(int(-np.log10(eps)) + 500)
    coeffs = synth.random_complex(rng, (2, 63, 63))
    phi = rng.uniform(-7, 14, 3000)
    theta = rng.uniform(-7, 14, 3000)
    plan, got = run_plan(torch_dev, "fp64", coeffs, phi, theta, eps)
    w = plan.info()["w"]
    say(f"case fp64 eps={eps:g} w={w}")
    errs = field_errors(got, oracle_mod.dfs_eval(coeffs, phi, theta))
    say(f"  rel l2 {errs}")
    assert w == int(np.ceil(-np.log10(eps) - 1e-9)) + 1
    assert max(errs) <= (3 if eps >= 1e-12 else 3.5) * eps
    plan.destroy()


def test_white_spectrum_meets_1e12_one_width_up(torch_dev, oracle_mod):
    """Asking for eps = 1e-13 (w = 14) brings a white spectrum under 1e-12."""
    rng = np.random.default_rng(77)
    coeffs = synth.random_complex(rng, (2, 127, 127))
    phi = rng.uniform(-7, 14, 3000)
    theta = rng.uniform(-7, 14, 3000)
    say("case white_spectrum_w14")
    plan, got = run_plan(torch_dev, "fp64", coeffs, phi, theta, 1e-13)
    assert plan.info()["w"] == 14
    errs = field_errors(got, oracle_mod.dfs_eval(coeffs, phi, theta))
    say(f"  rel l2 {errs}")
    assert max(errs) <= 1e-12


@pytest.mark.parametrize("prec,eps,tol", [("fp64", 1e-12, 3e-12), ("fp32", 1e-6, 3e-6)])
def test_largest_grid(torch_dev, oracle_mod, prec, eps, tol):
    """The 4096 x 4096 fine grid (K = 2047): plan limits hold in both precisions."""
    rng = np.random.default_rng(4096)
    K = 2047
    coeffs = synth.random_complex(rng, (2, K, K)) * synth.envelope_algebraic(K, K, 1.0)[None]
    phi = rng.uniform(0, 2 * np.pi, 600)
    theta = rng.uniform(-0.2, np.pi + 0.2, 600)
    say(f"case largest_grid prec={prec}")
    plan, got = run_plan(torch_dev, prec, coeffs, phi, theta, eps)
    info = plan.info()
    assert info["nf_theta"] == 4096 and plan.check() == 0
    torch = torch_dev[0]
    # more bins than one pass of the scan workgroup
    assert info["n_bins"] > 8192
    check_binlist(plan, torch, plan.debug_tensor(3, torch.int32, (info["n_bins"] + 1,)).cpu().numpy())
    errs = field_errors(got, oracle_mod.dfs_eval(coeffs, phi, theta))
    say(f"  rel l2 {errs}")
    assert max(errs) <= tol


@pytest.mark.parametrize("prec,eps,tol", [("fp32", 1e-6, 1e-6), ("fp64", 1e-12, 1e-12)])
def test_wind_1024x2048_full_size_sampled(torch_dev, wind_large_ref, prec, eps, tol):
    """The 1024 x 2048 workload at full size (2,097,152 wind departure points,
    K = 2047, 3 fields, algebraically decaying spectra) in the default plan
    configuration the bench times (side-by-side scan passes, 2048 x 2048
    theta/phi transforms, 16 x 32 gather tiles): the 10^4 outputs per field
    that default_rng(15) samples, against the oracle."""
    wl, sel, ref = wind_large_ref
    say(f"case wind1024 full size prec={prec}")
    plan, got = run_plan(torch_dev, prec, wl.coeffs, wl.phi, wl.theta, eps)
    info = plan.info()
    assert plan.check() == 0 and info["n_pts"] == wl.n_pts and info["n_bins"] > 8192
    errs = field_errors(got[:, sel], ref)
    say(f"  rel l2 {errs}")
    assert max(errs) <= tol
    plan.destroy()


@pytest.mark.parametrize("tt,tp", [(16, 16), (32, 64), (128, 16)])
def test_fp64_gather_tile_shapes(torch_dev, oracle_mod, tt, tp):
    """FP64 gather patches with padded LDS rows (16 x 16: 28 -> 32 elements;
    32 x 64: 76 -> 80) and with unpadded ones where the padded patch of a
    field would pass the LDS limit (128 x 16: 140 rows of 28, not of 32), on
    three fields and points around the whole torus."""
    rng = np.random.default_rng(1000 + tt + tp)
    K = 255
    coeffs = synth.random_complex(rng, (3, K, K)) * synth.envelope_algebraic(K, K, 1.5)[None]
    phi = rng.uniform(-1.0, 7.0, 3000)
    theta = rng.uniform(-0.5, 2 * np.pi + 0.5, 3000)
    say(f"case fp64_tiles tt={tt} tp={tp}")
    plan, got = run_plan(torch_dev, "fp64", coeffs, phi, theta, 1e-12, tile_theta=tt, tile_phi=tp)
    info = plan.info()
    assert (info["tile_theta"], info["tile_phi"]) == (tt, tp) and plan.check() == 0
    sel = synth.sample_indices(len(phi), 400)
    errs = field_errors(got[:, sel], oracle_mod.dfs_eval(coeffs, phi[sel], theta[sel]))
    say(f"  rel l2 {errs}")
    assert max(errs) <= 1e-12
    plan.destroy()


def test_setpts_paths_alternate_on_one_plan(torch_dev, oracle_mod):
    """Point counts on both sides of the limit of the fused sort (at most 256
    workgroups of 1024 points; above it the separate scan kernel runs) on one
    plan, one after another: each leaves the counters, row marks and ticket
    cleared for the next, so every call sorts and evaluates correctly."""
    torch, dev = torch_dev
    from paper_2605_01313_amd import Plan
    rng = np.random.default_rng(31)
    K = 63
    coeffs = synth.dfs_field_coeffs(rng, K, K, synth.envelope_algebraic(K, K))[None]
    plan = Plan("fp32", K, K, n_fields=1, eps=1e-6)
    c = torch.from_numpy(coeffs.astype(np.complex64)).to(dev)
    info = plan.info()
    nb = info["n_bins"]
    for n in (262144, 262145, 5000, 262144, 1):
        say(f"case setpts_paths n={n}")
        phi = rng.uniform(-7.0, 7.0, n)
        theta = rng.uniform(0.05, 3.1, n)
        plan.setpts(torch.from_numpy(phi).to(dev), torch.from_numpy(theta).to(dev))
        got = plan.exec(c).cpu().numpy()
        assert plan.check() == 0
        perm = plan.debug_tensor(2, torch.int32, (n,)).cpu().numpy()
        assert np.array_equal(np.sort(perm), np.arange(n))
        starts_all = plan.debug_tensor(3, torch.int32, (nb + 1,)).cpu().numpy()
        assert starts_all[0] == 0 and starts_all[-1] == n and np.all(np.diff(starts_all) >= 0)
        check_binlist(plan, torch, starts_all)
        sel = synth.sample_indices(n, 300)
        ref = oracle_mod.dfs_eval(coeffs, phi[sel], theta[sel])
        err = rel_l2(got[0, sel], ref[0])
        say(f"  rel l2 {err:.2e}")
        assert err <= 1e-6
    plan.destroy()


def test_scan_passes_side_by_side_on_a_large_plan(torch_dev, oracle_mod):
    """A plan of four scan passes (32768 bins): point sets with points use
    the side-by-side passes, an empty one the one-workgroup scan; each call
    leaves the counters cleared, so every sort is valid and every result
    meets the oracle."""
    torch, dev = torch_dev
    from paper_2605_01313_amd import Plan
    rng = np.random.default_rng(43)
    K = 1025
    coeffs = (synth.random_complex(rng, (1, K, K)) * synth.envelope_algebraic(K, K, 1.5)[None])
    plan = Plan("fp32", K, K, n_fields=1, eps=1e-6)
    info = plan.info()
    nb = info["n_bins"]
    assert nb > 3 * 8192
    c = torch.from_numpy(coeffs.astype(np.complex64)).to(dev)
    for n in (50000, 0, 30000, 300000):
        say(f"case scan_passes n={n}")
        phi = rng.uniform(-1.0, 7.0, n)
        theta = rng.uniform(0.0, np.pi, n)
        plan.setpts(torch.from_numpy(phi).to(dev), torch.from_numpy(theta).to(dev))
        got = plan.exec(c).cpu().numpy()
        assert plan.check() == 0
        starts_all = plan.debug_tensor(3, torch.int32, (nb + 1,)).cpu().numpy()
        assert starts_all[0] == 0 and starts_all[-1] == n and np.all(np.diff(starts_all) >= 0)
        check_binlist(plan, torch, starts_all)
        if n == 0:
            continue
        perm = plan.debug_tensor(2, torch.int32, (n,)).cpu().numpy()
        assert np.array_equal(np.sort(perm), np.arange(n))
        sel = synth.sample_indices(n, 200)
        ref = oracle_mod.dfs_eval(coeffs, phi[sel], theta[sel])
        err = rel_l2(got[0, sel], ref[0])
        say(f"  rel l2 {err:.2e}")
        assert err <= 1e-6
    plan.destroy()


def test_zero_points_and_exec_before_setpts(torch_dev):
    torch, dev = torch_dev
    from paper_2605_01313_amd import Plan, nufft2
    say("case zero_points")
    plan = Plan("fp64", 31, 31, n_fields=1, eps=1e-12)
    c = torch.zeros((1, 31, 31), dtype=torch.complex128, device=dev)
    st = nufft2.nufft2_exec(plan.handle, c.data_ptr(), c.data_ptr())
    assert st == nufft2.NUFFT2_ERR_NO_POINTS
    e = torch.empty(0, dtype=torch.float64, device=dev)
    plan.setpts(e, e)
    out = plan.exec(c)
    assert out.shape == (1, 0)
    assert plan.check() == 0


def test_binding_rejects_a_wrong_output_tensor(torch_dev):
    """The binding checks the caller's output tensor before the library
    writes F * n_pts values into it."""
    torch, dev = torch_dev
    from paper_2605_01313_amd import Plan
    say("case wrong_out")
    plan = Plan("fp32", 31, 31, n_fields=2, eps=1e-6)
    pts = torch.linspace(0.1, 3.0, 100, dtype=torch.float64, device=dev)
    plan.setpts(pts, pts)
    c = torch.zeros((2, 31, 31), dtype=torch.complex64, device=dev)
    for bad in (torch.empty((2, 99), dtype=torch.complex64, device=dev),
                torch.empty((2, 100), dtype=torch.complex128, device=dev),
                torch.empty((100, 2), dtype=torch.complex64, device=dev).t(),
                torch.empty((2, 100), dtype=torch.complex64)):
        with pytest.raises(ValueError):
            plan.exec(c, bad)
    assert plan.exec(c, torch.empty((2, 100), dtype=torch.complex64, device=dev)).shape == (2, 100)
    # rotate_uv rewrites two fields of the caller's output in place
    for bad in (torch.empty((2, 99), dtype=torch.complex64, device=dev),
                torch.empty((2, 100), dtype=torch.float32, device=dev)):
        with pytest.raises(ValueError):
            plan.rotate_uv(bad, 0, 1, pts, pts)
    plan.destroy()


def test_group_binding_rejects_a_wrong_output_tensor(torch_dev):
    """Group.exec checks every member's output tensor (dtype, device,
    contiguity, size, real or complex) before the group launch writes it."""
    torch, dev = torch_dev
    from paper_2605_01313_amd import Group, Plan
    say("case group_wrong_out")
    plans = [Plan("fp32", 31, 31, n_fields=2, eps=1e-6),
             Plan("fp32", 15, 15, n_fields=1, eps=1e-6, real_output=True)]
    g = Group(plans)
    pts = [torch.linspace(0.1, 3.0, n, dtype=torch.float64, device=dev) for n in (100, 50)]
    g.setpts(pts, pts)
    cs = [torch.zeros((2, 31, 31), dtype=torch.complex64, device=dev),
          torch.zeros((1, 15, 15), dtype=torch.complex64, device=dev)]
    good = [torch.empty((2, 100), dtype=torch.complex64, device=dev),
            torch.empty((1, 50), dtype=torch.float32, device=dev)]
    bads = [[torch.empty((2, 99), dtype=torch.complex64, device=dev), good[1]],
            [good[0], torch.empty((1, 50), dtype=torch.complex64, device=dev)],
            [good[0], torch.empty((1, 49), dtype=torch.float32, device=dev)],
            [torch.empty((100, 2), dtype=torch.complex64, device=dev).t(), good[1]],
            [good[0], torch.empty((1, 50), dtype=torch.float32)],
            [good[0]]]
    for bad in bads:
        with pytest.raises(ValueError):
            g.exec(cs, bad)
    with pytest.raises(TypeError):
        g.exec([cs[0], cs[1].to(torch.complex128)], good)
    outs = g.exec(cs, good)
    torch.cuda.synchronize()
    assert outs[0].shape == (2, 100) and outs[1].shape == (1, 50)
    g.destroy()
    for p in plans:
        p.destroy()


def test_nonfinite_points_give_nan_and_flag(torch_dev):
    torch, dev = torch_dev
    say("case nonfinite")
    rng = np.random.default_rng(8)
    coeffs = synth.random_complex(rng, (2, 15, 15))
    phi = rng.uniform(0, 6, 100)
    theta = rng.uniform(0, 3, 100)
    phi[[3, 50]] = [np.nan, np.inf]
    theta[77] = -np.inf
    plan, got = run_plan(torch_dev, "fp64", coeffs, phi, theta, 1e-12)
    bad = np.zeros(100, bool)
    bad[[3, 50, 77]] = True
    assert np.all(np.isnan(got[:, bad]))
    assert np.all(np.isfinite(got[:, ~bad]))
    assert plan.check() == 5        # NUFFT2_ERR_NONFINITE
    good = np.where(~bad)[0]
    import oracle
    ref = oracle.dfs_eval(coeffs, phi[good], theta[good])
    assert max(field_errors(got[:, good], ref)) <= 3e-12     # white spectrum, see above
    # resetting to finite points clears the flag
    torch_, _ = torch_dev
    plan.setpts(torch_.from_numpy(np.zeros(5)).to(dev), torch_.from_numpy(np.zeros(5)).to(dev))
    assert plan.check() == 0


@pytest.mark.parametrize("prec,eps,tol", [("fp32", 1e-6, 3e-6), ("fp64", 1e-12, 3e-12)])
def test_nonfinite_points_on_a_large_plan(torch_dev, oracle_mod, prec, eps, tol):
    """Non-finite coordinates on a plan whose scan passes run side by side
    (K = 1025, more than 8192 bins): NaN outputs, the flag from check(), the
    other points meet the oracle, and the next setpts with finite points
    (through the same passes) clears the flag."""
    torch, dev = torch_dev
    rng = np.random.default_rng(81)
    K, n = 1025, 40000
    coeffs = synth.random_complex(rng, (2, K, K))
    phi = rng.uniform(-1.0, 7.0, n)
    theta = rng.uniform(-0.3, np.pi + 0.3, n)
    bad_idx = [0, 17, 20000, n - 1]
    phi[bad_idx[:2]] = [np.nan, -np.inf]
    theta[bad_idx[2:]] = [np.inf, np.nan]
    say(f"case nonfinite large plan prec={prec}")
    plan, got = run_plan(torch_dev, prec, coeffs, phi, theta, eps)
    assert plan.info()["n_bins"] > 8192
    bad = np.zeros(n, bool)
    bad[bad_idx] = True
    assert np.all(np.isnan(got[:, bad])) and np.all(np.isfinite(got[:, ~bad]))
    assert plan.check() == 5        # NUFFT2_ERR_NONFINITE
    sel = np.where(~bad)[0][synth.sample_indices(n - len(bad_idx), 300)]
    errs = field_errors(got[:, sel], oracle_mod.dfs_eval(coeffs, phi[sel], theta[sel]))
    say(f"  rel l2 {errs}")
    assert max(errs) <= tol         # white spectrum: 3 eps
    phi2 = rng.uniform(0.0, 6.0, 30000)
    theta2 = rng.uniform(0.0, 3.0, 30000)
    plan.setpts(torch.from_numpy(phi2).to(dev), torch.from_numpy(theta2).to(dev))
    assert plan.check() == 0
    plan.destroy()


def test_repeatable_and_fieldwise(torch_dev, oracle_mod):
    """Two execs give identical bits; multi-field equals fields run one by one."""
    torch, dev = torch_dev
    say("case repeatable")
    rng = np.random.default_rng(31)
    coeffs = synth.random_complex(rng, (3, 63, 63))
    phi = rng.uniform(0, 2 * np.pi, 5000)
    theta = rng.uniform(0, np.pi, 5000)
    plan, a = run_plan(torch_dev, "fp32", coeffs, phi, theta, 1e-6)
    b = plan.exec(torch.from_numpy(coeffs.astype(np.complex64)).to(dev)).cpu().numpy()
    assert np.array_equal(a, b)
    for f in range(3):
        _, one = run_plan(torch_dev, "fp32", coeffs[f:f + 1], phi, theta, 1e-6)
        assert np.array_equal(one[0], a[f])


def test_real_output_is_real_part(torch_dev):
    torch, dev = torch_dev
    say("case real_output")
    wl = synth.workload_small_jitter()
    _, full = run_plan(torch_dev, "fp64", wl.coeffs, wl.phi, wl.theta, 1e-12)
    _, re = run_plan(torch_dev, "fp64", wl.coeffs, wl.phi, wl.theta, 1e-12, real_output=True)
    assert re.dtype == np.float64
    assert np.array_equal(re, full.real)


def test_width_convergence(torch_dev, oracle_mod):
    """Error falls roughly tenfold per unit of kernel width (ES kernel rule)."""
    say("case width_convergence")
    rng = np.random.default_rng(40)
    K = 63
    coeffs = synth.dfs_field_coeffs(rng, K, K, synth.envelope_algebraic(K, K, 1.5))[None]
    phi = rng.uniform(0, 2 * np.pi, 2000)
    theta = rng.uniform(0, np.pi, 2000)
    ref = oracle_mod.dfs_eval(coeffs, phi, theta)
    errs = []
    for w in (4, 6, 8, 10, 12):
        _, got = run_plan(torch_dev, "fp64", coeffs, phi, theta, 1e-12, w=w)
        errs.append(rel_l2(got[0], ref[0]))
    say(f"  errors by w: {errs}")
    for e0, e1 in zip(errs, errs[1:]):
        assert e1 < e0 / 20       # two units of width: at least ~20x


def test_shift_theorem(torch_dev):
    """Shifting all points by d in phi equals multiplying F[n,m] by e^{i m d}."""
    torch, dev = torch_dev
    say("case shift_theorem")
    rng = np.random.default_rng(41)
    K = 41
    coeffs = synth.random_complex(rng, (1, K, K))
    phi = rng.uniform(0, 2 * np.pi, 800)
    theta = rng.uniform(0, np.pi, 800)
    d = 0.3
    m = np.arange(K) - K // 2
    _, a = run_plan(torch_dev, "fp64", coeffs, phi + d, theta, 1e-12)
    _, b = run_plan(torch_dev, "fp64", coeffs * np.exp(1j * m * d)[None, None, :], phi, theta, 1e-12)
    assert rel_l2(a, b) < 2e-12
