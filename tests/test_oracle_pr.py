"""Pins of the oracle's partial-regularity expansion and zonal filter
(section 4: eq. pr_dfs, the conversion to eq. std_dfs, the least-squares
conditions, the zonal filter M_zf).

Every pin reaches its answer by another route than the oracle's formulas:
the basis functions of eq. pr_dfs evaluated directly as products of sines
and cosines, the paper's orthogonality conditions integrated by quadrature,
an exact rational solve built from product-to-sum identities, numpy's least
squares, and closed-form single modes for the filter.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle


def pr_factor(m, n, th):
    """The theta factor of eq. pr_dfs for column m, index n (direct)."""
    if m == 0:
        return np.cos(n * th)
    if m == 1:
        return np.sin(th) * np.cos(n * th)
    if m % 2 == 0:
        return np.sin(th) * np.sin(n * th)
    return np.sin(th) ** 2 * np.sin(n * th)


def std_factor(m, n, th):
    return np.cos(n * th) if m % 2 == 0 else np.sin(n * th)


def random_pr(rng, N, M):
    pc = np.zeros((N + 1, M + 1))
    ps = np.zeros((N + 1, M + 1))
    for m in range(M + 1):
        lo, hi = oracle.pr_range(m, N)
        pc[lo:hi + 1, m] = rng.standard_normal(hi - lo + 1)
        if m > 0:
            ps[lo:hi + 1, m] = rng.standard_normal(hi - lo + 1)
    return pc, ps


def random_std(rng, N, M):
    fc = rng.standard_normal((N + 1, M + 1))
    fs = rng.standard_normal((N + 1, M + 1))
    fs[:, 0] = 0.0
    fc[0, 1::2] = 0.0
    fs[0, 1::2] = 0.0
    return fc, fs


def eval_pr(pc, ps, phi, th):
    N, M = pc.shape[0] - 1, pc.shape[1] - 1
    out = np.zeros_like(phi)
    for m in range(M + 1):
        lo, hi = oracle.pr_range(m, N)
        for n in range(lo, hi + 1):
            b = pr_factor(m, n, th)
            out += pc[n, m] * b * np.cos(m * phi) + ps[n, m] * b * np.sin(m * phi)
    return out


def eval_std(fc, fs, phi, th):
    N, M = fc.shape[0] - 1, fc.shape[1] - 1
    out = np.zeros_like(phi)
    for m in range(M + 1):
        for n in range(N + 1):
            b = std_factor(m, n, th)
            out += fc[n, m] * b * np.cos(m * phi) + fs[n, m] * b * np.sin(m * phi)
    return out


@pytest.mark.parametrize("N,M", [(6, 5), (9, 8), (14, 11)])
def test_conversion_equals_direct_evaluation_of_the_pr_basis(N, M):
    rng = np.random.default_rng(N * 31 + M)
    pc, ps = random_pr(rng, N, M)
    fc, fs = oracle.pr_to_std(pc, ps)
    phi = rng.uniform(0, 2 * np.pi, 400)
    th = rng.uniform(-0.5, np.pi + 0.5, 400)
    want = eval_pr(pc, ps, phi, th)
    assert np.abs(eval_std(fc, fs, phi, th) - want).max() < 1e-12
    # and through the exp form and the C direct sum
    got = oracle.dfs_eval(oracle.std_to_exp(fc, fs)[None], phi, th)[0]
    assert np.abs(got.real - want).max() < 1e-12 and np.abs(got.imag).max() < 1e-12


def test_pole_values_and_the_printed_n0_entry():
    """The pr series is constant in phi at the poles (the property after
    eq. pr_dfs).  The printed even-m entry t_0 = 0 breaks this: a planted
    copy of it fails the direct evaluation."""
    rng = np.random.default_rng(3)
    N, M = 10, 8
    pc, ps = random_pr(rng, N, M)
    fc, fs = oracle.pr_to_std(pc, ps)
    phi = np.linspace(0, 2 * np.pi, 50, endpoint=False)
    for pole in (0.0, np.pi):
        v = eval_std(fc, fs, phi, np.full_like(phi, pole))
        assert np.ptp(v) < 1e-12
    printed = fc.copy()
    printed[0, 2::2] = 0.0
    th = rng.uniform(0, np.pi, 200)
    ph = rng.uniform(0, 2 * np.pi, 200)
    err = np.abs(eval_std(printed, fs, ph, th) - eval_pr(pc, ps, ph, th)).max()
    assert err > 1e-3


def _gl_on_0_pi(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return (x + 1) * np.pi / 2, w * np.pi / 2


@pytest.mark.parametrize("N,M", [(7, 6), (12, 9)])
def test_projection_meets_the_printed_conditions_by_quadrature(N, M):
    """int_0^pi (f_m - fbar_m) B_k dtheta = 0 for every k of every column,
    with f_m and B_k evaluated directly and the integral by Gauss-Legendre
    quadrature (120 nodes: the integrands are trigonometric polynomials of
    degree <= 2N + 4, integrated to rounding)."""
    rng = np.random.default_rng(N + 100 * M)
    fc, fs = random_std(rng, N, M)
    pc, ps = oracle.std_to_pr(fc, fs)
    th, w = _gl_on_0_pi(120)
    for m in range(M + 1):
        lo, hi = oracle.pr_range(m, N)
        for bar, x in ((fc, pc), (fs, ps)):
            if m == 0 and bar is fs:
                continue
            fbar = sum(bar[n, m] * std_factor(m, n, th) for n in range(N + 1))
            fpr = sum(x[n, m] * pr_factor(m, n, th) for n in range(lo, hi + 1))
            for k in range(lo, hi + 1):
                c = np.sum(w * (fpr - fbar) * pr_factor(m, k, th))
                assert abs(c) < 1e-12 * max(1.0, np.abs(bar[:, m]).max()), (m, k, c)
        # entries outside the range stay zero
        mask = np.ones(N + 1, bool)
        mask[lo:hi + 1] = False
        assert not pc[mask, m].any() and not ps[mask, m].any()


# exact route: product-to-sum identities in rationals -------------------------
def _basis_std_exact(m, j, N):
    """Standard coefficients of the pr factor (m, j) from the identities
    sin a cos b = (sin(a+b) + sin(a-b))/2, sin a sin b = (cos(a-b) - cos(a+b))/2,
    with sin(-x) = -sin x and cos(-x) = cos x; exact rationals."""
    t = [Fraction(0)] * (N + 1)
    if m == 0:
        t[j] += 1
        return t

    def add_sin(k, c):       # c sin(k theta)
        if k < 0:
            k, c = -k, -c
        if k:
            t[k] += c

    def add_cos(k, c):
        t[abs(k)] += c

    h, q = Fraction(1, 2), Fraction(1, 4)
    if m == 1:                                   # sin th cos j th
        add_sin(1 + j, h)
        add_sin(1 - j, h)
    elif m % 2 == 0:                             # sin th sin j th
        add_cos(j - 1, h)
        add_cos(j + 1, -h)
    else:                                        # (1 - cos 2th)/2 sin j th
        add_sin(j, h)
        add_sin(j + 2, -q)
        add_sin(j - 2, -q)
    return t


def _solve_exact(A, b):
    n = len(b)
    A = [row[:] + [b[i]] for i, row in enumerate(A)]
    for c in range(n):
        p = next(r for r in range(c, n) if A[r][c] != 0)
        A[c], A[p] = A[p], A[c]
        for r in range(n):
            if r != c and A[r][c] != 0:
                f = A[r][c] / A[c][c]
                A[r] = [x - f * y for x, y in zip(A[r], A[c])]
    return [A[i][n] / A[i][i] for i in range(n)]


@pytest.mark.parametrize("m", [0, 1, 2, 3, 4, 5])
def test_projection_against_an_exact_rational_solve(m):
    N = 8
    rng = np.random.default_rng(40 + m)
    b = [Fraction(int(v)) for v in rng.integers(-9, 10, N + 1)]
    if m % 2:
        b[0] = Fraction(0)
    lo, hi = oracle.pr_range(m, N)
    cols = [_basis_std_exact(m, j, N) for j in range(lo, hi + 1)]
    # weights / (pi/2): 2 for the constant cosine, 0 for sin(0), else 1
    wt = [Fraction(2) if m % 2 == 0 else Fraction(0)] + [Fraction(1)] * N
    G = [[sum(wt[i] * ci[i] * ck[i] for i in range(N + 1)) for ci in cols] for ck in cols]
    rhs = [sum(wt[i] * b[i] * ck[i] for i in range(N + 1)) for ck in cols]
    x = _solve_exact(G, rhs)
    fc = np.zeros((N + 1, 7))
    fc[:, m] = [float(v) for v in b]
    pc, _ = oracle.std_to_pr(fc, np.zeros_like(fc))
    assert np.abs(pc[lo:hi + 1, m] - np.array([float(v) for v in x])).max() < 1e-13


def test_projection_idempotent_and_minimal():
    rng = np.random.default_rng(9)
    N, M = 11, 9
    pc, ps = random_pr(rng, N, M)
    back = oracle.std_to_pr(*oracle.pr_to_std(pc, ps))
    assert np.abs(back[0] - pc).max() < 1e-12 and np.abs(back[1] - ps).max() < 1e-12
    # E_2 grows under any perturbation of the minimiser (brute force)
    fc, fs = random_std(rng, N, M)
    pc, ps = oracle.std_to_pr(fc, fs)
    th, w = _gl_on_0_pi(80)
    ph = np.linspace(0, 2 * np.pi, 2 * M + 6, endpoint=False)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    fbar = eval_std(fc, fs, PH.ravel(), TH.ravel())

    def e2(a, b):
        r = (eval_pr(a, b, PH.ravel(), TH.ravel()) - fbar).reshape(TH.shape)
        return np.sum(w[:, None] * r * r)

    best = e2(pc, ps)
    for _ in range(5):
        dc, ds = random_pr(rng, N, M)
        assert e2(pc + 1e-3 * dc, ps + 1e-3 * ds) > best


def test_exp_to_std_is_the_least_squares_inverse():
    rng = np.random.default_rng(12)
    N, M = 6, 5
    fc, fs = random_std(rng, N, M)
    gc, gs = oracle.exp_to_std(oracle.std_to_exp(fc, fs))
    assert np.abs(gc - fc).max() < 1e-14 and np.abs(gs - fs).max() < 1e-14
    # brute force: the real-linear map std -> exp as a matrix, numpy lstsq
    idx = [(n, m, part) for m in range(M + 1) for n in range(N + 1) for part in (0, 1)
           if not (part == 1 and m == 0) and not (m % 2 == 1 and n == 0)]
    cols = []
    for n, m, part in idx:
        a = np.zeros((N + 1, M + 1))
        b = np.zeros((N + 1, M + 1))
        (a if part == 0 else b)[n, m] = 1.0
        e = oracle.std_to_exp(a, b).ravel()
        cols.append(np.r_[e.real, e.imag])
    A = np.stack(cols, axis=1)
    z = rng.standard_normal((2 * N + 1, 2 * M + 1)) + 1j * rng.standard_normal((2 * N + 1, 2 * M + 1))
    sol = np.linalg.lstsq(A, np.r_[z.real.ravel(), z.imag.ravel()], rcond=None)[0]
    gc, gs = oracle.exp_to_std(z)
    for (n, m, part), v in zip(idx, sol):
        assert abs((gc if part == 0 else gs)[n, m] - v) < 1e-12


# zonal filter -----------------------------------------------------------------
def test_zonal_filter_single_modes():
    J = 64
    th, ph = oracle.grid0_nodes(J)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    lim = oracle.zonal_limit(J)
    assert lim.max() == J - 1 and lim.min() < 25         # filters near the poles only
    for m in (0, 5, 20, 21, 30, 45, 63):
        vals = np.cos(m * PH + 0.3) * (1.0 + np.cos(TH))
        got = oracle.zonal_filter(vals)
        keep = m <= lim
        want = np.where(keep[:, None], vals, 0.0)
        assert np.abs(got - want).max() < 1e-13, m
    # idempotent, linear in the field
    rng = np.random.default_rng(1)
    v = rng.standard_normal((2, J, 2 * J))
    once = oracle.zonal_filter(v)
    assert np.abs(oracle.zonal_filter(once) - once).max() < 1e-13


@pytest.mark.parametrize("M0", [0, 10, 20, 40])
def test_zonal_cutoff_decisions_are_not_borderline(M0):
    """M0 + M sin(theta_i) is never within 1e-7 of an integer for J = 16 ..
    2048 (powers of two), so any correctly rounded FP64 evaluation keeps the
    same wavenumbers; the filter's decisions are exact."""
    for lj in range(4, 12):
        J = 1 << lj
        M = J - 1
        th = (np.arange(J) + 0.5) * np.pi / J
        x = M0 + M * np.sin(th)
        x = x[x < M]
        if x.size:
            assert np.abs(x - np.rint(x)).min() > 1e-7, (J, M0)


# planted mistakes -------------------------------------------------------------
PLANTS = [
    ("t[0] = 0.5 * F(1)", "t[0] = 0.0 * F(1)"),                         # the printed n = 0 entry
    ("t[n] = 0.5 * (F(n - 1) - F(n + 1))", "t[n] = 0.5 * (F(n - 1) + F(n + 1))"),
    ("t[1] = 0.25 * (3.0 * F(1) - F(3))", "t[1] = 0.25 * (2.0 * F(1) - F(3))"),
    ("w[0] = np.pi if m % 2 == 0 else 0.0", "w[0] = np.pi / 2 if m % 2 == 0 else 0.0"),
    ("fc[n, m] = -S.imag", "fc[n, m] = S.imag"),
    ("spec[:, m[None, :] > lim[:, None]] = 0.0", "spec[:, m[None, :] >= lim[:, None]] = 0.0"),
    ("    return 1, N - 2\n", "    return 1, N - 1\n"),
]


def _all_pins_hold(o):
    """The pins above, run against module namespace o; False on any failure."""
    rng = np.random.default_rng(77)
    N, M = 9, 8
    pc = np.zeros((N + 1, M + 1))
    ps = np.zeros((N + 1, M + 1))
    for m in range(M + 1):
        lo, hi = oracle.pr_range(m, N)        # the true ranges
        pc[lo:hi + 1, m] = rng.standard_normal(hi - lo + 1)
        if m:
            ps[lo:hi + 1, m] = rng.standard_normal(hi - lo + 1)
    phi = rng.uniform(0, 2 * np.pi, 300)
    th = rng.uniform(0, np.pi, 300)
    fc, fs = o["pr_to_std"](pc, ps)
    if np.abs(eval_std(fc, fs, phi, th) - eval_pr(pc, ps, phi, th)).max() > 1e-12:
        return False
    fc, fs = random_std(rng, N, M)
    qc, qs = o["std_to_pr"](fc, fs)
    tq, wq = _gl_on_0_pi(100)
    for m in range(M + 1):
        lo, hi = oracle.pr_range(m, N)
        fbar = sum(fc[n, m] * std_factor(m, n, tq) for n in range(N + 1))
        fpr = sum(qc[n, m] * pr_factor(m, n, tq) for n in range(N + 1) if qc[n, m])
        for k in range(lo, hi + 1):
            if abs(np.sum(wq * (fpr - fbar) * pr_factor(m, k, tq))) > 1e-10:
                return False
        outside = np.ones(N + 1, bool)
        outside[lo:hi + 1] = False
        if qc[outside, m].any() or qs[outside, m].any():
            return False
    gc, gs = o["exp_to_std"](oracle.std_to_exp(fc, fs))
    if np.abs(gc - fc).max() > 1e-12 or np.abs(gs - fs).max() > 1e-12:
        return False
    J = 64
    T, P = np.meshgrid(*oracle.grid0_nodes(J), indexing="ij")
    lim = oracle.zonal_limit(J)
    for m in range(J):
        vals = np.cos(m * P) * (1.0 + np.cos(T))
        if np.abs(o["zonal_filter"](vals) - np.where((m <= lim)[:, None], vals, 0.0)).max() > 1e-12:
            return False
    return True


def test_planted_mistakes_are_caught():
    import oracle.partial_regularity as pr
    src = open(pr.__file__).read()
    clean = {}
    exec(compile(src, "pr_clean", "exec"), clean)
    assert _all_pins_hold(clean)
    for a, b in PLANTS:
        assert a in src, a
        ns = {}
        exec(compile(src.replace(a, b, 1), "pr_planted", "exec"), ns)
        assert not _all_pins_hold(ns), f"planted mistake not caught: {b}"
