#!/usr/bin/env python3
"""Throughput of the departure-point NUFFT interpolation on one MI355X.

A step is one pass of the whole path over one departure-point set: setpts
(wrap/split/sort of the points) and exec (deconvolve + pad, 2-D inverse FFT,
ES gather) for all fields.  The default workload is the 1024 x 2048 lat-lon
grid (2048 x 2048 doubled torus), 3 fields with a (1 + k^2 + l^2)^-1.5
spectrum (2047 x 2047 modes), 2,097,152 departure points of a random
8-mode stream-function wind at Courant number 8; the headline value is the
FP32 plan at eps = 1e-6 (w = 7), and the FP64 plan at eps = 1e-12 (w = 13)
is reported beside it.  Inputs are resident in HBM before the timed region
starts.  The default run adds, as extra keys: the 256 x 512 solid-body
rotation workload, the uneven ensemble, the serving loop and the kernels
around the interpolation.

Prints ONE JSON line.  `--gpus N` with N > 1 exits: the benchmark runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "departure-pt interps/s (points*fields) at eps 1e-6 FP32 vs 1e-12 FP64; p99 latency"
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6}   # dense matrix-core peaks of the MI355X
PROFILE_EVERY = 10   # timed steps per step with the dominant kernel bracketed by events
STAGES = ("setpts", "theta_pass", "phi_pass", "gather")
SINGLE_KERNEL_STAGES = ("theta_pass", "phi_pass", "gather")
# the sources each stage's kernels are built from (their hash keys the
# committed counter summaries)
KERNEL_SOURCES = {"setpts": ("setpts.hip", "nufft2_internal.hpp"),
                  "theta_pass": ("fft.hip", "nufft2_internal.hpp"),
                  "phi_pass": ("fft.hip", "nufft2_internal.hpp"),
                  "gather": ("gather_kernels.hpp", "gather.hip", "gather_f64.hip", "nufft2_internal.hpp")}
PLAN_KINDS = (("fp32", "fp32", 1e-6, True), ("fp64", "fp64", 1e-12, True),
              ("fp32_complex", "fp32", 1e-6, False), ("fp64_complex", "fp64", 1e-12, False))


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_hash(stage):
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[stage]:
        h.update(open(os.path.join(ROOT, "paper_2605_01313_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def stage_bytes(stage, info, n_touched, real_output=False):
    """Algorithmic HBM bytes of one launch of a stage (each datum moved once).
    Real-field plans read the m >= 0 half of the coefficients (K_phi/2 + 1
    columns), carry that many columns through the theta pass and write a real
    fine grid."""
    F, P = info["n_fields"], info["n_pts"]
    Kt, Kp, nfp = info["n_modes_theta"], info["n_modes_phi"], info["nf_phi"]
    cs = 8 if info["prec"] == 1 else 16
    rs = cs // 2
    herm = bool(info.get("hermitian", 0))
    cols = Kp // 2 + 1 if herm else Kp
    gs = rs if herm else cs
    rec = 16 if info["prec"] == 1 else 24
    if stage == "setpts":
        return P * (16 + rec + 4)
    if stage == "theta_pass":
        return F * Kt * cols * cs + F * n_touched * cols * cs
    if stage == "phi_pass":
        return F * n_touched * cols * cs + F * n_touched * nfp * gs
    if stage == "gather":
        return F * n_touched * nfp * gs + P * (rec + 4) + F * P * (rs if (real_output or herm) else cs)
    raise KeyError(stage)


def read_traffic(stage, workload, prec):
    """HBM bytes per launch from a committed rocprofv3 counter summary, or None
    if there is none or the kernel source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{stage}_{workload}_{prec}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != source_hash(stage):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


class Runner:
    """One plan on one workload.  hermitian: the real-field plan (the
    workloads' fields are real: their coefficients are Hermitian), real
    output; otherwise the complex plan, complex output.  The coefficients
    are held m-major ([F][K_phi][K_theta], the layout the analysis writes
    on request), so the theta pass reads whole mode columns."""

    def __init__(self, torch, wl, prec, eps, hermitian=False):
        from paper_2605_01313_amd import Plan
        self.torch = torch
        dev = torch.device("cuda:0")
        F, Kt, Kp = wl.coeffs.shape
        self.prec = prec
        self.hermitian = hermitian
        self.real_output = hermitian
        self.plan = Plan(prec, Kt, Kp, n_fields=F, eps=eps, hermitian=hermitian, m_major=True)
        cdt = torch.complex64 if prec == "fp32" else torch.complex128
        rdt = torch.float32 if prec == "fp32" else torch.float64
        self.coeffs = torch.from_numpy(wl.coeffs).to(dev).to(cdt).transpose(1, 2).contiguous()
        self.phi = torch.from_numpy(wl.phi).to(dev).contiguous()
        self.theta = torch.from_numpy(wl.theta).to(dev).contiguous()
        self.out = torch.empty((F, wl.n_pts), dtype=rdt if hermitian else cdt, device=dev)
        self.n_pf = F * wl.n_pts
        self.step()
        torch.cuda.synchronize()
        self.info = self.plan.info()
        touched = self.plan.debug_tensor(4, torch.uint8, (self.info["nf_theta"],))
        self.n_touched = int(touched.sum().item())

    def step(self):
        self.plan.setpts(self.phi, self.theta)
        self.plan.exec(self.coeffs, self.out)

    def timed(self, steps, warmup):
        torch = self.torch
        # warmup with every stage bracketed, to find the dominant kernel
        self.plan.profile(0b1111)
        for _ in range(max(warmup, 1)):
            self.step()
        prof = self.plan.profile_read()
        avg = {k: (ms / n if n else 0.0) for k, (ms, n) in prof.items()}
        # the roofline is taken for the longest single kernel: setpts is a
        # chain of two or three small kernels (bin count, scan, scatter), each
        # shorter than any of the other stages' one kernel.  The gather (the
        # per-point stage) is bracketed too, whichever kernel dominates.
        dominant = max(SINGLE_KERNEL_STAGES, key=avg.get)
        live_stages = sorted({dominant, "gather"}, key=STAGES.index)
        # timed region: the bracketed kernels get HIP events on the plan's
        # stream in every PROFILE_EVERY-th step (event records cost a few
        # microseconds; a sample keeps the timed steps close to unobserved
        # ones)
        mask = sum(1 << STAGES.index(k) for k in live_stages)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            if i % PROFILE_EVERY == 0:
                self.plan.profile(mask)
            elif i % PROFILE_EVERY == 1:
                self.plan.profile(0)
            self.step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof = self.plan.profile_read()
        live = {k: prof[k][0] / max(prof[k][1], 1) for k in live_stages}
        self.plan.profile(0)
        ms_step = (t1 - t0) * 1e3 / steps
        # per-step latency distribution (separate loop, events around each step)
        lat = []
        s = torch.cuda.current_stream()
        for _ in range(min(steps, 200)):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(s)
            self.step()
            b.record(s)
            b.synchronize()
            lat.append(a.elapsed_time(b))
        lat.sort()
        pct = lambda q: lat[min(len(lat) - 1, int(q * len(lat)))]
        # cold caches: a 1 GiB fill (past the 256 MB Infinity Cache and the
        # L2s) before each timed step; median of 10
        flush = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        cold = []
        for i in range(10):
            flush.fill_(float(i))
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(s)
            self.step()
            b.record(s)
            b.synchronize()
            cold.append(a.elapsed_time(b))
        del flush
        cold.sort()
        return {"ms_per_step": ms_step, "stage_avg_ms": avg, "dominant": dominant,
                "live_ms": live, "p50_ms": pct(0.50), "p99_ms": pct(0.99), "cold_ms": cold[len(cold) // 2]}

    def roofline(self, res, workload, tag):
        """HBM roofline of one kernel of this plan from the live events."""
        out = {}
        for k, ms in res["live_ms"].items():
            alg = stage_bytes(k, self.info, self.n_touched, self.real_output)
            achieved = alg / (ms * 1e-3) / 1e9
            out[k] = {"bound": "hbm", "kernel": k, "achieved": achieved, "peak": HBM_PEAK_GBS,
                      "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                      "traffic": read_traffic(k, workload, tag), "alg_bytes_per_launch": alg,
                      "avg_launch_ms": ms, "rows_reached": self.n_touched}
        return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, gpu_out, target_s, n_sample=None, one_core_s=5.0):
    """The oracle (FP64 direct sum) on host cores, on a bounded sample of
    points: with every thread it has, then on one core (a smaller sample).
    n_sample fixes the sample (default_rng(15) without replacement); None
    sizes it to about target_s of work.  The GPU outputs are compared with
    the oracle on the same sample."""
    import numpy as np

    import oracle
    import synth
    cores = oracle.num_threads()
    F = wl.coeffs.shape[0]
    calib = synth.sample_indices(wl.n_pts, 64, seed=99)
    t0 = time.perf_counter()
    oracle.dfs_eval(wl.coeffs, wl.phi[calib], wl.theta[calib])
    per_pt = (time.perf_counter() - t0) / calib.size
    if n_sample is None:
        n = int(min(wl.n_pts, max(256, target_s / max(per_pt, 1e-9))))
    else:
        n = int(min(wl.n_pts, n_sample))
    idx = synth.sample_indices(wl.n_pts, n, seed=15)
    t0 = time.perf_counter()
    ref = oracle.dfs_eval(wl.coeffs, wl.phi[idx], wl.theta[idx])
    dt = time.perf_counter() - t0
    errs = {}
    for name, out in gpu_out.items():
        # real-field plans return the real field: compare with the real part
        r = ref.real if not np.iscomplexobj(out) else ref
        e = [float(np.linalg.norm(out[f, idx] - r[f]) / np.linalg.norm(r[f])) for f in range(F)]
        errs[name] = {"max_over_fields": max(e), "per_field": e}
    # one core: a sample sized to about one_core_s seconds from the rate
    # just measured on every thread (one core is up to `cores` times slower)
    n1 = int(min(n, max(32, one_core_s / max(dt / n * cores, 1e-9))))
    idx1 = synth.sample_indices(wl.n_pts, n1, seed=16)
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.dfs_eval(wl.coeffs, wl.phi[idx1], wl.theta[idx1])
        dt1 = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(cores)
    return {"value": n * F / dt, "unit": "points*fields/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{n} of {wl.n_pts} points (default_rng(15) without replacement) x {F} fields "
                      f"({wl.name}), FP64 direct sum, {dt:.1f} s on {cores} threads",
            "one_core": {"value": n1 * F / dt1, "unit": "points*fields/s", "cores": 1,
                         "sample": f"{n1} points x {F} fields, {dt1:.1f} s"},
            "gpu_rel_l2_on_sample": errs}


def oracle_checks(samples):
    """Host-core leg: the oracle (FP64 direct sum) at the sampled points of
    GPU results kept by a section; worst relative l2 error over fields, per
    precision.  samples: (prec, FP64 coefficients [F][Kt][Kp], phi, theta,
    GPU values [F][n])."""
    import numpy as np

    import oracle
    worst = {}
    for prec, c, phi, theta, got in samples:
        ref = oracle.dfs_eval(c, phi, theta)
        if not np.iscomplexobj(got):
            ref = ref.real          # a real-field plan's output
        err = max(float(np.linalg.norm(got[f] - ref[f]) / np.linalg.norm(ref[f])) for f in range(ref.shape[0]))
        worst[prec] = max(worst.get(prec, 0.0), err)
    return worst


def attach_oracle_checks(section, label, check):
    """Replace a section's kept samples by the oracle's verdict on them (or
    drop them when the host-core leg is off)."""
    samples = section.pop("oracle_samples", [])
    if check:
        section[label] = {"samples": len(samples), "points_each": len(samples[0][2]) if samples else 0,
                          "max_rel_l2": oracle_checks(samples)}


def _member(spec):
    import synth
    return synth.ensemble_member(spec)


def build_members(specs):
    """Generate the members' inputs in worker processes (spawned: they import
    numpy and scipy only, never the GPU runtime)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    workers = max(1, min(16, os.cpu_count() or 1, len(specs)))
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_member, specs))


def _serving_points(job):
    """Departure points of one payload: J, wind seed, Courant number."""
    import numpy as np

    import synth
    J, seed, courant = job
    phi_a, theta_a = synth.grid0_points(J)
    wind = synth.StreamFunctionWind(np.random.default_rng(seed))
    wind.normalize_courant(phi_a, theta_a, courant, J)
    return wind.departures(phi_a, theta_a)


def serving_bench(args, torch):
    """Serving loop: Poisson arrivals (2000 requests/s by default) of requests
    with a grid drawn from 64x128 .. 512x1024, 1-3 fields, FP32 eps 1e-6 (80%)
    or FP64 eps 1e-12 (20%), each with the departure points of a random
    8-mode wind.  Payloads are pregenerated in pinned host memory and reused
    cyclically; latency runs from each request's scheduled arrival to the end
    of its device-to-host copy."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    import numpy as np

    import synth
    from paper_2605_01313_amd import Server
    Js = (64, 128, 256, 512)
    n_pts_pool, n_coef_pool = args.serve_pool, 2
    rng = np.random.default_rng(2000)
    jobs = [(J, 20000 + 100 * J + i, float(rng.uniform(2.0, 8.0))) for J in Js for i in range(n_pts_pool)]
    log(f"bench: generating {len(jobs)} departure-point payloads")
    workers = max(1, min(16, os.cpu_count() or 1))
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        pts = list(ex.map(_serving_points, jobs))
    pool = {J: {"pts": [], "c32": [], "c64": []} for J in Js}
    for (J, _, _), (phi, theta) in zip(jobs, pts):
        pool[J]["pts"].append((torch.from_numpy(phi).pin_memory(), torch.from_numpy(theta).pin_memory()))
    for J in Js:
        K = 2 * J - 1
        for i in range(n_coef_pool):
            c = synth.random_complex(np.random.default_rng(30000 + 10 * J + i), (3, K, K))
            c *= synth.envelope_algebraic(K, K, 1.5)[None]
            pool[J]["c64"].append(torch.from_numpy(c).pin_memory())
            pool[J]["c32"].append(torch.from_numpy(c).to(torch.complex64).pin_memory())
    # the request stream
    n_req = int(args.serve_rate * args.serve_seconds)
    gaps = rng.exponential(1.0 / args.serve_rate, n_req)
    arrivals = np.cumsum(gaps)
    sizes = rng.choice(Js, n_req)
    fields = rng.integers(1, 4, n_req)
    is64 = rng.random(n_req) < 0.2
    srv = Server(hbm_budget=args.serve_budget_gib << 30, max_inflight=args.serve_inflight)

    def request(i, J, F, fp64):
        c = pool[J]["c64" if fp64 else "c32"][i % n_coef_pool][:F]
        phi, theta = pool[J]["pts"][i % n_pts_pool]
        return ("fp64" if fp64 else "fp32", c, phi, theta, 1e-12 if fp64 else 1e-6)

    # 1% of the stream (every 100th request) keeps its result, to be checked
    # against the oracle on 64 sampled points and against a run of the same
    # request alone; pinned outputs allocated before the stream starts
    checked = list(range(0, n_req, 100))
    check_out = {}
    for i in checked:
        J, F, fp64 = int(sizes[i]), int(fields[i]), bool(is64[i])
        cdt = torch.complex128 if fp64 else torch.complex64
        check_out[i] = torch.empty((F, 2 * J * J), dtype=cdt).pin_memory()

    # warm-up: a burst of the largest request grows every slot's buffers,
    # then a burst of every (size, fields, precision) creates plans for the
    # concurrency the stream will need
    for k in range(args.serve_inflight):
        prec, c, phi, theta, eps = request(k, Js[-1], 3, True)
        srv.submit(prec, c, phi, theta, eps)
    srv.drain()
    copies = max(1, args.serve_inflight // 2)
    log(f"bench: serving warm-up ({copies} concurrent requests per plan key)")
    for J in Js:
        for F in (1, 2, 3):
            for fp64 in (False, True):
                for k in range(copies):
                    prec, c, phi, theta, eps = request(k, J, F, fp64)
                    srv.submit(prec, c, phi, theta, eps)
    srv.drain()
    warm = srv.stats()
    log(f"bench: serving {n_req} requests over {args.serve_seconds:.0f} s")
    t_start = srv.clock() + 0.05
    lag = 0.0
    for i in range(n_req):
        t_arr = t_start + arrivals[i]
        while True:
            now = srv.clock()
            if now >= t_arr:
                break
            if t_arr - now > 0.002:
                time.sleep(t_arr - now - 0.001)
        lag = max(lag, srv.clock() - t_arr)
        prec, c, phi, theta, eps = request(i, int(sizes[i]), int(fields[i]), bool(is64[i]))
        srv.submit(prec, c, phi, theta, eps, out=check_out.get(i), t_arrival=t_arr)
        if (i + 1) % 20000 == 0:
            log(f"bench: {i + 1} requests submitted")
    srv.drain()
    st = srv.stats()
    srv.destroy()
    # the kept results: each request run again alone on a one-slot server
    # must reproduce its in-stream result bit for bit; 64 sampled points of
    # each go to the oracle check of the host-core leg (FP64 direct sum of
    # the request's FP64 coefficients)
    log(f"bench: re-running {len(checked)} kept requests alone")
    alone = Server(hbm_budget=args.serve_budget_gib << 30, max_inflight=1)
    identical = 0
    samples = []
    for i in checked:
        J, F, fp64 = int(sizes[i]), int(fields[i]), bool(is64[i])
        prec, c, phi, theta, eps = request(i, J, F, fp64)
        got = check_out[i].numpy().copy()
        sel = synth.sample_indices(phi.numel(), 64, seed=i)
        samples.append((prec, pool[J]["c64"][i % n_coef_pool][:F].numpy(), phi.numpy()[sel],
                        theta.numpy()[sel], got[:, sel]))
        t = alone.submit(prec, c, phi, theta, eps, out=check_out[i])
        alone.wait(t)
        identical += int(np.array_equal(check_out[i].numpy(), got))
    alone.destroy()
    done = st["completed"] - warm["completed"]
    pf = st["points_fields"] - warm["points_fields"]
    span = st["last_completion"] - t_start
    offered_pf = float(sum(2 * int(J) ** 2 * int(F) for J, F in zip(sizes, fields))) / args.serve_seconds
    return {
        "value": pf / span, "unit": "points*fields/s", "requests": done, "span_s": span,
        "latency_ms": {"p50": st["latency_p50"] * 1e3, "p99": st["latency_p99"] * 1e3,
                       "max": st["latency_max"] * 1e3},
        "config": {"rate_per_s": args.serve_rate, "seconds": args.serve_seconds,
                   "grids": "64x128,128x256,256x512,512x1024", "fields": "1-3", "fp32_share": 0.8,
                   "hbm_budget_gib": args.serve_budget_gib, "max_inflight": args.serve_inflight,
                   "payload_pool_per_size": n_pts_pool},
        "time_breakdown_ms": {k: st[k] * 1e3 for k in ("queue_p50", "queue_p99", "h2d_p50", "h2d_p99",
                                                       "kernel_p50", "kernel_p99", "d2h_p50", "d2h_p99")},
        "kept_requests": {"count": len(checked), "every": 100, "identical_when_run_alone": identical},
        "oracle_samples": samples,
        "failed": st["failed"], "offered_points_fields_per_s": offered_pf,
        "submit_lag_max_ms": lag * 1e3, "plans_created": st["plans_created"],
        "plans_evicted": st["plans_evicted"], "hbm_high_water_gib": st["hbm_high_water"] / 2**30,
        "max_inflight_seen": st["max_inflight_seen"],
    }


def serving_line(args, torch):
    r = serving_bench(args, torch)
    attach_oracle_checks(r, "kept_requests_vs_oracle", not args.no_cpu_baseline)
    line = {
        "metric": METRIC, "value": r["value"], "unit": "points*fields/s", "n_gpus": 1,
        "steps": r["requests"], "warmup": 0, "ms_per_step": r["span_s"] * 1e3 / max(r["requests"], 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": dict(workload="serving_poisson_mixed_grids", step="one request: H2D, setpts, exec, D2H",
                       **r["config"]),
        "latency_ms": r["latency_ms"],
        "serving": {k: v for k, v in r.items() if k not in ("value", "unit", "latency_ms", "config")},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def ensemble_bench(args, torch, steps, warmup):
    """Uneven ensemble: 64 members on 128x256 grids + 16 on 256x512, 3 fields
    each, own seed, spectrum and 8-mode wind; FP32 eps 1e-6 real-field plans
    (the fields are real), width and tiles from the autotuner; every step is
    one group run: setpts and exec of all members as one graph launch.  Compared with the plain path on the same GPU: FP64
    eps 1e-12, one field per exec, synchronised after every exec."""
    import tempfile

    import synth
    from paper_2605_01313_amd import Group, Plan, autotune
    dev = torch.device("cuda:0")
    specs = synth.ensemble_members()
    log(f"bench: building {len(specs)} ensemble members")
    members = build_members(specs)
    F = members[0].n_fields
    cache = args.tune_cache or os.path.join(tempfile.gettempdir(), "nufft2_tune.json")
    tuned = {}
    for K in sorted({m.coeffs.shape[-1] for m in members}):
        # tiles are timed at the scale the group runs them: a group of as
        # many plans as there are members of this size, each with the first
        # such member's points
        same = [m for m in members if m.coeffs.shape[-1] == K]
        phi = torch.from_numpy(same[0].phi).to(dev)
        theta = torch.from_numpy(same[0].theta).to(dev)
        tuned[K] = autotune("fp32", K, K, F, 1e-6, phi, theta, cache_path=cache, hermitian=True,
                            members=len(same))
        log(f"bench: tuned K={K} as a group of {len(same)}: {tuned[K]}")
    plans, coeffs, phis, thetas, outs = [], [], [], [], []
    for m in members:
        K = m.coeffs.shape[-1]
        t = tuned[K]
        plans.append(Plan("fp32", K, K, n_fields=F, eps=1e-6, w=t["w"], tile_theta=t["tile_theta"],
                          tile_phi=t["tile_phi"], hermitian=True))
        coeffs.append(torch.from_numpy(m.coeffs).to(dev).to(torch.complex64).contiguous())
        phis.append(torch.from_numpy(m.phi).to(dev).contiguous())
        thetas.append(torch.from_numpy(m.theta).to(dev).contiguous())
        outs.append(torch.empty((F, m.n_pts), dtype=torch.float32, device=dev))
    g = Group(plans)
    n_pf = sum(F * m.n_pts for m in members)

    # setpts + exec of every member as one graph launch, on buffers bound
    # once (a time-stepping loop updates them in place)
    step = g.bind(phis, thetas, coeffs, outs)

    for _ in range(max(warmup, 1)):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    lat = []
    s = torch.cuda.current_stream()
    for _ in range(min(steps, 100)):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(s)
        step()
        b.record(s)
        b.synchronize()
        lat.append(a.elapsed_time(b))
    lat.sort()
    pct = lambda q: lat[min(len(lat) - 1, int(q * len(lat)))]
    log(f"bench: ensemble {ms:.3f} ms/step, {n_pf / ms * 1e3:.3e} points*fields/s")

    # plain path: one FP64 plan per grid size, one field per exec, synchronous
    plain = {}
    for m in members:
        K = m.coeffs.shape[-1]
        if K not in plain:
            plain[K] = Plan("fp64", K, K, n_fields=1, eps=1e-12)
    c64 = [torch.from_numpy(m.coeffs).to(dev).contiguous() for m in members]
    o64 = [torch.empty((1, m.n_pts), dtype=torch.complex128, device=dev) for m in members]

    def plain_step():
        for i, m in enumerate(members):
            p = plain[m.coeffs.shape[-1]]
            p.setpts(phis[i], thetas[i])
            for f in range(F):
                p.exec(c64[i][f], o64[i])
                torch.cuda.synchronize()

    plain_step()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        plain_step()
    ms64 = (time.perf_counter() - t0) * 1e3 / reps
    log(f"bench: plain FP64 path {ms64:.3f} ms/step")

    # results of a few members on 256 sampled points each, for the oracle
    # check of the host-core leg
    step()
    torch.cuda.synchronize()
    samples = []
    for i in (0, 31, 63, 64, 79):
        m = members[i]
        sel = synth.sample_indices(m.n_pts, 256, seed=20 + i)
        samples.append(("fp32", m.coeffs, m.phi[sel], m.theta[sel], outs[i].cpu().numpy()[:, sel]))
    info = g.info()
    g.destroy()
    return {
        "value": n_pf / (ms * 1e-3), "unit": "points*fields/s", "ms_per_step": ms, "steps": steps,
        "config": {"members": len(members), "points_x_fields": n_pf, "eps": 1e-6,
                   "tuned": {str(k): v for k, v in tuned.items()}, "classes": info["n_classes"],
                   "kernels_per_step": info["setpts_kernels"] + info["exec_kernels"],
                   "step": "group run: setpts + exec of all members as one graph launch (classes as parallel branches)"},
        "latency_ms": {"p50": pct(0.5), "p99": pct(0.99)},
        "plain_fp64_single_field": {"value": n_pf / (ms64 * 1e-3), "unit": "points*fields/s",
                                    "ms_per_step": ms64, "eps": 1e-12,
                                    "speedup_of_batched_fp32": ms64 / ms},
        "oracle_samples": samples,
    }


def upstream_bench(torch, prec, J=1024, F=3, reps=20):
    """The steps around the interpolation, on the 1024 x 2048 grid with 3
    fields: DFS analysis of grid values with the zonal filter (M0 = 20), the
    partial-regularity projection and synthesis (N = M = J - 1), the
    rotation of (u, v) into the arrival frame at 2,097,152 points, and the
    analysis of samples on the Gauss-Legendre grid of the same size.  Each is
    timed with HIP events on the stream it runs on; `frac` is its algorithmic
    bytes (inputs read once, outputs written once) per launch over its
    average time, against 8 TB/s, except for the Gauss-Legendre analysis,
    whose latitude product is a dense contraction priced against the MFMA
    peak of its precision."""
    import numpy as np

    import synth
    from paper_2605_01313_amd import Analysis, GLAnalysis, PartialRegularity, Plan
    dev = torch.device("cuda:0")
    rdt = torch.float32 if prec == "fp32" else torch.float64
    cdt = torch.complex64 if prec == "fp32" else torch.complex128
    rs = 4 if prec == "fp32" else 8
    cs = 2 * rs
    K, N = 2 * J - 1, J - 1
    gen = torch.Generator(device=dev)
    gen.manual_seed(3)
    vals = torch.randn((F, J, 2 * J), dtype=rdt, device=dev, generator=gen)
    an = Analysis(prec, J, n_fields=F)
    an.set_zonal_filter(20)
    coeffs = torch.empty((F, K, K), dtype=cdt, device=dev)
    pr = PartialRegularity(prec, N, N, n_fields=F)
    x = torch.empty((F, 2, N + 1, N + 1), dtype=rdt, device=dev)
    phi_a, theta_a = synth.grid0_points(J)
    rng = np.random.default_rng(4)
    P = phi_a.size
    phi_d = torch.from_numpy(phi_a + rng.uniform(-0.05, 0.05, P)).to(dev)
    theta_d = torch.from_numpy(theta_a + rng.uniform(-0.05, 0.05, P)).to(dev)
    phi_a = torch.from_numpy(phi_a).to(dev)
    theta_a = torch.from_numpy(theta_a).to(dev)
    plan = Plan(prec, K, K, n_fields=F, eps=1e-6 if prec == "fp32" else 1e-12)
    plan.setpts(phi_d, theta_d)
    out = torch.randn((F, P), dtype=cdt, device=dev, generator=gen)
    gl = GLAnalysis(prec, J, n_fields=F)
    gl_out = torch.empty((F, 2 * J + 1, K), dtype=cdt, device=dev)
    stream = torch.cuda.current_stream()

    def timeit(fn):
        for _ in range(3):
            fn()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        return sum(a.elapsed_time(b) for a, b in ev) / reps

    ops = {
        "analysis_zonal": (lambda: an.exec(vals, coeffs), F * J * 2 * J * rs + F * K * K * cs),
        "pr_project": (lambda: pr.project(coeffs, x), F * K * K * cs + F * 2 * J * J * rs),
        "pr_synthesize": (lambda: pr.synthesize(x, coeffs), F * 2 * J * J * rs + F * K * K * cs),
        "rotate_uv": (lambda: plan.rotate_uv(out, 1, 2, phi_a, theta_a), 4 * P * 8 + 4 * P * cs),
    }
    res = {}
    for name, (fn, nbytes) in ops.items():
        ms = timeit(fn)
        gbs = nbytes / (ms * 1e-3) / 1e9
        res[name] = {"ms": ms, "alg_bytes": nbytes, "achieved_gbs": gbs, "frac": gbs / HBM_PEAK_GBS}
        log(f"bench: upstream {prec} {name} {ms:.4f} ms, {gbs:.0f} GB/s")
    # Gauss-Legendre analysis: longitude FFT + the latitude product on the
    # matrix cores, 2 J^2 (4J - 2) flops per field (the two parities' J x J
    # inverses times 2(J - 1) and 2J real columns); MFMA-bound
    ms = timeit(lambda: gl.exec(vals, gl_out))
    flops = 2.0 * J * J * (4 * J - 2) * F
    peak = MFMA_PEAK_TFLOPS[prec]
    tfs = flops / (ms * 1e-3) / 1e12
    res["gl_analysis"] = {"ms": ms, "flops": flops, "achieved_tflops": tfs, "peak_tflops": peak,
                          "frac": tfs / peak, "bound": "mfma"}
    log(f"bench: upstream {prec} gl_analysis {ms:.4f} ms, {tfs:.1f} TFLOP/s")
    for o in (an, pr, plan, gl):
        o.destroy()
    return {"grid": f"{J}x{2 * J}", "n_fields": F, "n_points": P, "ops": res}


def upstream_line(args, torch):
    r = {prec: upstream_bench(torch, prec) for prec in ("fp32", "fp64")}
    ms = r["fp32"]["ops"]["analysis_zonal"]["ms"]
    line = {
        "metric": "upstream steps: analysis, pr projection / synthesis, (u, v) rotation, GL analysis",
        "value": None,
        "unit": None, "n_gpus": 1, "steps": 20, "warmup": 3, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic", "config": {"workload": "upstream_grid1024x2048_3fields"},
        "upstream": r, "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def ensemble_line(args, torch):
    r = ensemble_bench(args, torch, args.steps, args.warmup)
    attach_oracle_checks(r, "rel_l2_vs_oracle_sampled", not args.no_cpu_baseline)
    line = {
        "metric": METRIC, "value": r["value"], "unit": "points*fields/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": dict(workload="ensemble_64x128x256_16x256x512_3fields", **r["config"]),
        "latency_ms": r["latency_ms"],
        "plain_fp64_single_field": r["plain_fp64_single_field"],
        "rel_l2_vs_oracle_sampled": r.get("rel_l2_vs_oracle_sampled"),
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=("wind1024", "sbr256", "sbr256c5", "ensemble", "serving", "upstream"),
                    default="wind1024",
                    help="wind1024: 1024x2048 grid, 8-mode wind, Courant 8 (default); "
                         "sbr256: 256x512 grid, solid-body rotation (dt 1200 s); "
                         "sbr256c5: the same at dt 10125 s (Courant ~5); "
                         "ensemble: 64 + 16 members of uneven size as one group; "
                         "serving: Poisson request stream through the serving loop; "
                         "upstream: analysis, partial-regularity and rotation kernels at 1024x2048")
    ap.add_argument("--serve-rate", type=float, default=2000.0, help="requests per second")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serve-pool", type=int, default=8, help="point payloads per grid size")
    ap.add_argument("--serve-budget-gib", type=int, default=16)
    ap.add_argument("--serve-inflight", type=int, default=16)
    ap.add_argument("--no-extras", action="store_true",
                    help="default workload only: skip the ensemble, serving and upstream sections")
    ap.add_argument("--extra-serve-seconds", type=float, default=60.0,
                    help="length of the serving section of the default run")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file (ensemble)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy (counter scale for rocprofv3 --pmc)")
    ap.add_argument("--profile-plan", choices=[k[0] for k in PLAN_KINDS], default=None,
                    help="run only this plan kind of the workload and print its times (for profilers)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload == "ensemble":
        ensemble_line(args, torch)
        return
    if args.workload == "serving":
        serving_line(args, torch)
        return
    if args.workload == "upstream":
        upstream_line(args, torch)
        return
    headline = single_workload(args, torch, args.workload, args.steps, args.warmup)
    line, runners, wl = headline["line"], headline["runners"], headline["wl"]
    if args.profile_plan:
        print(json.dumps(line), flush=True)
        return
    cpu_args = None
    if not args.no_cpu_baseline:
        torch.cuda.synchronize()
        outs = {"fp32": runners[0].out.cpu().numpy().astype(np.float64),
                "fp64": runners[1].out.cpu().numpy(),
                "fp32_complex": runners[2].out.cpu().numpy().astype(np.complex128),
                "fp64_complex": runners[3].out.cpu().numpy()}
        # the 1024 x 2048 workload is sampled on 10^4 points (default_rng(15));
        # smaller ones on a sample sized to --cpu-seconds
        cpu_args = (wl, outs, args.cpu_seconds, 10000 if args.workload == "wind1024" else None)
    for r in runners:
        r.plan.destroy()
    if args.workload == "wind1024" and not args.no_extras:
        log("bench: 256x512 section")
        small = single_workload(args, torch, "sbr256", 100, 10)
        for r in small["runners"]:
            r.plan.destroy()
        line["grid256x512_sbr"] = {k: small["line"][k] for k in
                                   ("value", "unit", "ms_per_step", "config", "latency_ms", "cold_cache_ms_per_step",
                                    "stages_ms", "roofline", "gather_roofline", "fp64", "fp32_complex",
                                    "fp64_complex")}
        log("bench: 256x512 Courant-5 section")
        c5 = single_workload(args, torch, "sbr256c5", 100, 10)
        for r in c5["runners"]:
            r.plan.destroy()
        line["grid256x512_sbr_courant5"] = {k: c5["line"][k] for k in
                                            ("value", "unit", "ms_per_step", "config", "latency_ms",
                                             "cold_cache_ms_per_step", "stages_ms", "fp64")}
        log("bench: ensemble section")
        line["ensemble"] = ensemble_bench(args, torch, 20, 3)
        log("bench: serving section")
        sargs = argparse.Namespace(**vars(args))
        sargs.serve_seconds = args.extra_serve_seconds
        line["serving"] = serving_bench(sargs, torch)
        log("bench: upstream section")
        line["upstream"] = {prec: upstream_bench(torch, prec) for prec in ("fp32", "fp64")}
    if cpu_args is not None:
        log("bench: timing the oracle on host cores")
        line["cpu_baseline"] = cpu_baseline(*cpu_args)
    else:
        line["cpu_baseline"] = None
    # the sections' kept GPU results against the oracle (host-core leg)
    if "ensemble" in line:
        attach_oracle_checks(line["ensemble"], "rel_l2_vs_oracle_sampled", cpu_args is not None)
    if "serving" in line:
        attach_oracle_checks(line["serving"], "kept_requests_vs_oracle", cpu_args is not None)
    print(json.dumps(line), flush=True)


def single_workload(args, torch, which, steps, warmup):
    """One departure-point workload: the real-field FP32 plan (headline) and
    FP64 plan, and the complex plans of both precisions beside them."""
    import synth
    if which == "sbr256":
        log("bench: building the 256x512 solid-body-rotation workload")
        wl = synth.workload_sbr()
        workload = "grid256x512_sbr"
    elif which == "sbr256c5":
        # the same rotation with a time step of 10,125 s: Courant number ~5
        log("bench: building the 256x512 solid-body-rotation workload at Courant ~5")
        wl = synth.workload_sbr(dt=10125.0)
        workload = "grid256x512_sbr_courant5"
    else:
        log("bench: building the 1024x2048 8-mode-wind workload")
        wl = synth.workload_large()
        workload = "grid1024x2048_wind"
    log(f"bench: {wl.n_pts} points x {wl.n_fields} fields")
    runs = {}
    for key, prec, eps, herm in PLAN_KINDS:
        if args.profile_plan and key != args.profile_plan:
            continue
        r = Runner(torch, wl, prec, eps, hermitian=herm)
        res = r.timed(steps, warmup)
        log(f"bench: {key} {res['ms_per_step']:.4f} ms/step; stages {res['stage_avg_ms']}")
        tag = prec + ("" if herm else "_complex")
        runs[key] = (r, res, r.roofline(res, workload, tag))

    if args.copy_probe:
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("bench: copy probe 256 MiB x 5 done")
    if args.profile_plan:
        # profiling run of one plan kind: no headline line
        r, res, roof = runs[args.profile_plan]
        return {"line": {"profile_plan": args.profile_plan, "workload": workload,
                         "ms_per_step": res["ms_per_step"], "stages_ms": res["stage_avg_ms"]},
                "runners": [r], "wl": wl}

    def summary(key):
        r, res, roof = runs[key]
        return {"value": r.n_pf / (res["ms_per_step"] * 1e-3), "unit": "points*fields/s",
                "ms_per_step": res["ms_per_step"], "eps": 1e-6 if r.prec == "fp32" else 1e-12,
                "w": r.info["w"], "plan": "real-field" if r.hermitian else "complex",
                "latency_ms": {"p50": res["p50_ms"], "p99": res["p99_ms"]},
                "cold_cache_ms_per_step": res["cold_ms"],
                "stages_ms": res["stage_avg_ms"],
                "roofline": roof[res["dominant"]], "gather_roofline": roof["gather"]}

    r32, res32, roof32 = runs["fp32"]
    J = wl.J
    line = {
        "metric": METRIC, "value": r32.n_pf / (res32["ms_per_step"] * 1e-3), "unit": "points*fields/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": res32["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{workload}_{wl.n_fields}fields", "grid": f"{J}x{2*J} ({2*J}x{2*J} torus)",
                   "n_points": wl.n_pts, "n_fields": wl.n_fields, "modes": f"{2*J-1}x{2*J-1}", "eps": 1e-6,
                   "w": r32.info["w"], "nf": r32.info["nf_theta"],
                   "fields": "real (Hermitian coefficients): real-field plan, real output",
                   "coeff_layout": "m-major [F][K_phi][K_theta] (as the analysis writes it on request)",
                   "step": "setpts + exec (all fields)"},
        "latency_ms": {"p50": res32["p50_ms"], "p99": res32["p99_ms"]},
        "cold_cache_ms_per_step": res32["cold_ms"],
        "stages_ms": res32["stage_avg_ms"],
        "roofline": roof32[res32["dominant"]],
        "gather_roofline": roof32["gather"],
        "fp64": summary("fp64"),
        "fp32_complex": summary("fp32_complex"),
        "fp64_complex": summary("fp64_complex"),
    }
    runners = [runs[k][0] for k in ("fp32", "fp64", "fp32_complex", "fp64_complex")]
    return {"line": line, "runners": runners, "wl": wl}


if __name__ == "__main__":
    main()
