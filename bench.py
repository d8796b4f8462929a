"""Benchmark: lattice site-updates/s of the hybrid LB/EPD step on one MI355X.

A "step" is one hybrid step on the resident state: advection and EPD update,
densities (chain propagators, or the convolutional surrogate between exact
steps), force reconstruction and the D2Q9 LB step.

    python bench.py [--steps K] [--warmup W] [--workload cfg5q|cfg2|cfg3|cfg4|cfg5]

Default workload (cfg5q), plain versus surrogate: 512 x 512 periodic grid,
FP32 fields with FP64 partition-function reductions, N = 32, f_A = 0.5,
phi_P = 0.1, chi reading Q, g = 1e-5 f*, seeded Gaussian noise sigma = 0.05
(seed 1005).  Each path runs the workload's 2e4 steps from the seed.  Inside
that run a window of exactly K steps is timed with HIP events on the
context's stream, bracketed by stream synchronisations; it starts at an
exact (fallback) step at least W steps into the run, as late as the run
allows, so that it holds ceil(K/50) exact steps.  `value` is the surrogate
path's rate over that window, `plain.value` the plain path's over the same
window, `speedup` their ratio, and `whole_run` the rates over all 2e4 steps
(the surrogate's gated start-up included).  The surrogate's exact steps
(every 50 steps, on the residual test, and while the last measured network
error exceeds 9e-4) are inside every timed figure.

`roofline` is that of the kernel family with the largest share of the
surrogate path's GPU time (the 64 -> 64 convolution, MFMA-bound): useful
flops per launch over the mean launch duration, each launch timed by HIP
events at its own start and end in 100 steps that continue the run.
`plain_full_scale` adds the plain path on 1024 x 512, N = 64 with the HBM
roofline of its dominant kernel family; `fluid3d` and `densities3d` the
three-dimensional D3Q19 fluid (256^3, FP32) and the three-dimensional
propagators and densities (256^3, N = 32, FP32), each with its roofline;
`sync_costs` the launch and device-wide barrier costs the step's design
rests on, and `conv_floor` the matrix-work, store and combined ceilings of
one 64 -> 64 layer at 512^2 (separate probe processes).

`cpu_baseline` is the FP64 NumPy oracle's plain step of the same workload on
the host: one process (one thread), and one single-threaded process per
available core up to 16 running side by side, each for a bounded time.

`--workload cfg2|cfg3|cfg5|cfg4` prints a plain-path line instead: W steps
after the seed, then K timed steps.  Prints ONE JSON line.
"""
import argparse
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "lattice site-updates/s per hybrid step, plain vs surrogate at <=1e-3 density err"
HBM_PEAK_GBS = 8000.0
BF16_MFMA_PEAK_TFLOPS = 2500.0  # dense
WEIGHTS = os.path.join(ROOT, "paper_1804_02883_amd", "weights", "surrogate_q.npy")
FALLBACK_EVERY = 50
ERR_TOL = 9e-4

# useful flops per site of each network launch (multiply-add = 2 flops):
# 9 taps x cin x cout x 2; the first layer has 5 real input channels
NN_FLOPS_PER_SITE = {"nn_conv0": 9 * 5 * 64 * 2, "nn_conv": 9 * 64 * 64 * 2}

# HBM traffic per launch measured with rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE (one counter per run, averaged over the kernel's dispatches),
# scaled by the same counters' readings for a plain 256 MiB copy (FETCH x2.0,
# WRITE x1.0); the summaries with their commands are under profiles/.  An
# entry holds only while the sources its kernels are built from hash to
# `source_sha256`; otherwise the bench reports null.
_PROP_FILES = ("fft.hpp", "kernels.hpp")
_NN_FILES = ("kernels.hpp", "nn.hpp")
MEASURED_TRAFFIC = {
    # profiles/prop_cfg3_traffic.md: the tuned propagator passes on 1024 x 512, N = 64
    ("cfg3", "prop_row"): dict(bytes_per_launch=16168805, files=_PROP_FILES,
                               source_sha256="877088b805e92cfbe6994e99c9fc2c678ef2c3253a7fbadb1721b17fee5559c1"),
    ("cfg3", "prop_col"): dict(bytes_per_launch=17296672, files=_PROP_FILES,
                               source_sha256="877088b805e92cfbe6994e99c9fc2c678ef2c3253a7fbadb1721b17fee5559c1"),
    # profiles/nn_conv_cfg5q_traffic.md: mean over the two 64 -> 64 launches of a surrogate step
    ("cfg5q", "nn_conv"): dict(bytes_per_launch=63871133, files=_NN_FILES,
                               source_sha256="d085c160fd00ceae2554be7dfed9b4249a4a78738a1216f4bc593522dcf7a606"),
    # profiles/lb3_fluid3d_256_traffic.md: the step kernel without moment stores
    ("fluid3d_256", "lb3"): dict(bytes_per_launch=2873793431, files=("lb3.hpp",),
                                 source_sha256="e7e59f031e128b313dda272b0a26b0ab5c5fe413ad9252a506d9b009c091450e"),
    # profiles/epd3_densities_256_traffic.md: mean over the five FFT passes of a contour step
    ("densities3d_256_N32", "p3_fft"): dict(bytes_per_launch=295385359, files=("epd3.hpp",),
                                            source_sha256="0f8cbbb975abf58193e39b668c073a1b5acfb5f18cfb18bb1665b18b037520b1"),
}


def kernel_source_sha256(files):
    import hashlib
    csrc = os.path.join(ROOT, "paper_1804_02883_amd", "csrc")
    data = b"".join(open(os.path.join(csrc, f), "rb").read() for f in files)
    return hashlib.sha256(data).hexdigest()


def measured_traffic(workload, fam):
    tr = MEASURED_TRAFFIC.get((workload, fam))
    if tr and tr["source_sha256"] == kernel_source_sha256(tr["files"]):
        return tr["bytes_per_launch"]
    return None


# Algorithmic bytes per site per hybrid STEP of each kernel family of the
# plain step, in units of the element size P (forward and backward chains
# counted together):
#   advect_update : read Phi 3, omega 3, u 2; write omega 3, S~ 1        = 12P
#   prop_row/col  : per chain, the first launch reads omega_A and omega_B and
#                   writes one half-step factor plane and the scratch plane
#                   (4P); a fused boundary launch reads scratch + factor and
#                   writes q_{a+1} + scratch (4P); the last reads scratch +
#                   factor and writes q_N (3P)
#   density       : read 2N chain planes + omega_S + S~, write Phi 3 + S = (2N + 6)P
#   force_*       : 3P + 4P (row FFT of S, column pass)
#   force_inv_lb  : the row-inverse force pass fused with the LB step: read the
#                   force spectrum 2 and 9 populations; write F 2 (kept for
#                   reads), 9 populations, rho, u 2                      = 25P
#   (force_row_inv 4P and lb 23P when a row shape runs them separately)
def step_bytes_per_site(kind, N, P):
    last_row = (N - 1) % 2 == 1           # the final propagator launch is x-oriented
    n_fused_row = sum(1 for s in range(N - 1) if s % 2 == 1)
    n_fused_col = sum(1 for s in range(N - 1) if s % 2 == 0)
    per_chain_row = 4 + 4 * n_fused_row + (3 if last_row else 0)
    per_chain_col = 4 * n_fused_col + (0 if last_row else 3)
    return {
        "advect_update": 12 * P,
        "prop_row": 2 * per_chain_row * P, "prop_col": 2 * per_chain_col * P,
        "density": (2 * N + 6) * P,
        "force_row_fwd": 3 * P, "force_col": 4 * P, "force_inv_lb": 25 * P,
        "force_row_inv": 4 * P, "lb": 23 * P,
    }.get(kind)


def window_start(run_len, steps, warmup, every=FALLBACK_EVERY):
    """First step of the timed window: a multiple of `every` (an exact step),
    at least `warmup` steps into the run, as late as a run of `run_len` steps
    allows."""
    lo = every * math.ceil(warmup / every)
    late = every * ((run_len - steps) // every)
    return max(lo, late)


def timed(sim, n):
    """Queue n steps between two HIP events on the context's stream; returns ms."""
    import torch
    if n <= 0:
        return 0.0
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    sim.sync()
    ev0.record(sim.stream)
    sim.step(n)
    ev1.record(sim.stream)
    ev1.synchronize()
    sim.sync()
    return ev0.elapsed_time(ev1)


def kernel_profile(sim, steps, launches_per_step):
    """Per-family launch durations over `steps` further steps, each launch timed
    by HIP events at its own start and end on the context's stream."""
    sim.profile_start(steps * launches_per_step + 64)
    sim.step(steps)
    prof = sim.profile_read()
    tot = sum(v["total_ms"] for v in prof.values())
    return prof, 1e3 * tot / steps


def say(msg):
    """Progress on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def gpu_info():
    import torch
    pr = torch.cuda.get_device_properties(0)
    return dict(name=pr.name, arch=getattr(pr, "gcnArchName", ""), cus=pr.multi_processor_count)


# ---------------------------------------------------------------------------
# The default line: plain vs surrogate on the 512^2 quench
# ---------------------------------------------------------------------------

def run_path(p, seed, sigma, weights, run_len, start, steps, tune_cache):
    """One path of the comparison: seed, then the run in three timed segments
    [0, start), [start, start + steps) (the window), and the rest up to run_len."""
    from paper_1804_02883_amd import Simulation
    sim = Simulation(p)
    if weights is not None:
        sim.surrogate_set_weights(weights)
    sim.seed(seed, sigma)
    if tune_cache:
        sim.autotune(20, tune_cache)
    ms_pre = timed(sim, start)
    d_pre = sim.diag()
    ms_win = timed(sim, steps)
    d_win = sim.diag()
    rest = max(0, run_len - start - steps)
    ms_post = timed(sim, rest)
    return sim, dict(ms_pre=ms_pre, ms_win=ms_win, ms_post=ms_post, d_pre=d_pre, d_win=d_win,
                     total_steps=start + steps + rest)


def surrogate_line(args):
    import numpy as np
    from seeded_inputs import PRESETS
    cfg = PRESETS["cfg5q"]
    p = dict(cfg["params"])
    n = p["nx"] * p["ny"]
    K, W = args.steps, args.warmup
    run_len = cfg["steps"]
    start = window_start(run_len, K, W)
    tc = None if args.no_tune else args.tune_cache
    w = np.load(WEIGHTS).astype(np.float32)

    pp = dict(p, density_mode=0)
    say(f"cfg5q plain path: {run_len} steps, window [{start}, {start + K})")
    sim_p, rp = run_path(pp, cfg["seed"], cfg["sigma"], None, run_len, start, K, tc)
    prof_p, ksum_p = kernel_profile(sim_p, 10, p["n_contour"] + 8)
    phi_plain = sim_p.densities()
    sim_p.close()

    ps = dict(p, density_mode=1, fallback_every=FALLBACK_EVERY, check_every=10, resid_tol=1e-3, err_tol=ERR_TOL)
    say(f"cfg5q surrogate path: {run_len} steps, window [{start}, {start + K})")
    sim_s, rs = run_path(ps, cfg["seed"], cfg["sigma"], w, run_len, start, K, tc)
    d_end = sim_s.diag()
    phi_sur = sim_s.densities()
    # per-launch durations in 100 further steps (two of them exact)
    prof_s, ksum_s = kernel_profile(sim_s, 100, 2 * (p["n_contour"] + 8) + 16)
    sim_s.close()

    fam = max(prof_s, key=lambda k: prof_s[k]["total_ms"])
    st = prof_s[fam]
    if fam in NN_FLOPS_PER_SITE:
        fl = NN_FLOPS_PER_SITE[fam] * n
        achieved = fl / (st["avg_ms"] / 1e3) / 1e12
        roofline = dict(bound="mfma", kernel=fam, achieved=round(achieved, 1), peak=BF16_MFMA_PEAK_TFLOPS,
                        unit="TFLOP/s", frac=round(achieved / BF16_MFMA_PEAK_TFLOPS, 4),
                        traffic=measured_traffic("cfg5q", fam), alg_flops_per_launch=fl)
    else:  # a memory-bound family dominates
        b = step_bytes_per_site(fam, p["n_contour"], 4) * n * 100 / st["launches"]
        achieved = b / (st["avg_ms"] / 1e3) / 1e9
        roofline = dict(bound="hbm", kernel=fam, achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=round(achieved / HBM_PEAK_GBS, 4), traffic=measured_traffic("cfg5q", fam),
                        alg_bytes_per_launch=int(b))
    roofline.update(avg_launch_us=round(st["avg_ms"] * 1e3, 3), launches_per_step=st["launches"] / 100,
                    kernel_sum_us_per_step=round(ksum_s, 2))
    breakdown = {k: dict(launches_per_step=v["launches"] / 100, avg_us=round(v["avg_ms"] * 1e3, 3),
                         tflops=(round(NN_FLOPS_PER_SITE[k] * n / (v["avg_ms"] / 1e3) / 1e12, 1)
                                 if k in NN_FLOPS_PER_SITE else None))
                 for k, v in sorted(prof_s.items(), key=lambda kv: -kv[1]["total_ms"])}

    win_sur = n * K / (rs["ms_win"] / 1e3)
    win_plain = n * K / (rp["ms_win"] / 1e3)
    tot_s = rs["ms_pre"] + rs["ms_win"] + rs["ms_post"]
    tot_p = rp["ms_pre"] + rp["ms_win"] + rp["ms_post"]
    nsteps = rs["total_steps"]
    ex_win = rs["d_win"]["n_exact"] - rs["d_pre"]["n_exact"]
    phiP_s, phiP_p = phi_sur[0] + phi_sur[1], phi_plain[0] + phi_plain[1]
    wl = (f"cfg5q: {cfg['name']}, seed {cfg['seed']}; each path runs {nsteps} steps from the seed; "
          f"timed window steps [{start}, {start + K}); surrogate with an exact step every {FALLBACK_EVERY} "
          f"steps, on the residual test, and while the last measured network error exceeds {ERR_TOL:g}")
    return dict(
        metric=METRIC, value=win_sur, unit="site-updates/s", n_gpus=1, steps=K, warmup=W,
        ms_per_step=rs["ms_win"] / K, higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f32+bf16", data="synthetic",
        config=dict(workload=wl, nx=p["nx"], ny=p["ny"], n_contour=p["n_contour"], path="surrogate",
                    window_start=start, window_exact_steps=ex_win),
        roofline=roofline,
        plain=dict(value=win_plain, ms_per_step=rp["ms_win"] / K,
                   kernel_sum_us_per_step=round(ksum_p, 2)),
        speedup=win_sur / win_plain,
        density_err=dict(bar=1e-3, in_use=rs["d_win"]["nn_err_in_use"], last=rs["d_win"]["nn_err_last"],
                         max_at_exact_steps=d_end["nn_err_max"],
                         note="in_use: max network error measured at exact steps that ended surrogate "
                              "steps, from the seed to the window's end; max_at_exact_steps includes the "
                              "gated start-up, where the network is not used",
                         uniform_density_err_at_end=float(np.max(np.abs(
                             phi_plain[:2] - phi_plain[:2].mean(axis=(1, 2), keepdims=True))))),
        whole_run=dict(steps=nsteps, surrogate=n * nsteps / (tot_s / 1e3), plain=n * nsteps / (tot_p / 1e3),
                       speedup=tot_p / tot_s, n_exact=d_end["n_exact"], n_triggered=d_end["n_triggered"]),
        sigma_delta_at_end=float(np.mean(np.abs(phiP_s - phiP_p))),
        breakdown=breakdown,
    )


# ---------------------------------------------------------------------------
# Plain-path lines
# ---------------------------------------------------------------------------

def plain_line(args, workload, steps, warmup):
    from paper_1804_02883_amd import Batch, Simulation
    say(f"{workload} plain path: {warmup} + {steps} steps")
    from seeded_inputs import PRESETS, replica_manifest
    if workload == "cfg4":
        man = replica_manifest()
        plist = [m["params"] for m in man]
        p = dict(plist[0])
        n = sum(q["nx"] * q["ny"] for q in plist)
        sim = Batch(plist)
        sim.seed([m["seed"] for m in man], man[0]["sigma"])
        if not args.no_tune:
            sim.autotune(20, args.tune_cache)
        shapes = None
        wl = (f"cfg4: {len(plist)} replicas from the seeded manifest (grids 64x64, 128x128, 256x128, "
              f"512x256; g in [0, 5e-5] f*, f_A in {{0.3, 0.5}}), N=32, FP32, chi reading L, seeds 4000+r, "
              f"{n} sites, plain (exact propagator)")
        cfgd = dict(workload=wl, replicas=len(plist), sites=n, n_contour=32, path="plain")
        per_step = (p["n_contour"] + 8) * sim.info()[0]
    else:
        cfg = PRESETS[workload]
        p = dict(cfg["params"])
        lb_note = "BGK tau=%g" % p["lb_tau"]
        if args.lb == "mrt":
            # the paper's fluid: eta = eta_B = 1 R_G^2/tau rho (Sec. III) at this dx, dt
            from paper_1804_02883_amd import mrt_gammas
            gs, gb = mrt_gammas(1.0, 1.0, 1.0, p["dx"], p["dt"])
            p.update(lb_mrt=1, lb_gamma_s=gs, lb_gamma_b=gb, lb_gamma_g=0.0)
            lb_note = "multi-relaxation, eta = eta_B = 1 (gamma_s = gamma_b = %.4f, gamma_g = 0)" % gs
        n = p["nx"] * p["ny"]
        sim = Simulation(p)
        sim.seed(cfg["seed"], cfg["sigma"])
        shapes = sim.shapes() if args.no_tune else sim.autotune(20, args.tune_cache)
        wl = (f"{workload}: {cfg['name']}, g={p['g']}, "
              f"seed {cfg['seed']} noise sigma {cfg['sigma']}, plain (exact propagator)")
        cfgd = dict(workload=wl, nx=p["nx"], ny=p["ny"], n_contour=p["n_contour"], path="plain", lb=lb_note)
        per_step = p["n_contour"] + 8
    N = p["n_contour"]
    P = 8 if p["precision"] == 0 else 4
    timed(sim, warmup)
    ms = timed(sim, steps)
    prof_steps = max(1, min(20, 4096 // per_step))
    prof, ksum = kernel_profile(sim, prof_steps, per_step)
    d = sim.diag() if workload != "cfg4" else sim.diag(0)
    sim.close()
    fams = [k for k in prof if step_bytes_per_site(k, N, P) is not None]
    fam = max(fams, key=lambda k: prof[k]["total_ms"])
    alg = step_bytes_per_site(fam, N, P) * n * prof_steps / prof[fam]["launches"]
    achieved = alg / (prof[fam]["avg_ms"] / 1e3) / 1e9
    roofline = dict(bound="hbm", kernel=fam, achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=measured_traffic(workload, fam),
                    avg_launch_us=round(prof[fam]["avg_ms"] * 1e3, 3),
                    launches_per_step=prof[fam]["launches"] / prof_steps, alg_bytes_per_launch=int(alg),
                    kernel_sum_us_per_step=round(ksum, 2))
    breakdown = {k: dict(launches_per_step=v["launches"] / prof_steps, avg_us=round(v["avg_ms"] * 1e3, 3),
                         gbs=(round(step_bytes_per_site(k, N, P) * n * prof_steps / (v["total_ms"] / 1e3) / 1e9, 1)
                              if step_bytes_per_site(k, N, P) else None))
                 for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["total_ms"])}
    return dict(metric=METRIC, value=n * steps / (ms / 1e3), unit="site-updates/s", n_gpus=1, steps=steps,
                warmup=warmup, ms_per_step=ms / steps, higher_is_better=True, scaling="weak",
                vs_baseline=None, dtype="f32" if P == 4 else "f64", data="synthetic",
                config=cfgd, roofline=roofline, breakdown=breakdown, shapes=shapes, Q_P=d["Q_P"])


# ---------------------------------------------------------------------------
# CPU baseline: the oracle as it stands
# ---------------------------------------------------------------------------

def _oracle_steps(preset_name, seconds, barrier=None, out=None):
    import numpy as np  # noqa: F401
    from oracle import epdlb_oracle as O
    from seeded_inputs import PRESETS, initial_omega
    cfg = PRESETS[preset_name]
    p = dict(cfg["params"])
    s = O.init_state(p, initial_omega(p["nx"], p["ny"], cfg["seed"], cfg["sigma"]))
    if barrier is not None:
        barrier.wait()
    t0 = time.perf_counter()
    steps = 0
    while steps == 0 or time.perf_counter() - t0 < seconds:
        s = O.step(s, p)
        steps += 1
    r = (steps, time.perf_counter() - t0)
    if out is not None:
        out.put(r)
    return r


def host_cpu():
    model = ""
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in txt.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    if not model and os.path.exists("/proc/cpuinfo"):
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return dict(model=model, nproc=os.cpu_count(), available=avail)


def cpu_baseline(preset_name, seconds, max_procs=16):
    """The oracle's plain hybrid step on the host, in one process and in one
    single-threaded process per available core (at most max_procs) side by side."""
    import multiprocessing as mp
    from seeded_inputs import PRESETS
    p = PRESETS[preset_name]["params"]
    n = p["nx"] * p["ny"]
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    info = host_cpu()
    steps1, dt1 = _oracle_steps(preset_name, seconds)
    procs = max(1, min(max_procs, info["available"] or 1))
    ctx = mp.get_context("spawn")
    bar = ctx.Barrier(procs)
    q = ctx.Queue()
    ws = [ctx.Process(target=_oracle_steps, args=(preset_name, seconds, bar, q)) for _ in range(procs)]
    for w in ws:
        w.start()
    res = [q.get(timeout=600) for _ in ws]
    for w in ws:
        w.join(timeout=60)
    rate_all = sum(n * s / t for s, t in res)
    name = f"{preset_name} ({p['nx']}x{p['ny']}, N={p['n_contour']})"
    return dict(value=rate_all, unit="site-updates/s", cores=procs, kind="oracle",
                sample=f"plain hybrid steps (exact propagator) of {name}, FP64 NumPy oracle: {procs} "
                       f"single-threaded processes side by side, {sum(s for s, _ in res)} steps in about "
                       f"{max(t for _, t in res):.1f} s",
                single_core=dict(value=n * steps1 / dt1, cores=1,
                                 sample=f"{steps1} steps in {dt1:.1f} s, one process, one thread"),
                host=info)


# ---------------------------------------------------------------------------
# Secondary objects
# ---------------------------------------------------------------------------

def fluid3d_cpu_baseline(seconds=3.0, n=64):
    """The FP64 NumPy oracle's BGK step on an n^3 box (elementwise NumPy: one
    thread), for `seconds` of host time."""
    import numpy as np
    from oracle import lb3d_oracle as L3
    rng = np.random.default_rng(3)
    f = L3.equilibrium(np.ones((n, n, n)), 1e-3 * rng.standard_normal((3, n, n, n)))
    F = 1e-5 * rng.standard_normal((3, n, n, n))
    steps, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        f, _, _ = L3.step(f, F, 0.8)
        steps += 1
    dt = time.perf_counter() - t0
    return dict(value=steps * n ** 3 / dt, unit="site-updates/s", cores=1, kind="oracle",
                sample=f"{steps} BGK steps of a {n}^3 box, FP64 NumPy oracle, single thread, {dt:.1f} s")


def densities3d_cpu_baseline(seconds=3.0, n=32, N=16):
    """The FP64 NumPy oracle's density evaluation on an n^3 grid (numpy.fft)."""
    import numpy as np
    from oracle import epd3d_oracle as E3
    from seeded_inputs import preset
    p = preset("cfg1", n_contour=N, f_A=0.3, phi_P=0.15)
    w = 0.2 * np.random.default_rng(5).standard_normal((3, n, n, n))
    evals, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        E3.densities3(w, p)
        evals += 1
    dt = time.perf_counter() - t0
    return dict(value=evals * n ** 3 * 2 * N / dt, unit="site contour steps/s", cores=1, kind="oracle",
                sample=f"{evals} density evaluations of a {n}^3 grid, N = {N}, FP64 NumPy oracle, {dt:.1f} s")


def fluid3d_line(cpu=True):
    from paper_1804_02883_amd import fluid3d_timing
    r = fluid3d_timing.measure(256, 40, 1)
    r["roofline"]["traffic"] = measured_traffic("fluid3d_256", "lb3")
    if cpu:
        r["cpu_baseline"] = fluid3d_cpu_baseline()
    return r


def densities3d_line(cpu=True):
    from paper_1804_02883_amd import epd3_timing
    r = epd3_timing.measure(256, 32, 3, 1)
    r["roofline"]["traffic"] = measured_traffic("densities3d_256_N32", "p3_fft")
    if cpu:
        r["cpu_baseline"] = densities3d_cpu_baseline()
    return r


def run_probe(name):
    """Run a stand-alone probe built with the library (paper_1804_02883_amd/probes/<name>.hip)
    and return its JSON line:
      sync_costs  host and GPU cost of a dependent kernel launch (stream and graph
                  node) and of a device-wide barrier in a cooperative kernel;
      conv_floor  the matrix work, the activation stores and both together of one
                  64 -> 64 layer at 512^2, launched as the layer kernel is."""
    exe = os.path.join(ROOT, "paper_1804_02883_amd", "probes", name)
    if not os.path.exists(exe):
        return dict(note="probe not built")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    if r.returncode != 0:
        return dict(note="probe failed: " + r.stderr[-300:])
    return json.loads(r.stdout.strip().splitlines()[-1])


def positive(v):
    i = int(v)
    if i < 1:
        raise argparse.ArgumentTypeError("must be a positive integer")
    return i


def non_negative(v):
    i = int(v)
    if i < 0:
        raise argparse.ArgumentTypeError("must be a non-negative integer")
    return i


def parse_args(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=positive, default=2000, help="timed steps K")
    ap.add_argument("--warmup", type=non_negative, default=50, help="untimed steps W before the window")
    ap.add_argument("--workload", default="cfg5q", choices=["cfg5q", "cfg3", "cfg2", "cfg4", "cfg5"])
    ap.add_argument("--secondary-steps", type=positive, default=1000,
                    help="timed steps of the secondary plain run (plain_full_scale)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="host time of each oracle baseline leg (whole steps)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_1804_02883_amd", "tune", "gfx950.txt"),
                    help="autotuner results file (read first, new results appended)")
    ap.add_argument("--lb", default="bgk", choices=["bgk", "mrt"],
                    help="LB collision of a plain single-grid workload: BGK at the preset's tau, or the "
                         "multi-relaxation collision at the paper's eta = eta_B")
    ap.add_argument("--no-secondary", action="store_true",
                    help="only the workload's own line (no plain_full_scale, fluid3d, densities3d)")
    return ap.parse_args(argv)


def main(argv=None):
    args = parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU (asked for --gpus {args.gpus}); "
              "the library has no multi-GPU sharding", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    if args.workload == "cfg5q":
        out = surrogate_line(args)
        if not args.no_secondary:
            pl = plain_line(args, "cfg3", args.secondary_steps, 20)
            out["plain_full_scale"] = dict(workload=pl["config"]["workload"], value=pl["value"],
                                           steps=pl["steps"], ms_per_step=pl["ms_per_step"],
                                           roofline=pl["roofline"], breakdown=pl["breakdown"])
    else:
        out = plain_line(args, args.workload, args.steps, args.warmup)
    if not args.no_secondary:
        say("fluid3d 256^3")
        out["fluid3d"] = fluid3d_line(cpu=not args.no_cpu_baseline)
        say("densities3d 256^3")
        out["densities3d"] = densities3d_line(cpu=not args.no_cpu_baseline)
    out["gpu"] = gpu_info()
    out["gpu_wall_s"] = round(time.perf_counter() - t0, 1)
    if not args.no_secondary:
        say("sync costs probe")
        out["sync_costs"] = run_probe("sync_costs")
        say("convolution floor probe")
        out["conv_floor"] = run_probe("conv_floor")
    if not args.no_cpu_baseline and args.workload != "cfg4":
        say(f"cpu baseline: the oracle on {args.workload}, {args.cpu_seconds:g} s per leg")
        out["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
