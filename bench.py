"""Benchmark: lattice site-updates/s of the hybrid LB/EPD step on one MI355X.

A "step" is one full hybrid step (advection + EPD update, densities, force
reconstruction, D2Q9 LB) on the resident state.

Default workload (cfg5q), plain versus surrogate: 512 x 512 periodic grid,
FP32 fields with FP64 partition-function reductions, N = 32, f_A = 0.5,
phi_P = 0.1, chi reading Q, g = 1e-5 f*, seeded Gaussian noise sigma = 0.05
(seed 1005), 2e4 steps from the seed for each path.  `value` is the
surrogate path's rate over its whole run: its exact steps (every 50 steps,
on the residual test, and while the last measured network error exceeds
9e-4) included; `density_err.in_use` is the largest network error measured
at an exact step that ended surrogate steps.  `roofline` is the MFMA
roofline of the 64 -> 64 convolution.  `plain_full_scale` adds the plain
path on 1024 x 512, N = 64 with its HBM roofline, and `fluid3d` the
three-dimensional D3Q19 fluid on a 256^3 box (FP32) with the HBM roofline of
its step kernel (paper_1804_02883_amd/fluid3d_timing.py), and `densities3d`
the propagators and densities on a 256^3 grid (FP32, N = 32) with the HBM
roofline of its FFT kernel (paper_1804_02883_amd/epd3_timing.py).

`--workload cfg3` (or cfg2, cfg5, cfg4) reports a plain line instead.

Prints ONE JSON line.  `value` is timed with events around K graph-replayed
steps.  `roofline` covers the kernel family with the largest share of GPU
time; its kernel durations come from HIP start/stop events that each launch
records at the kernel's own start and end (stream launches of the same
workload right after the timed region).  `cpu_baseline` is the FP64 NumPy
oracle on a bounded sample of the same workload on the host.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "lattice site-updates/s per hybrid step, plain vs surrogate at <=1e-3 density err"

# HBM traffic per launch measured with rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE
# (one counter per run, averaged over the kernel's dispatches), scaled by the
# same counters' readings for a plain 256 MiB copy (FETCH x2.0, WRITE x1.0);
# the summaries with their commands are profiles/prop_cfg3_traffic.md and
# profiles/nn_conv_cfg5q_traffic.md.  An entry is valid only while the sources
# its kernels are built from hash to `source_sha256`.
_PROP_FILES = ("fft.hpp", "kernels.hpp")
_NN_FILES = ("kernels.hpp", "nn.hpp")
MEASURED_TRAFFIC = {
    ("cfg3", "prop_col"): dict(bytes_per_launch=17284293, files=_PROP_FILES,
                               source_sha256="09839588ecde426f14350f4230b579f6c49ce5e55f9ba4f31f96cd374db85421"),
    ("cfg3", "prop_row"): dict(bytes_per_launch=16173527, files=_PROP_FILES,
                               source_sha256="09839588ecde426f14350f4230b579f6c49ce5e55f9ba4f31f96cd374db85421"),
    # mean over the two 64 -> 64 launches of a surrogate step
    ("cfg5q", "nn_conv"): dict(bytes_per_launch=63970359, files=_NN_FILES,
                               source_sha256="4f00c90da1997534e3811f0beb2591c36ceaec6e5898195cfffe087c312feb2d"),
    # profiles/lb3_fluid3d_256_traffic.md: the step kernel without moment stores
    # profiles/epd3_densities_256_traffic.md: mean over the five FFT passes of a contour step
    ("densities3d_256_N32", "p3_fft"): dict(bytes_per_launch=295385359, files=("epd3.hpp",),
                                            source_sha256="0f8cbbb975abf58193e39b668c073a1b5acfb5f18cfb18bb1665b18b037520b1"),
    ("fluid3d_256", "lb3"): dict(bytes_per_launch=2873793431, files=("lb3.hpp",),
                                 source_sha256="e7e59f031e128b313dda272b0a26b0ab5c5fe413ad9252a506d9b009c091450e"),
}


def kernel_source_sha256(files=_PROP_FILES):
    import hashlib
    csrc = os.path.join(ROOT, "paper_1804_02883_amd", "csrc")
    data = b"".join(open(os.path.join(csrc, f), "rb").read() for f in files)
    return hashlib.sha256(data).hexdigest()


def measured_traffic(workload, fam):
    tr = MEASURED_TRAFFIC.get((workload, fam))
    if tr and tr["source_sha256"] == kernel_source_sha256(tr["files"]):
        return tr["bytes_per_launch"]
    return None


HBM_PEAK_GBS = 8000.0
BF16_MFMA_PEAK_TFLOPS = 2500.0  # dense
WEIGHTS = os.path.join(ROOT, "paper_1804_02883_amd", "weights", "surrogate_q.npy")
# useful flops per site of each network launch (multiply-add = 2 flops):
# 9 taps x cin x cout x 2; conv0 has 5 real input channels, the output layer 2
NN_FLOPS_PER_SITE = {"nn_conv0": 9 * 5 * 64 * 2, "nn_conv": 9 * 64 * 64 * 2}

# Algorithmic bytes per site per hybrid STEP of each kernel family, in units
# of the element size P (forward and backward chains counted together):
#   advect_update : read Phi 3, omega 3, u 2; write omega 3, S~ 1        = 12P
#   prop_row/col  : per chain, the first launch reads omega_A and omega_B and
#                   writes one half-step factor plane and the scratch plane
#                   (4P); a fused boundary launch
#                   reads scratch + factor and writes q_{a+1} + scratch (4P);
#                   the last reads scratch + factor and writes q_N (3P)
#   density       : read 2N chain planes + omega_S + S~, write Phi 3 + S = (2N + 6)P
#   force_*       : 3P + 4P + 4P (row FFT of S, column pass, row inverse)
#   lb            : read 9 populations + F 2; write 9 + rho + u 2        = 23P
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
        "force_row_fwd": 3 * P, "force_col": 4 * P, "force_row_inv": 4 * P,
        "lb": 23 * P,
    }.get(kind)


def cpu_baseline(preset_name, seconds):
    """The oracle's plain hybrid step on the host: whole steps until `seconds` have passed."""
    import numpy as np  # noqa: F401
    from oracle import epdlb_oracle as O
    from seeded_inputs import PRESETS, initial_omega
    cfg = PRESETS[preset_name]
    p = dict(cfg["params"])
    w0 = initial_omega(p["nx"], p["ny"], cfg["seed"], cfg["sigma"])
    s = O.init_state(p, w0)
    t0 = time.perf_counter()
    steps = 0
    while steps == 0 or time.perf_counter() - t0 < seconds:
        s = O.step(s, p)
        steps += 1
    dt = time.perf_counter() - t0
    n = p["nx"] * p["ny"]
    return dict(value=n * steps / dt, unit="site-updates/s", cores=1, kind="oracle",
                sample=f"{steps} plain hybrid steps (exact propagator) of {preset_name}, {p['nx']}x{p['ny']} "
                       f"N={p['n_contour']}, FP64 NumPy oracle, single thread, {dt:.1f} s")


def surrogate_summary(steps, tune_cache=None):
    """Plain vs surrogate on the 512^2 quench (cfg5q), full runs from the seed, both
    with the autotuned FFT launch shapes when a tune cache is given."""
    import numpy as np
    from paper_1804_02883_amd.surrogate_eval import compare
    from seeded_inputs import PRESETS
    cfg = PRESETS["cfg5q"]
    w = np.load(WEIGHTS)
    r = compare(dict(cfg["params"]), cfg["seed"], cfg["sigma"], w, steps, tune_cache=tune_cache)
    r["workload"] = f"cfg5q: {cfg['name']}, seed {cfg['seed']}, {r['steps']} steps from the seed"
    return r


def surrogate_line(args):
    """The surrogate path on the 512^2 quench (cfg5q) as a bench line."""
    import numpy as np
    from paper_1804_02883_amd import Simulation
    from seeded_inputs import PRESETS
    cfg = PRESETS["cfg5q"]
    p = dict(cfg["params"])
    n = p["nx"] * p["ny"]
    steps = args.steps if args.steps_given else cfg["steps"]
    tc = None if args.no_tune else args.tune_cache
    r = surrogate_summary(steps - 50, tc)
    # per-kernel durations of surrogate steps (100 steps, 2 of them exact)
    sim = Simulation(dict(p, density_mode=1, fallback_every=50, check_every=10, resid_tol=1e-3, err_tol=0.0))
    sim.surrogate_set_weights(np.load(WEIGHTS))
    sim.seed(cfg["seed"], cfg["sigma"])
    if tc:
        sim.autotune(20, tc)
    sim.step(100)
    sim.sync()
    sim.profile_start(4000)
    sim.step(100)
    prof = sim.profile_read()
    sim.close()
    conv = prof["nn_conv"]
    achieved = NN_FLOPS_PER_SITE["nn_conv"] * n / (conv["avg_ms"] / 1e3) / 1e12
    roofline = dict(bound="mfma", kernel="nn_conv", achieved=round(achieved, 1), peak=BF16_MFMA_PEAK_TFLOPS,
                    unit="TFLOP/s", frac=round(achieved / BF16_MFMA_PEAK_TFLOPS, 4),
                    traffic=measured_traffic("cfg5q", "nn_conv"),
                    avg_launch_us=round(conv["avg_ms"] * 1e3, 3), launches_per_step=conv["launches"] / 100,
                    alg_flops_per_launch=NN_FLOPS_PER_SITE["nn_conv"] * n)
    tot = sum(x["total_ms"] for x in prof.values())
    breakdown = {k: dict(launches_per_step=v["launches"] / 100, avg_us=round(v["avg_ms"] * 1e3, 3),
                         share=round(v["total_ms"] / tot, 4),
                         tflops=(round(NN_FLOPS_PER_SITE[k] * n / (v["avg_ms"] / 1e3) / 1e12, 1)
                                 if k in NN_FLOPS_PER_SITE else None))
                 for k, v in prof.items()}
    breakdown["kernel_sum_us_per_step"] = round(1e3 * tot / 100, 2)
    sur = r["surrogate"]
    return dict(metric=METRIC, value=sur["value"], unit="site-updates/s", n_gpus=1, steps=r["steps"], warmup=50,
                ms_per_step=sur["ms_per_step"], higher_is_better=True, scaling="weak", vs_baseline=None,
                dtype="f32+bf16", data="synthetic",
                config=dict(workload=r["workload"] + "; exact step every 50 steps, on the residual test, and "
                            "while the last measured surrogate error exceeds 9e-4",
                            nx=p["nx"], ny=p["ny"], n_contour=p["n_contour"], path="surrogate"),
                roofline=roofline, breakdown=breakdown,
                plain=dict(value=r["plain"]["value"], ms_per_step=r["plain"]["ms_per_step"]),
                speedup=r["speedup"],
                density_err=dict(in_use=sur["density_err_in_use"], bar=1e-3,
                                 max_at_exact_steps=sur["max_density_err"], last=sur["last_density_err"],
                                 uniform_density_err_at_end=r["fluct_max"]),
                n_exact=sur["n_exact"], n_triggered=sur["n_triggered"], sigma_delta=r["sigma_delta"])


def plain_line(args, workload):
    """The plain (exact propagator) path on one workload as a bench line."""
    import torch
    from paper_1804_02883_amd import Batch, Simulation
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
    else:
        cfg = PRESETS[workload]
        p = dict(cfg["params"])
        lb_note = "BGK tau=%g" % p["lb_tau"]
        if getattr(args, "lb", "bgk") == "mrt":
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
    N = p["n_contour"]
    P = 8 if p["precision"] == 0 else 4
    steps = args.steps if args.steps_given else 2000
    sim.step(args.warmup)
    sim.sync()

    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    sim.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    sim.sync()
    # per-kernel durations: HIP start/stop events recorded by each kernel launch
    # itself (stream launches of the same workload, right after the timed region)
    per_step = (N + 8) * (1 if workload != "cfg4" else sim.info()[0])
    prof_steps = max(1, min(50, args.profile_launches // per_step))
    sim.profile_start(prof_steps * per_step + 16)
    sim.step(prof_steps)
    prof = sim.profile_read()
    ms_per_step = ms / steps
    value = n * steps / (ms / 1e3)

    # dominant kernel family by GPU time; achieved = its algorithmic bytes over
    # the profiled steps / its summed kernel durations
    fams = [k for k in prof if step_bytes_per_site(k, N, P) is not None]
    fam = max(fams, key=lambda k: prof[k]["total_ms"])
    alg_bytes = step_bytes_per_site(fam, N, P) * n * prof_steps
    achieved = alg_bytes / (prof[fam]["total_ms"] / 1e3) / 1e9
    traffic = measured_traffic(workload, fam)
    roofline = dict(bound="hbm", kernel=fam, achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                    avg_launch_us=round(prof[fam]["avg_ms"] * 1e3, 3),
                    launches_per_step=prof[fam]["launches"] // prof_steps,
                    alg_bytes_per_launch=int(alg_bytes / prof[fam]["launches"]))
    tot = sum(x["total_ms"] for x in prof.values())
    breakdown = {k: dict(launches_per_step=v["launches"] / prof_steps, avg_us=round(v["avg_ms"] * 1e3, 3),
                         share=round(v["total_ms"] / tot, 4),
                         gbs=(round(step_bytes_per_site(k, N, P) * n * prof_steps / (v["total_ms"] / 1e3) / 1e9, 1)
                              if step_bytes_per_site(k, N, P) else None))
                 for k, v in prof.items()}
    breakdown["kernel_sum_us_per_step"] = round(1e3 * tot / prof_steps, 2)
    d = sim.diag() if workload != "cfg4" else sim.diag(0)
    sim.close()
    return dict(metric=METRIC, value=value, unit="site-updates/s", n_gpus=1, steps=steps,
                warmup=args.warmup, ms_per_step=ms_per_step, higher_is_better=True, scaling="weak",
                vs_baseline=None, dtype="f32" if P == 4 else "f64", data="synthetic",
                config=cfgd, roofline=roofline, breakdown=breakdown, shapes=shapes, Q_P=d["Q_P"])


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


def fluid3d_line(cpu=True):
    """The three-dimensional D3Q19 fluid on a 256^3 box (FP32), with the HBM
    roofline of its step kernel."""
    from paper_1804_02883_amd import fluid3d_timing
    r = fluid3d_timing.measure(256, 40, 1)
    r["roofline"]["traffic"] = measured_traffic("fluid3d_256", "lb3")
    if cpu:
        r["cpu_baseline"] = fluid3d_cpu_baseline()
    return r


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


def densities3d_line(cpu=True):
    """Propagators and densities on a 256^3 grid (FP32, N = 32), with the HBM
    roofline of the FFT kernel."""
    from paper_1804_02883_amd import epd3_timing
    r = epd3_timing.measure(256, 32, 3, 1)
    r["roofline"]["traffic"] = measured_traffic("densities3d_256_N32", "p3_fft")
    if cpu:
        r["cpu_baseline"] = densities3d_cpu_baseline()
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 20000 for cfg5q, the run from the seed; 2000 otherwise)")
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="cfg5q", choices=["cfg5q", "cfg3", "cfg2", "cfg4", "cfg5"])
    ap.add_argument("--profile-launches", type=int, default=8192)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="host time budget of the oracle baseline (whole steps)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_1804_02883_amd", "tune", "gfx950.txt"),
                    help="autotuner results file (read first, new results appended)")
    ap.add_argument("--lb", default="bgk", choices=["bgk", "mrt"],
                    help="LB collision of the plain single-grid workloads: BGK at the preset's tau, or "
                         "the multi-relaxation collision at the paper's eta = eta_B")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the secondary measurements on the line (the 1024x512 plain run for cfg5q, "
                         "the cfg5q plain vs surrogate run otherwise, and the 256^3 D3Q19 fluid)")
    args = ap.parse_args()
    args.steps_given = args.steps is not None
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU (asked for --gpus {args.gpus}); "
              "the library has no multi-GPU sharding", file=sys.stderr)
        sys.exit(2)

    import torch
    torch.cuda.set_device(0)
    if args.workload == "cfg5q":
        out = surrogate_line(args)
        if not args.no_secondary:
            a3 = argparse.Namespace(**vars(args))
            a3.steps_given = False
            pl = plain_line(a3, "cfg3")
            out["plain_full_scale"] = dict(workload=pl["config"]["workload"], value=pl["value"],
                                           ms_per_step=pl["ms_per_step"], roofline=pl["roofline"])
    if not args.no_secondary:
        out["fluid3d"] = fluid3d_line(cpu=not args.no_cpu_baseline)
        out["densities3d"] = densities3d_line(cpu=not args.no_cpu_baseline)
    else:
        out = plain_line(args, args.workload)
        if not args.no_secondary and args.workload != "cfg4":
            out["surrogate"] = surrogate_summary(20000 - 50, None if args.no_tune else args.tune_cache)
    if not args.no_cpu_baseline and args.workload != "cfg4":
        out["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
