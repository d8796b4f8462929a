"""Benchmark: lattice site-updates/s of the plain hybrid LB/EPD step on one MI355X.

Workload (default): 1024 x 512 periodic grid, FP32 fields with FP64
partition-function reductions, N = 64 contour steps, f_A = 0.3, phi_P = 0.15,
chi reading L, g = 1e-5 f*, seeded Gaussian noise sigma = 1e-3 (seed 1003).
A "step" is one full hybrid step (advection + EPD update, both chain
propagators, densities, force reconstruction, D2Q9 LB) on the resident state.

Prints ONE JSON line.  `roofline` covers the kernel family with the largest
share of GPU time, timed with HIP events on the library's stream over the
first launches of the timed region; `cpu_baseline` is the FP64 NumPy oracle
on a bounded sample of the same workload on the host.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "lattice site-updates/s per hybrid step, plain vs surrogate at <=1e-3 density err"
HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per site per launch of each kernel family, in units of the
# element size P (forward and backward chains counted together):
#   prop_row / prop_col : 2 chains x (read P + write P)            = 4P
#   density             : read 2(N+1) chain planes, write 3 + S   = 2(N+1)P + 4P
#   advect_update       : read Phi 3, omega 3, u 2; write omega 3, S~ 1 = 12P
#   force (3 passes)    : 11P in total
#   lb                  : read 9 + F 2, write 9 + rho + u 2        = 23P
def bytes_per_site(kind, N, P):
    return {
        "prop_row": 4 * P, "prop_col": 4 * P,
        "density": (2 * (N + 1) + 4) * P,
        "advect_update": 12 * P,
        "force_row_fwd": 3 * P, "force_col": 4 * P, "force_row_inv": 4 * P,
        "lb": 23 * P,
    }.get(kind)


def cpu_baseline(preset_name, steps):
    import numpy as np  # noqa: F401
    from oracle import epdlb_oracle as O
    from seeded_inputs import PRESETS, initial_omega
    cfg = PRESETS[preset_name]
    p = dict(cfg["params"])
    w0 = initial_omega(p["nx"], p["ny"], cfg["seed"], cfg["sigma"])
    s = O.init_state(p, w0)
    t0 = time.perf_counter()
    for _ in range(steps):
        s = O.step(s, p)
    dt = time.perf_counter() - t0
    n = p["nx"] * p["ny"]
    return dict(value=n * steps / dt, unit="site-updates/s", cores=1, kind="oracle",
                sample=f"{steps} hybrid steps of {p['nx']}x{p['ny']} N={p['n_contour']} FP64 "
                       f"(NumPy, single thread), {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="cfg3")
    ap.add_argument("--profile-launches", type=int, default=8192)
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--tune-cache", default=None)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "multi-GPU sharding is described in DESIGN.md, not built", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1804_02883_amd import Simulation
    from seeded_inputs import PRESETS

    cfg = PRESETS[args.workload]
    p = dict(cfg["params"])
    n = p["nx"] * p["ny"]
    N = p["n_contour"]
    P = 8 if p["precision"] == 0 else 4
    torch.cuda.set_device(0)
    sim = Simulation(p)
    sim.seed(cfg["seed"], cfg["sigma"])
    shapes = sim.shapes() if args.no_tune else sim.autotune(20, args.tune_cache)
    sim.step(args.warmup)
    sim.sync()

    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    sim.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    sim.sync()
    # per-kernel event timing (stream launches, after the timed region)
    sim.profile_start(args.profile_launches)
    sim.step(max(1, args.profile_launches // (2 * N + 8)))
    prof = sim.profile_read()
    ms_per_step = ms / args.steps
    value = n * args.steps / (ms / 1e3)

    # dominant kernel family by recorded GPU time
    fam = max((k for k in prof if bytes_per_site(k, N, P) is not None), key=lambda k: prof[k]["total_ms"])
    avg_s = prof[fam]["avg_ms"] / 1e3
    alg_bytes = bytes_per_site(fam, N, P) * n
    achieved = alg_bytes / avg_s / 1e9
    roofline = dict(bound="hbm", kernel=fam, achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None,
                    avg_launch_us=round(prof[fam]["avg_ms"] * 1e3, 3),
                    alg_bytes_per_launch=alg_bytes)
    breakdown = {k: dict(launches=v["launches"], avg_us=round(v["avg_ms"] * 1e3, 3),
                         share=round(v["total_ms"] / max(sum(x["total_ms"] for x in prof.values()), 1e-30), 4))
                 for k, v in prof.items()}
    d = sim.diag()
    sim.close()

    out = dict(metric=METRIC, value=value, unit="site-updates/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=ms_per_step, higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="f32" if P == 4 else "f64", data="synthetic",
               config=dict(workload=f"{args.workload}: {cfg['name']}, chi reading L, g={p['g']}, "
                                    f"seed {cfg['seed']} noise sigma {cfg['sigma']}, plain (exact propagator)",
                           nx=p["nx"], ny=p["ny"], n_contour=N, path="plain"),
               roofline=roofline, breakdown=breakdown, shapes=shapes, Q_P=d["Q_P"])
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
