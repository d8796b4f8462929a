"""Timing of steps with the Phi -> omega inversion (App. C) against the default
step on the same workload (library calls only).

    python -m paper_1804_02883_amd.cg_timing --workload cfg3 --g 5e-7 --steps 10

The fields are FP64 (the paper's tolerance 1e-8 is below FP32 resolution).
--g is the body-force amplitude in lattice units (--g-paper: the preset's
amplitude in the paper's force unit, whose flow leaves the auxiliary-convected
omega within the tolerance, so most steps need no iteration).  The inversion
steps run eagerly (the host reads two sums per line search); the default
steps replay captured graphs.  Prints one JSON line: wall time per step of
both, iterations and density evaluations per inversion step, and the wall
time per evaluation implied by the difference.
"""
import argparse
import json
import time

import numpy as np


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="cfg3")
    ap.add_argument("--g", type=float, default=5e-7, help="lattice-unit force amplitude")
    ap.add_argument("--g-paper", action="store_true", help="use the preset's force in paper units")
    ap.add_argument("--sigma", type=float, default=0.05, help="seeded noise amplitude of omega")
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--tune-cache", default=None)
    ap.add_argument("--precond", type=int, default=0, help="1: diagonal preconditioning of the iteration")
    args = ap.parse_args(argv)
    import torch
    from paper_1804_02883_amd import Simulation
    from seeded_inputs import PRESETS, initial_omega, preset
    torch.cuda.set_device(0)
    over = dict(precision=0) if args.g_paper else dict(precision=0, g=args.g, g_units=1)
    base = preset(args.workload, **over)
    w0 = initial_omega(base["nx"], base["ny"], PRESETS[args.workload]["seed"], args.sigma)
    base["cg_precond"] = args.precond
    out = dict(workload=args.workload, precond=args.precond, nx=base["nx"], ny=base["ny"], N=base["n_contour"],
               g=base["g"], g_units=base["g_units"], sigma=args.sigma, steps=args.steps)
    for cg in (0, 1):
        sim = Simulation(dict(base, cg_invert=cg))
        sim.set_fields(w0)
        if args.tune_cache:
            sim.autotune(cache_path=args.tune_cache)
        sim.step(args.warmup)
        sim.sync()
        t0 = time.perf_counter()
        sim.step(args.steps)
        sim.sync()
        dt = (time.perf_counter() - t0) / args.steps
        key = "cg" if cg else "plain"
        out[f"ms_per_step_{key}"] = dt * 1e3
        if cg:
            last, tot = sim.cg_stats()
            n = tot["inversions"]
            out["iters_per_step"] = tot["iterations"] / n
            out["evals_per_step"] = tot["evals"] / n
            out["unconverged"] = tot["unconverged"]
            out["last_resid0"] = last["resid0"]
            out["last_resid"] = last["resid"]
        sim.close()
    extra = out["ms_per_step_cg"] - out["ms_per_step_plain"]
    out["ms_per_eval"] = extra / out["evals_per_step"] if out["evals_per_step"] > 0 else None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
