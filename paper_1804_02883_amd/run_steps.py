"""Run hybrid steps of a named workload and print its diagnostics (library calls
only); a short driver for profiler runs.

    python -m paper_1804_02883_amd.run_steps --workload cfg5q --path surrogate --steps 60
    python -m paper_1804_02883_amd.run_steps --workload cfg3 --path plain --steps 4
    python -m paper_1804_02883_amd.run_steps --workload cfg3 --path invert --steps 5
    python -m paper_1804_02883_amd.run_steps --workload cfg3 --path observables --steps 20

--path surrogate loads the committed network weights and uses the network from
the first step on (no error gate: every fallback_every-th step is exact).
--path invert runs FP64 steps whose stage 1 is the Phi -> omega inversion with
the Fletcher-Reeves iteration (App. C), diagonally preconditioned, under a
body force of 5e-7 lattice units, from a seeded noisy omega (sigma 0.05).
--path observables writes a seeded smooth particle field of the workload's
size (FP32) with set_state and runs the observables (labels, particle
moments, sigma) --steps times.
--tune-cache names the autotuner cache to read (default: the committed one).
Prints one JSON line, with the host wall time per step of the run (after the
seed), which for --path invert includes the iteration's host reads.
"""
import argparse
import json
import os
import time

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))


def particle_field(ny, nx, seed, width=100.0):
    """A smooth seeded field around 0.3 with many regions above 0.5."""
    rng = np.random.default_rng(seed)
    k2 = np.add.outer(np.fft.fftfreq(ny) ** 2, np.fft.fftfreq(nx) ** 2)
    f = np.real(np.fft.ifft2(np.fft.fft2(rng.standard_normal((ny, nx))) * np.exp(-k2 * width)))
    f = (f - f.mean()) / f.std()
    return 0.3 + 0.25 * f


def run_observables(cfg, reps):
    from paper_1804_02883_amd import Simulation
    p = dict(cfg["params"], precision=1)
    ny, nx = p["ny"], p["nx"]
    phiP = particle_field(ny, nx, 7)
    phi = np.stack([0.6 * phiP, 0.4 * phiP, 1 - phiP])
    w9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)[:, None, None] * np.ones((9, ny, nx))
    sim = Simulation(p)
    sim.set_state(np.zeros((3, ny, nx)), phi, w9, np.zeros((2, ny, nx)))
    obs = None
    for _ in range(reps):
        obs, _, _ = sim.observables(0.5, max_particles=0)
    sim.close()
    return dict(n_particles=obs["n_particles"], sigma=obs["sigma"])


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="cfg5q")
    ap.add_argument("--path", default="surrogate", choices=["surrogate", "plain", "invert", "observables"])
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--tune-cache", default=os.path.join(PKG, "tune", "gfx950.txt"))
    args = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    from paper_1804_02883_amd import Simulation
    from seeded_inputs import PRESETS, initial_omega
    cfg = PRESETS[args.workload]
    if args.path == "observables":
        r = run_observables(cfg, args.steps)
        print(json.dumps(dict(workload=args.workload, path=args.path, calls=args.steps, **r)), flush=True)
        return
    sur = args.path == "surrogate"
    p = dict(cfg["params"], density_mode=1 if sur else 0, fallback_every=50, check_every=10, resid_tol=1e-3,
             err_tol=0.0)
    if args.path == "invert":
        p.update(precision=0, g=5e-7, g_units=1, cg_invert=1, cg_precond=1)
    sim = Simulation(p)
    if sur:
        sim.surrogate_set_weights(np.load(os.path.join(PKG, "weights", "surrogate_q.npy")))
    if args.path == "invert":
        sim.set_fields(initial_omega(p["nx"], p["ny"], cfg["seed"], 0.05))
    else:
        sim.seed(cfg["seed"], cfg["sigma"])
    if args.path != "invert":  # the FP64 inversion runs the default launch shapes
        sim.autotune(20, args.tune_cache)
    sim.sync()
    t0 = time.perf_counter()
    sim.step(args.steps)
    sim.sync()
    wall = (time.perf_counter() - t0) / max(args.steps, 1)
    d = sim.diag()
    out = dict(workload=args.workload, path=args.path, steps=args.steps, ms_per_step_wall=1e3 * wall, Q_P=d["Q_P"],
               n_exact=d["n_exact"])
    if args.path == "invert":
        _, tot = sim.cg_stats()
        out.update(inversions=tot["inversions"], iterations=tot["iterations"], evals=tot["evals"])
    sim.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
