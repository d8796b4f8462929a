"""Nucleation statistics of one run (Sec. IV, nucleation stage): the particle
density n_p(t) and its maximum, and the nucleation events as (time, y) points
with y measured from the centre of the Poiseuille channel the nucleus sits in
(the paper plots events of both channels together).

    python -m paper_1804_02883_amd.nucleation_study --workload cfg5q --steps 20000 --every 100

With --replicas R the ensemble of R runs (seeds seed + r) advances in one
batch and n_p(t) is the ensemble average, as in the paper's figures.

The run starts from the workload's seeded noise; every --every steps the
library labels the particles (Phi_P >= 0.5) and reports those that are new
since the previous sample.  The body force acts along x with opposite signs
in the lower (y < ny/2) and upper half, so the channel centres are at y = ny/4
and 3 ny/4 (cell-centre coordinates).  Prints one JSON line.
"""
import argparse
import json
import sys
import time


def channel_offset(cy, ny, dx):
    """Distance (in R_G) of a centroid row from the centre of its channel, signed."""
    y = cy + 0.5
    centre = ny / 4.0 if y < ny / 2.0 else 3.0 * ny / 4.0
    return (y - centre) * dx


def paper_system(system):
    """The paper's parameter set (Sec. III): N = 17, A fraction 0.882, phibar_P = 0.1,
    kappa_H = 1.176, chi_AB = 1.05, chi_AS = 1.20, chi_BS = 0.75 (droplets) or -0.15
    (vesicles), D_A = D_B = D_S / N with D_S = 1."""
    return dict(n_contour=17, f_A=0.882, phi_P=0.1, kappa_H=1.176, chi_AB=1.05, chi_AS=1.20,
                chi_BS=0.75 if system == "droplet" else -0.15, D_A=1 / 17, D_B=1 / 17)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="cfg5q")
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--g", type=float, default=None, help="override the force amplitude (paper units)")
    ap.add_argument("--threshold", type=float, default=0.5)
    ap.add_argument("--system", choices=["droplet", "vesicle"], default=None,
                    help="the paper's parameter set of Sec. III on the workload's grid")
    ap.add_argument("--replicas", type=int, default=1, help="runs of the ensemble (seeds seed + r)")
    ap.add_argument("--nx", type=int, default=None)
    ap.add_argument("--ny", type=int, default=None)
    ap.add_argument("--tune-cache", default=None)
    args = ap.parse_args(argv)
    import torch
    from paper_1804_02883_amd import Batch, Simulation
    from seeded_inputs import PRESETS, preset
    torch.cuda.set_device(0)
    over = {} if args.g is None else dict(g=args.g)
    if args.nx:
        over["nx"] = args.nx
    if args.ny:
        over["ny"] = args.ny
    if args.system:
        over.update(paper_system(args.system))
    p = preset(args.workload, **over)
    cfg = PRESETS[args.workload]
    R = args.replicas
    if R == 1:
        sim = Simulation(p)
        sim.seed(cfg["seed"], cfg["sigma"])
        track = lambda r: sim.track_particles(args.threshold, max_events=1 << 16)  # noqa: E731
    else:
        # an ensemble: the same parameters, seeds seed + r, advanced together
        sim = Batch([p] * R)
        sim.seed([cfg["seed"] + r for r in range(R)], cfg["sigma"])
        track = lambda r: sim.track_particles(r, args.threshold, max_events=1 << 16)  # noqa: E731
    if args.tune_cache:
        sim.autotune(20, args.tune_cache)
    area = p["nx"] * p["ny"] * p["dx"] ** 2
    n_p, events = [], []
    first = [None] * R
    t_track = 0.0
    done = 0
    while done <= args.steps:
        sim.sync()
        t = done * p["dt"]
        t0 = time.perf_counter()
        counts = []
        for r in range(R):
            obs, ev, n_ev = track(r)
            counts.append(obs["n_particles"])
            if n_ev and first[r] is None:
                first[r] = t
            for e in ev:
                events.append((t, channel_offset(e["centroid"][1], p["ny"], p["dx"]), e["area"]))
        t_track += time.perf_counter() - t0
        n_p.append((t, sum(counts) / (R * area)))
        if done == args.steps:
            break
        k = min(args.every, args.steps - done)
        sim.step(k)
        done += k
        if len(n_p) % 50 == 0:
            print(f"step {done}: {sum(counts)} particles over {R} runs, {len(events)} events so far",
                  file=sys.stderr, flush=True)
    sim.close()
    print(json.dumps(dict(workload=args.workload, system=args.system, replicas=R, steps=args.steps,
                          every=args.every, g=p["g"], n_p_max=max(v for _, v in n_p), first_nucleation=first,
                          n_p=n_p, events=events, ms_per_track=1e3 * t_track / (len(n_p) * R))), flush=True)


if __name__ == "__main__":
    main()
