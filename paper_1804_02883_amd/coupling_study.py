"""Runs with and without LB coupling from the same start (Sec. III: sigma(t)
and sigma_Delta(t)).  Library calls only.

    python -m paper_1804_02883_amd.coupling_study --preset cfg2 --chi Q --steps 20000 --every 1000

Two contexts share the seed and every parameter except couple_lb (1: the
flow advects the fields and the polymer force drives it; 0: pure EPD
diffusion, the LB still runs under the external force).  Every `every`
steps one JSON line: step, sigma of both runs, sigma_Delta between them,
the particle counts, and the wall time per step pair.
"""
import argparse
import json
import time


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--nx", type=int, default=256)
    ap.add_argument("--ny", type=int, default=256)
    ap.add_argument("--N", type=int, default=32)
    ap.add_argument("--fA", type=float, default=0.5)
    ap.add_argument("--phiP", type=float, default=0.1)
    ap.add_argument("--chi", default="Q", choices=["L", "Q"])
    ap.add_argument("--g", type=float, default=1e-5)
    ap.add_argument("--precision", type=int, default=1)
    ap.add_argument("--lb", default="bgk", choices=["bgk", "mrt"])
    ap.add_argument("--seed", type=int, default=1002)
    ap.add_argument("--sigma0", type=float, default=1e-3, help="initial noise amplitude")
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--every", type=int, default=200)
    args = ap.parse_args(argv)
    import torch
    from paper_1804_02883_amd import Simulation, mrt_gammas
    from seeded_inputs.presets import base_params
    torch.cuda.set_device(0)
    p = base_params(args.nx, args.ny, args.N, args.fA, args.phiP, args.chi, args.g, precision=args.precision)
    if args.lb == "mrt":
        gs, gb = mrt_gammas(1.0, 1.0, 1.0, p["dx"], p["dt"])
        p.update(lb_mrt=1, lb_gamma_s=gs, lb_gamma_b=gb, lb_gamma_g=0.0)
    runs = [Simulation(dict(p, couple_lb=1)), Simulation(dict(p, couple_lb=0))]
    for s in runs:
        s.seed(args.seed, args.sigma0)
    done = 0
    while done < args.steps:
        n = min(args.every, args.steps - done)
        t0 = time.perf_counter()
        for s in runs:
            s.step(n)
        for s in runs:
            s.sync()
        dt = (time.perf_counter() - t0) / n
        done += n
        oc, _, _ = runs[0].observables(0.5, max_particles=0)
        ou, _, _ = runs[1].observables(0.5, max_particles=0)
        print(json.dumps(dict(step=done, sigma_lb=oc["sigma"], sigma_nlb=ou["sigma"],
                              sigma_delta=runs[0].sigma_delta(runs[1]), particles_lb=oc["n_particles"],
                              particles_nlb=ou["n_particles"], y2p_lb=oc["y2p"], ms_per_step_pair=dt * 1e3)),
              flush=True)
    for s in runs:
        s.close()


if __name__ == "__main__":
    main()
