"""Timing of the observables on a synthetic particle field (library calls only).

    python -m paper_1804_02883_amd.obs_timing --nx 1024 --ny 512 --reps 20

The densities are a smooth random field (seeded) with many particles above
Phi_P = 0.5, written with set_state; each call labels and measures them.
Prints one JSON line: host wall time per call and the particle count.
"""
import argparse
import json
import time

import numpy as np


def field(ny, nx, seed, width=100.0):
    rng = np.random.default_rng(seed)
    k2 = np.add.outer(np.fft.fftfreq(ny) ** 2, np.fft.fftfreq(nx) ** 2)
    f = np.real(np.fft.ifft2(np.fft.fft2(rng.standard_normal((ny, nx))) * np.exp(-k2 * width)))
    f = (f - f.mean()) / f.std()
    return 0.3 + 0.25 * f


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--nx", type=int, default=1024)
    ap.add_argument("--ny", type=int, default=512)
    ap.add_argument("--precision", type=int, default=1)
    ap.add_argument("--reps", type=int, default=20)
    args = ap.parse_args(argv)
    import torch
    from paper_1804_02883_amd import Simulation
    from seeded_inputs import preset
    torch.cuda.set_device(0)
    p = preset("cfg1", nx=args.nx, ny=args.ny, precision=args.precision)
    phiP = field(args.ny, args.nx, 7)
    phi = np.stack([0.6 * phiP, 0.4 * phiP, 1 - phiP])
    zeros = np.zeros((3, args.ny, args.nx))
    u = np.zeros((2, args.ny, args.nx))
    w9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)[:, None, None] * np.ones((9, args.ny, args.nx))
    sim = Simulation(p)
    sim.set_state(zeros, phi, w9, u)
    obs, _, _ = sim.observables(0.5, max_particles=0)  # allocates the scratch
    t0 = time.perf_counter()
    for _ in range(args.reps):
        obs, parts, _ = sim.observables(0.5, max_particles=0)
    dt = (time.perf_counter() - t0) / args.reps
    print(json.dumps(dict(nx=args.nx, ny=args.ny, precision=args.precision, ms_per_call=dt * 1e3,
                          n_particles=obs["n_particles"], n_wrapping=obs["n_wrapping"], sigma=obs["sigma"])),
          flush=True)
    sim.close()


if __name__ == "__main__":
    main()
