"""GPU time of one density evaluation on a 3D grid (library calls only).

    python -m paper_1804_02883_amd.epd3_timing --n 128 --N 32 --reps 5

Box n^3, FP32 planes (FP64 sums), f_A = 0.3, phibar_P = 0.15, seeded
potentials 0.2 xi.  An evaluation runs both chains over N contour steps, each
step 5 FFT launches (the half-step factors ride on the two x passes), plus
the gauge and partition-function sums and the density kernel.  Prints
one JSON line: ms per evaluation (events on the stream around `reps`
evaluations), `value` in site contour steps per second (n^3 sites x 2N
steps), and the HBM roofline of the FFT kernel: the mean algorithmic bytes
of its launches over their mean duration, each launch timed from its own
start to its end in one further evaluation.
"""
import argparse
import json

import numpy as np


def measure(n=128, N=32, reps=5, precision=1):
    import torch
    from paper_1804_02883_amd import Densities3D
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        d = Densities3D(n, n, n, N, 0.3, 0.15, 1.0, 1.0 / 3.0, precision)
    w = 0.2 * np.random.default_rng(5).standard_normal((3, n, n, n))
    d.densities(w)  # uploads the potentials and warms up
    ms = d.time(reps)
    fft_ms, fft_launches = d.profile()
    d.close()
    sites = n ** 3
    es = 4 if precision else 8
    # per FFT launch: the complex plane in and out (16 B per site in FP32); the two
    # x passes of a contour step read or write q, wA, wB (12 B) in place of one
    # complex plane, so a step's 5 launches move 2 * 20 + 3 * 16 B per site (FP32)
    alg = sites * es * (2 * 5 + 3 * 4) / 5
    avg = fft_ms / fft_launches
    achieved = alg / (avg * 1e-3) / 1e9
    return dict(workload=f"densities3d_{n}^3_N{N}", precision="f32" if precision else "f64", ms_per_eval=ms,
                value=sites * 2 * N / (ms * 1e-3), unit="site contour steps/s",
                launches_per_eval=2 * N * 5 + 2 + 5 * 2 + 1,
                roofline=dict(bound="hbm", kernel="p3_fft", achieved=achieved, peak=8000.0, unit="GB/s",
                              frac=achieved / 8000.0, algorithmic_bytes_per_launch=alg, avg_launch_us=avg * 1e3,
                              traffic=None))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--N", type=int, default=32)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--precision", type=int, default=1, choices=[0, 1])
    args = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    print(json.dumps(measure(args.n, args.N, args.reps, args.precision)), flush=True)


if __name__ == "__main__":
    main()
