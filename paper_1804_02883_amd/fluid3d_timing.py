"""Throughput and HBM roofline of the three-dimensional D3Q19 fluid (library
calls only).

    python -m paper_1804_02883_amd.fluid3d_timing --n 256 --steps 40

Box n^3 (periodic), FP32 deviations, tau = 0.8, started from the equilibrium
of a seeded random velocity field (standard deviation 1e-3) under a seeded
random force field (standard deviation 1e-5); BGK, or with --mrt the
multi-relaxation collision.  A step is one launch; the last
launch of a run also stores rho and u.  Prints one JSON line:
`value` site-updates/s over `steps` steps timed with events on the fluid's
stream, and `roofline` of the step kernel: algorithmic bytes per launch (per
site 19 populations read and 19 written plus the 3 force components)
over the mean duration of the launches that store no moments, each timed
from its own start to its end.
"""
import argparse
import json

import numpy as np

HBM_PEAK_GBS = 8000.0


def bytes_per_site(precision):
    return (19 * 2 + 3) * (4 if precision else 8)


def measure(n=256, steps=40, precision=1, tau=0.8, seed=3, mrt=None):
    import torch
    from paper_1804_02883_amd import Fluid3D
    # a stream of its own (default priority), so that the events below are
    # recorded on the stream the library launches on
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        fl = Fluid3D(n, n, n, tau, precision)
    assert fl.stream.cuda_stream == stream.cuda_stream != 0
    if mrt is not None:
        fl.set_collision(1, *mrt)
    sites = n ** 3
    rng = np.random.default_rng(seed)
    fl.set_equilibrium(None, 1e-3 * rng.standard_normal(3 * sites))
    fl.set_force(1e-5 * rng.standard_normal(3 * sites))
    fl.profile(5)  # warm-up
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    fl.sync()
    t0.record(fl.stream)
    fl.step(steps)
    t1.record(fl.stream)
    t1.synchronize()
    ms = t0.elapsed_time(t1) / steps
    launches = fl.profile(max(steps, 2))
    avg = float(np.mean(launches[:-1]))
    b = sites * bytes_per_site(precision)
    achieved = b / avg / 1e6
    fl.close()
    return dict(workload=f"fluid3d_{n}^3", n=n, precision="f32" if precision else "f64",
                collision="bgk" if mrt is None else "mrt", tau=tau, gammas=mrt,
                value=sites / (ms * 1e-3), unit="site-updates/s", ms_per_step=ms,
                roofline=dict(bound="hbm", kernel="lb3", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                              frac=achieved / HBM_PEAK_GBS, algorithmic_bytes_per_launch=b,
                              avg_launch_us=avg * 1e3))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--precision", type=int, default=1, choices=[0, 1])
    ap.add_argument("--mrt", type=float, nargs=3, default=None, metavar=("GAMMA_S", "GAMMA_B", "GAMMA_G"),
                    help="the multi-relaxation collision with these factors (default: BGK at tau)")
    args = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    print(json.dumps(measure(args.n, args.steps, args.precision, mrt=args.mrt)), flush=True)


if __name__ == "__main__":
    main()
