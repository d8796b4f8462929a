"""Run hybrid steps of a named workload and print its diagnostics (library calls
only); a short driver for profiler runs.

    python -m paper_1804_02883_amd.run_steps --workload cfg5q --path surrogate --steps 60
    python -m paper_1804_02883_amd.run_steps --workload cfg3 --path plain --steps 4

--path surrogate loads the committed network weights and uses the network from
the first step on (no error gate: every fallback_every-th step is exact).
--tune-cache names the autotuner cache to read (default: the committed one).
"""
import argparse
import json
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="cfg5q")
    ap.add_argument("--path", default="surrogate", choices=["surrogate", "plain"])
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--tune-cache", default=os.path.join(PKG, "tune", "gfx950.txt"))
    args = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    from paper_1804_02883_amd import Simulation
    from seeded_inputs import PRESETS
    cfg = PRESETS[args.workload]
    sur = args.path == "surrogate"
    p = dict(cfg["params"], density_mode=1 if sur else 0, fallback_every=50, check_every=10, resid_tol=1e-3,
             err_tol=0.0)
    sim = Simulation(p)
    if sur:
        sim.surrogate_set_weights(np.load(os.path.join(PKG, "weights", "surrogate_q.npy")))
    sim.seed(cfg["seed"], cfg["sigma"])
    sim.autotune(20, args.tune_cache)
    sim.step(args.steps)
    sim.sync()
    d = sim.diag()
    sim.close()
    print(json.dumps(dict(workload=args.workload, path=args.path, steps=args.steps, Q_P=d["Q_P"],
                          n_exact=d["n_exact"])), flush=True)


if __name__ == "__main__":
    main()
