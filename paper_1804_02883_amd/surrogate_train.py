"""Training driver of the density surrogate.

Pairs (potentials -> exact densities) come from the library's exact GPU path:
seeded quenches (chi reading Q, initial noise amplitudes `sigmas`) on
256 x 256 grids, sampled every `every` steps, with the two model parameter
sets of the 256^2 and 1024x512 workloads (N = 32, f_A = 0.5,
phibar_P = 0.1 and N = 64, f_A = 0.3, phibar_P = 0.15).
Training runs entirely in the library's HIP kernels (forward, backward-data,
weight-gradient, Adam); this script only schedules them.

    python -m paper_1804_02883_amd.surrogate_train --out weights.npy
"""
import argparse
import json
import math
import sys
import time

import numpy as np

CH = [(5, 64), (64, 64), (64, 64), (64, 2)]


def init_weights(seed, phibar=0.05):
    """He-initialised layers; output bias at softplus^-1(phibar), small output weights."""
    rng = np.random.default_rng(seed)
    parts = []
    for l, (ci, co) in enumerate(CH):
        W = rng.standard_normal((9, ci, co)) * math.sqrt(2.0 / (9 * ci))
        b = np.zeros(co)
        if l == 3:
            W *= 0.1
            b[:] = math.log(math.expm1(phibar))
        parts += [W.ravel(), b]
    return np.concatenate(parts).astype(np.float32)


def param_sets(grid):
    from seeded_inputs import base_params
    return [
        dict(base_params(grid, grid, 32, 0.5, 0.1, "Q", 1e-5), density_mode=0),
        dict(base_params(grid, grid, 64, 0.3, 0.15, "Q", 1e-5), density_mode=0),
    ]


def schedule(steps, every, early, early_every):
    """Step counts between captures: every `early_every` steps up to step
    `early` (the fast relaxation right after the quench), then every `every`."""
    out = [early_every] * (early // early_every) if early_every else []
    out += [every] * ((steps - sum(out)) // every)
    return out


def generate(trainer, psets, runs, sched, slot0, log):
    """Runs each (parameter set, seed, sigma) quench and captures a pair after each schedule entry."""
    from paper_1804_02883_amd import Simulation
    slot = slot0
    for pi, seed, sigma in runs:
        sim = Simulation(psets[pi])
        sim.seed(int(seed), float(sigma))
        t0 = time.perf_counter()
        amp = []
        for k, gap in enumerate(sched):
            sim.step(gap)
            trainer.capture(slot, sim)
            slot += 1
            if (k + 1) % max(1, len(sched) // 4) == 0:
                phi = sim.densities()
                amp.append(round(float(np.max(np.abs(phi[0] - phi[0].mean()))), 5))
        sim.sync()
        log(dict(event="generated", pset=pi, seed=int(seed), sigma=sigma, pairs=len(sched),
                 seconds=round(time.perf_counter() - t0, 2), amp_phiA=amp))
        sim.close()
    return slot


def train(trainer, train_slots, val_slots, epochs, batch, lr, phi_scale, seed, log):
    rng = np.random.default_rng(seed)
    nb = len(train_slots) // batch
    total = epochs * nb
    it = 0
    for ep in range(epochs):
        perm = rng.permutation(train_slots)
        t0 = time.perf_counter()
        for b in range(nb):
            # cosine decay to 5% of the initial rate
            rate = lr * (0.05 + 0.95 * 0.5 * (1 + math.cos(math.pi * it / total)))
            trainer.train_step(perm[b * batch:(b + 1) * batch], phi_scale, rate)
            it += 1
        tl, te = trainer.last_loss()
        vl, ve = evaluate(trainer, val_slots, batch, phi_scale)
        log(dict(event="epoch", epoch=ep, train_loss=tl, train_max_err=te, val_loss=vl, val_max_err=ve,
                 seconds=round(time.perf_counter() - t0, 2)))


def evaluate(trainer, slots, batch, phi_scale):
    losses, mx = [], 0.0
    for i in range(0, len(slots), batch):
        s = slots[i:i + batch]
        l, e, _ = trainer.evaluate(s, phi_scale)
        losses.append(l * len(s))
        mx = max(mx, e)
    return sum(losses) / len(slots), mx


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--grid", type=int, default=256)
    ap.add_argument("--seeds", type=int, default=3, help="quenches per sigma, 256^2-workload parameters")
    ap.add_argument("--seeds1", type=int, default=1, help="quenches per sigma, 1024x512-workload parameters")
    ap.add_argument("--sigmas", default="0.03,0.05,0.08", help="initial noise amplitudes of the quenches")
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--every", type=int, default=25)
    ap.add_argument("--early", type=int, default=500)
    ap.add_argument("--early-every", type=int, default=5)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--phi-scale", type=float, default=0.1)
    ap.add_argument("--init-seed", type=int, default=0)
    ap.add_argument("--init", default=None, help="start from these weights (.npy)")
    ap.add_argument("--eval-steps", type=int, default=2000,
                    help="steps of the 512x512 quench compared plain vs surrogate after training (0: skip)")
    args = ap.parse_args(argv)

    import torch
    from paper_1804_02883_amd import Trainer
    torch.cuda.set_device(0)

    def log(d):
        print(json.dumps(d), flush=True)

    psets = param_sets(args.grid)
    sigmas = [float(x) for x in args.sigmas.split(",")]
    sched = schedule(args.steps, args.every, args.early, args.early_every)
    per = len(sched)
    train_runs = [(pi, 20000 + 1000 * pi + 100 * j + i, sg) for pi, ns in ((0, args.seeds), (1, args.seeds1))
                  for j, sg in enumerate(sigmas) for i in range(ns)]
    val_runs = [(0, 29999, sigmas[len(sigmas) // 2])]
    n_train = len(train_runs) * per
    n_val = len(val_runs) * per
    tr = Trainer(args.grid, args.grid, n_train + n_val, args.batch)
    t0 = time.perf_counter()
    end = generate(tr, psets, train_runs, sched, 0, log)
    generate(tr, psets, val_runs, sched, end, log)
    log(dict(event="data", train_pairs=n_train, val_pairs=n_val, seconds=round(time.perf_counter() - t0, 1)))
    w0 = np.load(args.init) if args.init else init_weights(args.init_seed)
    tr.set_weights(w0)
    train(tr, np.arange(n_train), np.arange(n_train, n_train + n_val), args.epochs, args.batch, args.lr,
          args.phi_scale, args.init_seed, log)
    w = tr.get_weights()
    np.save(args.out, w)
    log(dict(event="saved", path=args.out, params=int(w.size), seconds=round(time.perf_counter() - t0, 1)))
    tr.close()
    if args.eval_steps:
        from paper_1804_02883_amd.surrogate_eval import compare, error_trace
        from seeded_inputs import PRESETS
        cfg = PRESETS["cfg5q"]
        r = compare(dict(cfg["params"]), cfg["seed"], cfg["sigma"], w, args.eval_steps)
        log(dict(event="eval", workload="cfg5q", **r))
        tr_ = error_trace(dict(cfg["params"]), cfg["seed"], cfg["sigma"], w, args.eval_steps)
        log(dict(event="error_trace", workload="cfg5q", **tr_))


if __name__ == "__main__":
    sys.exit(main())
