"""Batched replicas (uneven grids, drives, A fractions, seeds) through the C ABI.

Each replica of a batch must equal, bit for bit, the same replica run alone
(same kernels and launch shapes), and FP64 replicas must match the oracle.
"""
import sys

import numpy as np
import pytest

from oracle import epdlb_oracle as O
from seeded_inputs import initial_omega, replica_manifest
from seeded_inputs.presets import base_params

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_batch_equals_single_runs_bitwise():
    _need_gpu()
    from paper_1804_02883_amd import Batch, Simulation
    specs = [(64, 64, 0.3, 2e-5, 11), (128, 64, 0.5, 0.0, 12), (64, 64, 0.5, 5e-5, 13),
             (32, 32, 0.3, 1e-5, 14), (128, 64, 0.3, 3e-5, 15)]
    params = [base_params(nx, ny, 32, fA, 0.1, "L", g) for nx, ny, fA, g, _ in specs]
    say(f"[batch] {len(params)} replicas, shapes {[(p['nx'], p['ny']) for p in params]}")
    b = Batch(params)
    assert b.info() == (5, sum(p["nx"] * p["ny"] for p in params))
    b.seed([s[-1] for s in specs], 1e-3)
    b.step(7)
    b.sync()
    for r, (p, s) in enumerate(zip(params, specs)):
        sim = Simulation(p)
        sim.seed(s[-1], 1e-3)
        sim.step(7)
        sim.sync()
        assert np.array_equal(b.densities(r), sim.densities()), r
        assert np.array_equal(b.fields(r), sim.fields()), r
        rb, ub = b.velocity(r)
        rs, us = sim.velocity()
        assert np.array_equal(ub, us), r
        assert b.diag(r)["Q_P"] == sim.diag()["Q_P"]
        sim.close()
    b.close()


def test_batch_fp64_vs_oracle():
    _need_gpu()
    from paper_1804_02883_amd import Batch
    params = [base_params(32, 32, 16, 0.3, 0.1, "L", 2e-4, precision=0),
              base_params(64, 32, 16, 0.5, 0.1, "Q", 1e-4, precision=0),
              base_params(32, 32, 16, 0.5, 0.1, "L", 0.0, precision=0)]
    params[2].update(chi_AB=params[0]["chi_AB"], chi_AS=params[0]["chi_AS"])
    params[1].update(chi_AB=params[0]["chi_AB"], chi_AS=params[0]["chi_AS"])
    say("[batch fp64] 3 replicas vs oracle, 20 steps")
    b = Batch(params)
    seeds = [21, 22, 23]
    b.seed(seeds, 1e-3)
    b.step(20)
    b.sync()
    for r, p in enumerate(params):
        s = O.init_state(p, initial_omega(p["nx"], p["ny"], seeds[r], 1e-3))
        for _ in range(20):
            s = O.step(s, p)
        phi = b.densities(r)
        for I in range(3):
            assert np.max(np.abs(phi[I] - s["phi"][I])) < 1e-10 * np.max(np.abs(s["phi"][I])), (r, I)
        rho, u = b.velocity(r)
        assert np.max(np.abs(u - s["u"])) < 1e-10 * np.max(np.abs(s["u"])) + 1e-14, r
    b.close()


def test_batch_rejects_mismatched_models():
    _need_gpu()
    from paper_1804_02883_amd import Batch, EpdlbError
    a = base_params(32, 32, 16, 0.5, 0.1)
    c = base_params(32, 32, 32, 0.5, 0.1)
    with pytest.raises(EpdlbError):
        Batch([a, c])
    # the batch runs the exact densities only
    with pytest.raises(EpdlbError):
        Batch([a, dict(a, density_mode=1)])


def test_cfg4_manifest_two_steps():
    """The 64-replica workload: every replica advances and two of them match
    their single runs bit for bit after 2 steps."""
    _need_gpu()
    from paper_1804_02883_amd import Batch, Simulation
    man = replica_manifest()
    params = [m["params"] for m in man]
    say(f"[cfg4] 64 replicas, {sum(p['nx'] * p['ny'] for p in params)} sites")
    b = Batch(params)
    b.seed([m["seed"] for m in man], 1e-3)
    b.step(2)
    b.sync()
    for r in (0, 37):
        sim = Simulation(params[r])
        sim.seed(man[r]["seed"], 1e-3)
        sim.step(2)
        sim.sync()
        assert np.array_equal(b.densities(r), sim.densities()), r
        sim.close()
        phi = b.densities(r)
        assert abs(phi.sum(axis=0).mean() - 1) < 1e-6
    b.close()


def _wells(ny, nx, centres, depth=0.2):
    """Potentials with wells that gather the polymer into disks (Phi_P >= 0.5)."""
    yy, xx = np.mgrid[0:ny, 0:nx]
    blob = np.zeros((ny, nx))
    for cy, cx, r in centres:
        d2 = ((yy - cy + ny / 2) % ny - ny / 2) ** 2 + ((xx - cx + nx / 2) % nx - nx / 2) ** 2
        blob = np.maximum(blob, (d2 <= r * r).astype(float))
    return np.stack([-depth * blob, -depth * blob, depth * blob])


def test_batch_observables_and_tracking_per_replica():
    """Replicas of one group (two 64x64) and of another (128x64), FP64: each
    replica's particles match the oracle on its stored densities; tracking
    keeps one sample per replica (a reset of one replica leaves the others)."""
    _need_gpu()
    from oracle import observables_oracle as B
    from paper_1804_02883_amd import Batch
    params = [base_params(64, 64, 16, 0.5, 0.1, "L", 1e-5, precision=0),
              base_params(64, 64, 16, 0.5, 0.1, "L", 1e-5, precision=0),
              base_params(128, 64, 16, 0.5, 0.1, "L", 1e-5, precision=0)]
    wells = [[(16, 16, 5), (40, 44, 4)], [(10, 50, 4), (30, 20, 6), (52, 8, 3)], [(20, 100, 5), (44, 30, 4)]]
    say("[batch] observables and tracking, 3 replicas in 2 groups")
    b = Batch(params)
    b.seed([1, 2, 3], 1e-3)
    for r, (p, wl) in enumerate(zip(params, wells)):
        b.set_fields(r, _wells(p["ny"], p["nx"], wl))
    prev = []
    for r, p in enumerate(params):
        phiP = b.densities(r)[0] + b.densities(r)[1]
        obs, parts, lab = b.observables(r, labels=True)
        table = B.particle_table(phiP)
        assert np.array_equal(lab.astype(np.int64), B.label_particles(phiP)), r
        assert obs["n_particles"] == len(table) == len(wells[r]) == len(parts), r
        for g, t in zip(parts, table):
            assert (g["label"], g["area"]) == (t["label"], t["area"])
            assert abs(g["content"] - t["content"]) <= 1e-12 * t["content"]
        assert abs(obs["sigma"] - B.sigma(b.densities(r), p["phi_P"])) <= 1e-12 * obs["sigma"]
        # first tracking sample of each replica: every particle is new
        _, ev, n_ev = b.track_particles(r)
        assert n_ev == len(table) and [e["label"] for e in ev] == [t["label"] for t in table]
        prev.append(phiP)
    b.step(5)
    b.sync()
    b.track_reset(1)
    for r in range(3):
        phiP = b.densities(r)[0] + b.densities(r)[1]
        _, ev, n_ev = b.track_particles(r)
        ref = B.nucleation_events(None if r == 1 else prev[r], phiP)
        assert n_ev == len(ref) == (len(wells[r]) if r == 1 else 0), r
        assert [e["label"] for e in ev] == [t["label"] for t in ref]
    b.close()
