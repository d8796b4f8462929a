"""Runs with and without LB coupling from the same start (Sec. III): sigma of
both runs and sigma_Delta between them, GPU against the FP64 oracle."""
import sys

import numpy as np
import pytest

from oracle import epdlb_oracle as O
from oracle import observables_oracle as B
from seeded_inputs import initial_omega, preset

pytestmark = pytest.mark.gpu


def test_sigma_delta_coupled_vs_uncoupled_fp64():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1804_02883_amd import Simulation
    print("[coupling] 32x32 FP64, 20 steps, lattice drive 1e-4", flush=True)
    sys.stdout.flush()
    base = preset("cfg1", g=1e-4, g_units=1)
    w0 = initial_omega(32, 32, 1001, 1e-2)
    sims, refs = [], []
    for couple in (1, 0):
        p = dict(base, couple_lb=couple)
        s = Simulation(p)
        s.set_fields(w0)
        sims.append(s)
        refs.append((p, O.init_state(p, w0)))
    for chunk in (5, 15):
        for s in sims:
            s.step(chunk)
        for k, (p, st) in enumerate(refs):
            for _ in range(chunk):
                st = O.step(st, p)
            refs[k] = (p, st)
        for s in sims:
            s.sync()
        phiP = [r[1]["phi"][0] + r[1]["phi"][1] for r in refs]
        sd_ref = B.sigma_delta(phiP[0], phiP[1])
        sd = sims[0].sigma_delta(sims[1])
        assert sd_ref > 1e-9  # the flow changes the densities measurably
        # both runs match the oracle to 1e-10 relative on densities of size 0.05
        assert abs(sd - sd_ref) <= 1e-10 * 0.1 + 1e-6 * sd_ref, (chunk, sd, sd_ref)
        for s, (p, st) in zip(sims, refs):
            o, _, _ = s.observables(0.5, max_particles=0)
            ref = B.sigma(st["phi"], p["phi_P"])
            assert abs(o["sigma"] - ref) <= 1e-10 * 0.1 + 1e-9 * ref
    for s in sims:
        s.close()
