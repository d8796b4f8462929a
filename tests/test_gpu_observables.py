"""GPU parity of the observables (sigma, Y_2^P, particles, sigma_Delta; Sec. III
and IV) through the C ABI, against the observables oracle on the same stored
densities.

Phi_P = Phi_A + Phi_B is formed in the storage precision on both sides, so
the threshold decides the same sites: labels, counts, areas and wrap flags
must agree exactly; FP64 sums (content, centroid, tensor, R, c_rel, sigma,
Y_2^P) to 1e-12 relative (summation order differs).
"""
import sys

import numpy as np
import pytest

from oracle import observables_oracle as B
from seeded_inputs import preset

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _sim(p):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1804_02883_amd import Simulation
    return Simulation(p)


def _blobs(ny, nx, seed, frac=0.5):
    """Smooth periodic random field scaled so that about `frac` of the peaks exceed 0.5."""
    rng = np.random.default_rng(seed)
    k2 = np.add.outer(np.fft.fftfreq(ny) ** 2, np.fft.fftfreq(nx) ** 2)
    width = min(400.0, (min(nx, ny) / 4.0) ** 2)  # correlation length ~ a few sites on small grids
    f = np.real(np.fft.ifft2(np.fft.fft2(rng.standard_normal((ny, nx))) * np.exp(-k2 * width)))
    f = (f - f.mean()) / f.std()
    return 0.3 + 0.25 * f * frac * 2


def _state(p, phiP):
    ny, nx = phiP.shape
    phi = np.stack([0.6 * phiP, 0.4 * phiP, 1 - phiP])
    w = np.zeros((3, ny, nx))
    u = np.zeros((2, ny, nx))
    from oracle import epdlb_oracle as O
    f = O.lb_equilibrium(np.ones((ny, nx)), u)
    return w, phi, f, u


def _stored_phiP(sim, prec):
    phi = sim.densities()
    if prec == 0:
        return phi[0] + phi[1]
    return (phi[0].astype(np.float32) + phi[1].astype(np.float32)).astype(np.float64)


def _compare(sim, p, prec, phiP_ref_in=None):
    obs, parts, lab = sim.observables(0.5, max_particles=p["nx"] * p["ny"], labels=True)
    phiP = _stored_phiP(sim, prec)
    ref_lab = B.label_particles(phiP, 0.5)
    assert np.array_equal(lab.astype(np.int64), ref_lab)
    table = B.particle_table(phiP, 0.5)
    assert obs["n_particles"] == len(table) == len(parts)
    assert obs["n_wrapping"] == sum(t["wraps"] for t in table)
    for g, r in zip(parts, table):
        assert (g["label"], g["area"], g["wraps"]) == (r["label"], r["area"], r["wraps"])
        assert abs(g["content"] - r["content"]) <= 1e-12 * r["content"]
        if not r["wraps"]:
            scale = max(r["R"] ** 2, 1e-300)
            assert np.max(np.abs(np.array(g["G"]) - np.array(r["G"]))) <= 1e-12 * max(scale, 1.0)
            assert abs(g["R"] - r["R"]) <= 1e-12 * max(r["R"], 1.0)
            assert abs(g["c_rel"] - r["c_rel"]) <= 1e-10
            dc = np.abs(np.array(g["centroid"]) - np.array(r["centroid"]))
            dc = np.minimum(dc, np.array([p["nx"], p["ny"]]) - dc)
            assert np.max(dc) <= 1e-10
    s_ref = np.mean(np.abs(phiP - p["phi_P"]))
    assert abs(obs["sigma"] - s_ref) <= 1e-12 * s_ref
    y_ref = B.y2p(phiP, p["phi_P"])
    assert abs(obs["y2p"] - y_ref) <= 1e-12 * y_ref
    return obs


@pytest.mark.parametrize("nx,ny,prec,seed", [(32, 16, 0, 1), (64, 64, 0, 2), (256, 128, 1, 3),
                                             (1024, 32, 1, 4), (128, 256, 0, 5)])
def test_particles_vs_oracle(nx, ny, prec, seed):
    say(f"[observables] {nx}x{ny} prec={prec} seed={seed}")
    p = preset("cfg1", nx=nx, ny=ny, precision=prec)
    phiP = _blobs(ny, nx, seed)
    sim = _sim(p)
    sim.set_state(*_state(p, phiP))
    obs = _compare(sim, p, prec)
    assert obs["n_particles"] >= 2
    sim.close()


def test_degenerate_fields():
    """No particle; one particle covering the grid (wrapping); a checkerboard (the
    largest particle count, n/2); a list shorter than the particle count."""
    say("[observables] degenerate")
    nx, ny = 32, 16
    p = preset("cfg1", nx=nx, ny=ny, precision=0)
    sim = _sim(p)
    for phiP, n_exp in ((np.full((ny, nx), 0.1), 0), (np.full((ny, nx), 0.7), 1),
                        (np.where(np.add.outer(np.arange(ny), np.arange(nx)) % 2 == 0, 0.8, 0.2), nx * ny // 2)):
        sim.set_state(*_state(p, phiP))
        obs = _compare(sim, p, 0)
        assert obs["n_particles"] == n_exp
    obs, parts, _ = sim.observables(0.5, max_particles=5)
    assert obs["n_particles"] == nx * ny // 2 and [q["label"] for q in parts] == [0, 2, 4, 6, 8]
    obs0, parts0, _ = sim.observables(0.5, max_particles=0)
    assert parts0 == [] and obs0["n_particles"] == nx * ny // 2
    sim.close()


def test_sigma_delta_two_contexts():
    say("[observables] sigma_delta")
    nx, ny = 64, 32
    for prec in (0, 1):
        p = preset("cfg1", nx=nx, ny=ny, precision=prec)
        a, b = _sim(p), _sim(p)
        a.set_state(*_state(p, _blobs(ny, nx, 11)))
        b.set_state(*_state(p, _blobs(ny, nx, 12)))
        pa, pb = _stored_phiP(a, prec), _stored_phiP(b, prec)
        ref = B.sigma_delta(pa, pb)
        got = a.sigma_delta(b)
        assert abs(got - ref) <= 1e-12 * ref, prec
        assert a.sigma_delta(a) == 0.0
        a.close()
        b.close()


def test_observables_after_steps():
    """On a simulated state (cfg1, 20 hybrid steps): sigma and Y_2^P against the oracle."""
    say("[observables] cfg1 after 20 steps")
    from seeded_inputs import initial_omega
    p = preset("cfg1")
    sim = _sim(p)
    sim.set_fields(initial_omega(32, 32, 1001, 1e-3))
    sim.step(20)
    sim.sync()
    _compare(sim, p, 0)
    sim.close()


def _disk(ny, nx, cy, cx, r, inside=0.8, outside=0.1):
    yy, xx = np.mgrid[0:ny, 0:nx]
    d2 = ((yy - cy + ny / 2) % ny - ny / 2) ** 2 + ((xx - cx + nx / 2) % nx - nx / 2) ** 2
    return np.where(d2 <= r * r, inside, outside)


@pytest.mark.parametrize("prec", [0, 1])
def test_nucleation_tracking_vs_oracle(prec):
    """A sequence of hand-built samples (set_state keeps the tracking sample):
    first sample, one kept + two new + one vanished, a merge, a jump, a reset;
    the new particles agree with the oracle's events on the stored densities."""
    say(f"[tracking] 64x32 prec={prec}")
    nx, ny = 64, 32
    p = preset("cfg1", nx=nx, ny=ny, precision=prec)
    d = lambda cy, cx, r: _disk(ny, nx, cy, cx, r)  # noqa: E731
    samples = [
        np.maximum(d(8, 8, 3), d(20, 40, 3)),
        np.maximum.reduce([d(8, 9, 3), d(26, 4, 2), d(4, 52, 2.5)]),
        np.maximum.reduce([d(8, 9, 3), d(8, 14, 3), d(4, 52, 2.5), d(26, 4, 2)]),
        np.maximum(d(8, 9, 3), d(20, 30, 3)),
    ]
    sim = _sim(p)
    prev = None
    counts = []
    for k, phiP in enumerate(samples):
        sim.set_state(*_state(p, phiP))
        obs, ev, n_ev = sim.track_particles(0.5)
        cur = _stored_phiP(sim, prec)
        ref = B.nucleation_events(prev, cur)
        assert n_ev == len(ev) == len(ref), k
        for g, r in zip(ev, ref):
            assert (g["label"], g["area"]) == (r["label"], r["area"]), k
            assert abs(g["content"] - r["content"]) <= 1e-12 * r["content"]
            assert np.max(np.abs(np.array(g["centroid"]) - np.array(r["centroid"]))) <= 1e-10
        assert obs["n_particles"] == len(B.particle_table(cur))
        counts.append(n_ev)
        prev = cur
    assert counts == [2, 2, 0, 1]
    # a truncated event list still reports the count
    sim.track_reset()
    obs, ev, n_ev = sim.track_particles(0.5, max_events=1)
    assert n_ev == obs["n_particles"] == 2 and len(ev) == 1 and ev[0]["label"] == B.particle_table(prev)[0]["label"]
    # set_fields starts a new run: every particle counts again
    sim.set_fields(np.zeros((3, ny, nx)))
    obs, ev, n_ev = sim.track_particles(0.5)
    assert n_ev == obs["n_particles"] == 0
    sim.close()
