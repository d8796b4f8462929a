"""GPU parity of the Phi -> omega inversion (App. C, comments 1-3) through the
C ABI, against the oracle's Fletcher-Reeves iteration on the same inputs.

Both sides iterate in FP64 from the same start with the same rules, so the
starting residual agrees to rounding and the iteration counts to within one or
two (a run that ends just above or below the tolerance).  The solution is
unique up to one constant per field, and every direction has zero mean per
field (the totals of Phi and Phi~ agree), so omega is compared directly:
both sides stop within N_tr = 1e-8 (RMS over the three fields) of Phi~, which
bounds their potentials' difference by the inverse curvature times that
residual (1e-5 here); the densities that follow from them agree to 1e-7.
"""
import sys

import numpy as np
import pytest

from oracle import epdlb_oracle as O
from seeded_inputs import initial_omega, preset

pytestmark = pytest.mark.gpu


def _sim(p):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1804_02883_amd import Simulation
    return Simulation(p)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rms(a, b):
    n = a.shape[-1] * a.shape[-2]
    return float(np.sqrt(np.sum((a - b) ** 2) / n))


@pytest.mark.parametrize("nx,ny,N,fA,pc", [(32, 32, 16, 0.5, 0), (64, 32, 8, 0.3, 0), (32, 64, 24, 0.7, 0),
                                            (32, 32, 16, 0.5, 1), (64, 64, 32, 0.3, 1)])
def test_invert_vs_oracle(nx, ny, N, fA, pc):
    say(f"[invert] {nx}x{ny} N={N} f_A={fA} FP64 precond={pc}")
    p = preset("cfg1", nx=nx, ny=ny, n_contour=N, f_A=fA, cg_precond=pc)
    w_star = np.array(initial_omega(nx, ny, 2000 + nx + ny, 0.05))
    phi_star = O.densities(w_star, p)["phi"]
    rng = np.random.default_rng(nx * ny + N)
    seed = w_star + 0.02 * rng.standard_normal(w_star.shape)
    ref = O.invert_densities(phi_star, seed, p, tol=1e-8, max_iter=1000, precond=pc)
    sim = _sim(p)
    sim.set_fields(seed)
    got = sim.invert_densities(phi_star, max_iter=1000, tol=1e-8)
    say(f"  gpu iters {got['iters']} evals {got['evals']} resid {got['resid']:.2e}; "
        f"oracle iters {ref['iters']} resid {ref['resid']:.2e}")
    assert abs(got["resid0"] / ref["resid0"] - 1) < 1e-10
    assert got["converged"] and ref["converged"] and got["resid"] < 1e-8
    assert abs(got["iters"] - ref["iters"]) <= 2 and got["restarts"] == ref["restarts"] == 0
    assert got["evals"] == 2 * got["iters"] + 1
    w = sim.fields()
    phi = sim.densities()
    assert np.max(np.abs(w - ref["omega"])) < 1e-5
    # the densities the library now holds are those of its omega, and reach the target
    assert _rms(phi, phi_star) < 1e-8
    assert _rms(O.densities(w, p)["phi"], phi_star) < 1.5e-8
    last, tot = sim.cg_stats()
    assert last == got and tot == dict(inversions=1, iterations=got["iters"], evals=got["evals"], unconverged=0)
    sim.close()


def test_invert_measure_only_and_cap():
    """max_iter = 0 only measures the residual (omega unchanged); a cap of 3
    stops unconverged with the oracle's residual after 3 iterations."""
    say("[invert] cap 0 and 3")
    p = preset("cfg1")
    w_star = np.array(initial_omega(32, 32, 12, 0.05))
    phi_star = O.densities(w_star, p)["phi"]
    start = np.zeros_like(w_star)
    sim = _sim(p)
    sim.set_fields(start)
    r0 = sim.invert_densities(phi_star, max_iter=0)
    assert r0["iters"] == 0 and r0["evals"] == 1 and not r0["converged"] and r0["resid"] == r0["resid0"]
    assert np.array_equal(sim.fields(), start)
    ref = O.invert_densities(phi_star, start, p, max_iter=3)
    r3 = sim.invert_densities(phi_star, max_iter=3)
    assert r3["iters"] == 3 and not r3["converged"] and r3["evals"] == 7
    assert abs(r3["resid"] / ref["resid"] - 1) < 1e-6
    assert np.max(np.abs(sim.fields() - ref["omega"])) < 1e-9
    assert sim.cg_stats()[1]["unconverged"] == 2
    # already at the solution: no iteration
    sim.set_fields(w_star)
    r = sim.invert_densities(phi_star)
    assert r["iters"] == 0 and r["converged"] and r["resid0"] < 1e-13
    sim.close()


def test_invert_rejects_bad_targets():
    say("[invert] argument checks")
    p = preset("cfg1")
    sim = _sim(p)
    from paper_1804_02883_amd import EpdlbError
    with pytest.raises(EpdlbError):  # before any state
        sim.invert_densities(np.full((3, 32, 32), 1 / 3))
    sim.seed(1, 1e-3)
    bad = np.full((3, 32, 32), 1 / 3)
    bad[1, 3, 4] = 0.0
    with pytest.raises(EpdlbError):
        sim.invert_densities(bad)
    with pytest.raises(EpdlbError):
        sim.invert_densities(np.full((3, 32, 32), 1 / 3), tol=0.0)
    sim.close()


@pytest.mark.parametrize("pc", [0, 1])
def test_steps_with_inversion_vs_oracle(pc):
    """cfg1 under a strong lattice force (the convected composition then needs
    several iterations per step): 4 steps against the oracle's steps."""
    say(f"[cg step] cfg1, lattice force 1e-4, 4 steps, precond={pc}")
    p = preset("cfg1", g=1e-4, g_units=1, cg_invert=1, cg_precond=pc)
    w0 = np.array(initial_omega(32, 32, 1001, 0.05))
    sim = _sim(p)
    sim.set_fields(w0)
    s = O.init_state(p, w0)
    iters = []
    for k in range(4):
        sim.step(1)
        s = O.step(s, p)
        last, _ = sim.cg_stats()
        say(f"  step {k}: gpu iters {last['iters']} resid0 {last['resid0']:.2e}, oracle iters {s['cg']['iters']}")
        assert last["converged"] and abs(last["iters"] - s["cg"]["iters"]) <= 2
        assert abs(last["resid0"] / s["cg"]["resid0"] - 1) < 1e-6
        iters.append(last["iters"])
    sim.sync()
    assert min(iters) >= 3
    assert np.max(np.abs(sim.fields() - s["omega"])) < 1e-5
    assert np.max(np.abs(sim.densities() - s["phi"])) < 1e-7
    # the force differences the densities' tolerance-level differences (S divides
    # them by D_A = 1/16), so the velocity agrees to the same relative order
    rho, u = sim.velocity()
    err_u = np.max(np.abs(u - s["u"])) / np.max(np.abs(s["u"]))
    say(f"  velocity rel err {err_u:.2e}")
    assert err_u < 1e-4
    tot = sim.cg_stats()[1]
    assert tot["inversions"] == 4 and tot["unconverged"] == 0 and tot["iterations"] == sum(iters)
    sim.close()


def test_zero_flow_step_equals_default_step():
    """Without flow the convected composition is the stored one: no iteration,
    and the step is bit-for-bit the default step."""
    say("[cg step] no flow, 3 steps, against the default step")
    out = []
    for cg in (0, 1):
        p = preset("cfg1", couple_lb=0, cg_invert=cg)
        sim = _sim(p)
        sim.set_fields(initial_omega(32, 32, 1001, 0.05))
        sim.step(3)
        sim.sync()
        out.append((sim.fields(), sim.densities(), sim.populations()))
        if cg:
            last, tot = sim.cg_stats()
            assert tot["inversions"] == 3 and tot["iterations"] == 0 and last["resid0"] < 1e-13
        sim.close()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


def test_fp32_inversion_step():
    """FP32 fields with the FP32 bound on the tolerance (1e-6): converges, and the
    state stays within FP32 round-off of the FP64 oracle's step."""
    say("[cg step] 64x64 FP32, tol 1e-6, 3 steps")
    p = preset("cfg1", nx=64, ny=64, precision=1, g=1e-4, g_units=1, cg_invert=1, cg_tol=1e-6)
    w0 = np.array(initial_omega(64, 64, 7, 0.05))
    sim = _sim(p)
    sim.set_fields(w0)
    s = O.init_state(p, w0)
    for k in range(3):
        sim.step(1)
        s = O.step(s, p)
        last, _ = sim.cg_stats()
        say(f"  step {k}: gpu iters {last['iters']} resid {last['resid']:.2e}, oracle iters {s['cg']['iters']}")
        assert last["converged"]
    sim.sync()
    assert np.max(np.abs(sim.densities() - s["phi"])) < 2e-5
    sim.close()


def test_full_size_inversion_steps():
    """1024x512, N = 64, f_A = 0.3, FP64 (the paper's tolerance needs FP64
    fields) under a strong lattice force: every inversion converges; the
    auxiliary-convected omega misses the convected composition by far more than
    the tolerance, so the composition leaves the default step's; the totals of
    each species stay exact (any omega gives them)."""
    say("[cg step] 1024x512 N=64 FP64, lattice force 5e-7, 2 steps")
    p = preset("cfg3", precision=0, g=5e-7, g_units=1)
    w0 = np.array(initial_omega(1024, 512, 1003, 0.05))
    res = []
    for cg in (0, 1):
        sim = _sim(dict(p, cg_invert=cg))
        sim.set_fields(w0)
        sim.step(2)
        sim.sync()
        res.append((sim.fields(), sim.densities()))
        if cg:
            last, tot = sim.cg_stats()
            say(f"  iters {tot['iterations']} over 2 steps, last resid0 {last['resid0']:.2e} resid {last['resid']:.2e}")
            assert tot["unconverged"] == 0 and tot["inversions"] == 2 and last["resid"] < 1e-8
            assert last["resid0"] > 1e-6
        sim.close()
    phi = res[1][1]
    n = 1024 * 512
    totals = (p["f_A"] * p["phi_P"], (1 - p["f_A"]) * p["phi_P"], 1 - p["phi_P"])
    for I in range(3):
        assert abs(phi[I].sum() / n - totals[I]) < 1e-12, I
    assert np.all(np.isfinite(res[1][0]))
    say(f"  max |Phi_cg - Phi_default| {np.max(np.abs(phi - res[0][1])):.2e}")
    assert np.max(np.abs(phi - res[0][1])) > 1e-5


def test_full_size_invert_vs_oracle_densities():
    """1024x512, N = 64, f_A = 0.3, FP64: the direct inversion from a perturbed
    start reaches the oracle's densities of a known omega*, checked by the
    oracle's own density evaluation of the result (a full oracle iteration at
    this size would take minutes)."""
    say("[invert] 1024x512 N=64 FP64 against oracle densities")
    p = preset("cfg3", precision=0)
    w_star = np.array(initial_omega(1024, 512, 1003, 0.05))
    phi_star = O.densities(w_star, p)["phi"]
    rng = np.random.default_rng(5)
    seed = w_star + 0.01 * rng.standard_normal(w_star.shape)
    sim = _sim(p)
    sim.set_fields(seed)
    got = sim.invert_densities(phi_star, max_iter=5000, tol=1e-8)
    say(f"  iters {got['iters']} resid0 {got['resid0']:.2e} resid {got['resid']:.2e}")
    assert got["converged"] and got["resid"] < 1e-8
    w = sim.fields()
    assert _rms(O.densities(w, p)["phi"], sim.densities()) < 1e-12
    assert _rms(O.densities(w, p)["phi"], phi_star) < 1.5e-8
    d = w - w_star
    d -= d.mean(axis=(1, 2), keepdims=True)
    say(f"  max |omega - omega*| up to constants {np.max(np.abs(d)):.2e}")
    assert np.max(np.abs(d)) < 1e-3
    sim.close()
