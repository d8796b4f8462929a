"""Pins of the Phi -> omega inversion in the oracle (App. C comments 1-3; readings
R21-R23 in oracle/epdlb_oracle.py).

What fixes the result independently of the iteration:
* the functional's gradient is dA (Phi~ - Phi[omega]) (central differences of
  the log partition functions, which the density integrals must equal);
* Phi_S = V phibar_S exp(-omega_S) / Q_S inverts in closed form:
  omega_S = -ln Phi~_S + const;
* the minimiser is unique up to one constant per field (G is convex, and a
  uniform shift of omega_A, omega_B or omega_S changes no density, since every
  chain carries the same number of A segments), so a round trip Phi[omega*]
  recovers omega* up to those constants from any nearby start.
"""
import numpy as np
import pytest

from oracle import epdlb_oracle as O
from seeded_inputs import initial_omega, preset


def _omega(nx, ny, seed, sigma):
    return np.array(initial_omega(nx, ny, seed, sigma))


def _gauge_free(w):
    return w - w.mean(axis=(1, 2), keepdims=True)


def test_gradient_is_density_mismatch():
    p = preset("cfg1", nx=16, ny=16, n_contour=8, f_A=0.3)
    rng = np.random.default_rng(3)
    w0 = _omega(16, 16, 7, 0.05) + 0.01 * rng.standard_normal((3, 16, 16))
    target = O.densities(_omega(16, 16, 8, 0.05), p)["phi"]
    g = tuple(O.field_means(w0))
    grad = p["dx"] ** 2 * (target - O.densities(w0, p, g)["phi"])
    h = 1e-4
    for I, y, x in [(0, 3, 4), (0, 9, 2), (1, 10, 13), (1, 0, 15), (2, 15, 0), (2, 6, 6)]:
        wp = w0.copy()
        wp[I, y, x] += h
        wm = w0.copy()
        wm[I, y, x] -= h
        fd = (O.legendre_objective(wp, target, p, g) - O.legendre_objective(wm, target, p, g)) / (2 * h)
        assert abs(fd - grad[I, y, x]) <= 1e-4 * abs(grad[I, y, x]) + 1e-11, (I, y, x, fd, grad[I, y, x])


@pytest.mark.parametrize("a,b,alpha_t", [(2.0, 0.5, 1.0), (1e-6, 3e-4, 7.5), (0.3, 2.0, 0.01)])
def test_secant_root_exact_for_quadratic(a, b, alpha_t):
    """Along a direction where G is quadratic the derivative is a - b alpha, with
    root a / b; a non-negative slope falls back to the trial length."""
    got = O.secant_root(alpha_t, a, a - b * alpha_t)
    assert abs(got - a / b) <= 1e-12 * a / b
    assert O.secant_root(alpha_t, a, a + 0.1) == alpha_t
    assert O.secant_root(alpha_t, a, a) == alpha_t


def test_round_trip_recovers_potentials_up_to_constants():
    p = preset("cfg1")
    w_star = _omega(32, 32, 1001, 0.05)
    phi_star = O.densities(w_star, p)["phi"]
    rng = np.random.default_rng(0)
    seed = w_star + 0.02 * rng.standard_normal(w_star.shape) + np.array([0.3, -0.2, 0.1])[:, None, None]
    r = O.invert_densities(phi_star, seed, p)
    assert r["converged"] and r["resid"] < 1e-8 < r["resid0"] and r["iters"] >= 5
    # the residual it reports is the one of its result
    got = O.densities(r["omega"], p)["phi"]
    assert np.sqrt(np.sum((got - phi_star) ** 2) / (32 * 32)) < 1e-8
    assert np.max(np.abs(_gauge_free(r["omega"]) - _gauge_free(w_star))) < 2e-5


def test_solvent_field_closed_form():
    """Whatever the polymer target, the solvent potential of the solution is
    -ln Phi~_S plus a constant (Eq. phi_s solved for omega_S)."""
    p = preset("cfg1", f_A=0.7)
    w_star = _omega(32, 32, 5, 0.08)
    phi_star = O.densities(w_star, p)["phi"]
    r = O.invert_densities(phi_star, np.zeros_like(w_star), p)
    assert r["converged"]
    c = r["omega"][2] + np.log(phi_star[2])
    assert np.ptp(c) < 1e-6


def test_start_at_the_solution_takes_no_iteration():
    p = preset("cfg1")
    w = _omega(32, 32, 11, 0.05)
    phi = O.densities(w, p)["phi"]
    r = O.invert_densities(phi, w, p)
    assert r["iters"] == 0 and r["evals"] == 1 and r["converged"] and r["resid0"] < 1e-14
    assert np.array_equal(r["omega"], w)


def test_iteration_cap_reports_unconverged():
    p = preset("cfg1")
    w_star = _omega(32, 32, 12, 0.05)
    phi_star = O.densities(w_star, p)["phi"]
    r = O.invert_densities(phi_star, np.zeros_like(w_star), p, max_iter=3)
    assert r["iters"] == 3 and r["evals"] == 7 and not r["converged"]
    assert 1e-8 < r["resid"] < r["resid0"]


def test_step_with_inversion():
    """Without flow the advected fields are the old ones, Phi^n = Phi[omega^n], so the
    inversion stops at once and the step equals the default one.  Under a strong
    flow the auxiliary-convected omega misses the advected composition by more
    than N_tr, and the inverted one reproduces it."""
    w0 = _omega(32, 32, 1001, 0.05)
    p0 = preset("cfg1", couple_lb=0)
    a = O.step(O.init_state(p0, w0), p0)
    b = O.step(O.init_state(p0, w0), dict(p0, cg_invert=1))
    assert b["cg"]["iters"] == 0
    assert np.array_equal(a["omega"], b["omega"]) and np.array_equal(a["phi"], b["phi"])
    p = preset("cfg1", g=1e-4, g_units=1)
    s0 = O.init_state(p, w0)
    plain = O.step(s0, p)
    cg = O.step(s0, dict(p, cg_invert=1))
    n = 32 * 32
    miss = np.sqrt(np.sum((O.densities(plain["omega_t"], p)["phi"] - plain["phi_t"]) ** 2) / n)
    hit = np.sqrt(np.sum((O.densities(cg["omega_t"], p)["phi"] - cg["phi_t"]) ** 2) / n)
    assert miss > 1e-6 and hit < 1e-8
    assert cg["cg"]["converged"] and cg["cg"]["iters"] >= 3
    # same advected composition, different potentials
    assert np.array_equal(plain["phi_t"], cg["phi_t"])
    assert np.max(np.abs(plain["omega_t"] - cg["omega_t"])) > 1e-6


def test_preconditioned_iteration_same_solution_fewer_iterations():
    """cg_precond = 1 (reading R25): the same potentials up to constants, the same
    stopping test, and fewer iterations where the plain iteration needs many."""
    p = preset("cfg1", nx=64, ny=64, n_contour=32, f_A=0.3)
    w_star = _omega(64, 64, 5, 0.05)
    phi_star = O.densities(w_star, p)["phi"]
    rng = np.random.default_rng(1)
    seed = w_star + 0.02 * rng.standard_normal(w_star.shape)
    plain = O.invert_densities(phi_star, seed, p)
    pre = O.invert_densities(phi_star, seed, p, precond=1)
    assert plain["converged"] and pre["converged"] and pre["resid"] < 1e-8
    assert pre["resid0"] == plain["resid0"]
    assert pre["iters"] < 0.8 * plain["iters"], (pre["iters"], plain["iters"])
    assert np.max(np.abs(_gauge_free(pre["omega"]) - _gauge_free(w_star))) < 2e-5
    c = pre["omega"][2] + np.log(phi_star[2])
    assert np.ptp(c) < 1e-6
    m = O.local_response(phi_star, p)
    assert np.array_equal(m[0], 32 * phi_star[0]) and np.array_equal(m[2], phi_star[2])
