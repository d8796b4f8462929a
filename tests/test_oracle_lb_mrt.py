"""Pins of the oracle's multi-relaxation LB (Sec. II: the collision with
relaxation parameters gamma_s, gamma_b, the force term of Eq. force_col and
the viscosity relations; reading R17)."""
import numpy as np
import pytest

from oracle import epdlb_oracle as O


def _near_equilibrium(shape, seed, amp=0.05):
    rng = np.random.default_rng(seed)
    f = O.W9[:, None, None] * (1 + amp * rng.standard_normal((9,) + shape))
    F = 1e-3 * rng.standard_normal((2,) + shape)
    return f, F


def test_hermite_expansion_carries_its_moments():
    """The populations built from (rho, j, Pi) have exactly those moments, and an
    equilibrium population is its own expansion."""
    rng = np.random.default_rng(3)
    rho = 1 + 0.1 * rng.standard_normal((4, 5))
    j = 0.05 * rng.standard_normal((2, 4, 5))
    A = 0.02 * rng.standard_normal((2, 2, 4, 5))
    Pi = rho * O.CS2 * np.eye(2)[:, :, None, None] + 0.5 * (A + A.transpose(1, 0, 2, 3))
    r2, j2, P2 = O.lb_moments(O.lb_hermite(rho, j, Pi))
    assert np.max(np.abs(r2 - rho)) < 1e-15
    assert np.max(np.abs(j2 - j)) < 1e-15
    assert np.max(np.abs(P2 - Pi)) < 1e-15
    u = 0.05 * rng.standard_normal((2, 4, 5))
    feq = O.lb_equilibrium(rho, u)
    assert np.max(np.abs(O.lb_hermite(*O.lb_moments(feq)) - feq)) < 1e-15


@pytest.mark.parametrize("tau", [0.554, 0.8, 1.0, 1.7])
def test_equal_rates_reduce_to_bgk(tau):
    """With gamma_s = gamma_b = gamma_g = 1 - 1/tau the collision is the BGK
    collision at relaxation time tau with second-order forcing (the pinned
    lb_step), population by population."""
    f, F = _near_equilibrium((6, 7), 11)
    g = 1.0 - 1.0 / tau
    a, ra, ua = O.lb_step_mrt(f, F, g, g, g)
    b, rb, ub = O.lb_step(f, F, tau)
    assert np.max(np.abs(a - b)) < 1e-15
    assert np.max(np.abs(ua - ub)) < 1e-16 and np.max(np.abs(ra - rb)) < 1e-15


def test_conservation_and_momentum_gain():
    """Mass is conserved and each site's momentum gains exactly F (unequal rates)."""
    f, F = _near_equilibrium((5, 6), 5)
    out, rho, u = O.lb_collide_mrt(f, F, -0.805, 0.3, 0.0)
    r0, j0, _ = O.lb_moments(f)
    r1, j1, _ = O.lb_moments(out)
    assert np.max(np.abs(r1 - r0)) < 1e-15
    assert np.max(np.abs(j1 - j0 - F)) < 1e-15


@pytest.mark.parametrize("gg", [0.0, 0.4])
def test_non_hydrodynamic_modes_scale_by_gamma_g(gg):
    """The part of the populations outside the hydrodynamic moments is multiplied
    by gamma_g in one collision (with or without force)."""
    f, F = _near_equilibrium((4, 4), 8, amp=0.2)
    out, _, _ = O.lb_collide_mrt(f, F, -0.5, 0.2, gg)
    ghost_in = f - O.lb_hermite(*O.lb_moments(f))
    ghost_out = out - O.lb_hermite(*O.lb_moments(out))
    assert np.max(np.abs(ghost_in)) > 1e-3
    assert np.max(np.abs(ghost_out - gg * ghost_in)) < 1e-15


def test_uniform_acceleration_stress_first_order_in_F():
    """A uniform fluid under a uniform force: after a collision the stress equals the
    equilibrium stress of the new momentum up to O(F^2), for unequal gamma_s and
    gamma_b.  This is what the force's stress term is for; it holds with the d = 2
    trace split of reading R17 (the d = 3 factors leave a term linear in F)."""
    shape = (1, 1)
    j0 = np.array([0.02, -0.01]).reshape(2, 1, 1)
    rho = np.ones(shape)
    f = O.lb_equilibrium(rho, j0)  # equilibrium at velocity j0
    errs = []
    for s in (1e-4, 2e-4, 4e-4):
        F = s * np.array([0.6, 0.8]).reshape(2, 1, 1)
        out, _, _ = O.lb_collide_mrt(f, F, -0.805, 0.35, 0.0)
        r1, j1, P1 = O.lb_moments(out)
        target = r1 * O.CS2 * np.eye(2)[:, :, None, None] + np.einsum("a...,b...->ab...", j1, j1) / r1
        errs.append(np.max(np.abs(P1 - target)))
    # quadratic in F: doubling F quadruples the deviation
    assert 3.9 < errs[1] / errs[0] < 4.1 and 3.9 < errs[2] / errs[1] < 4.1
    assert errs[0] < 1e-8


def _shear_rate(gs, gb, gg, ny=64, steps=(100, 400)):
    k = 2 * np.pi / ny
    y = np.arange(ny) + 0.5
    u = np.zeros((2, ny, 2))
    u[0] = 1e-4 * np.sin(k * y)[:, None]
    f = O.lb_equilibrium(np.ones((ny, 2)), u)
    F = np.zeros((2, ny, 2))
    amps = []
    for t in range(steps[1]):
        f, rho, u = O.lb_step_mrt(f, F, gs, gb, gg)
        if t + 1 in steps:
            amps.append(np.sum(u[0, :, 0] * np.sin(k * y)) * 2 / ny)
    return np.log(amps[0] / amps[1]) / (steps[1] - steps[0]), k


@pytest.mark.parametrize("gs,gb,gg", [(-0.5, 0.3, 0.0), (-0.5, -0.7, 0.5), (-0.805, -0.805, 0.0)])
def test_shear_wave_decay_sets_shear_viscosity(gs, gb, gg):
    """A transverse shear wave decays at nu k^2 with nu = (c_s^2/2)(1+gamma_s)/(1-gamma_s)
    (the shear-viscosity relation of Sec. II in lattice units), whatever gamma_b, gamma_g."""
    rate, k = _shear_rate(gs, gb, gg)
    nu = 0.5 * O.CS2 * (1 + gs) / (1 - gs)
    assert abs(rate / (nu * k * k) - 1) < 5e-3


@pytest.mark.parametrize("gs,gb", [(-0.5, 0.5), (-0.805, 0.2)])
def test_sound_wave_damping_sets_bulk_viscosity(gs, gb):
    """A standing sound wave's energy decays at 2 Gamma with
    Gamma = (k^2/2)(nu (2 - 2/d) + nu_B) for d = 2, nu_B = (c_s^2/d)(1+gamma_b)/(1-gamma_b)
    (the bulk-viscosity relation of Sec. II, linearised Navier-Stokes)."""
    nx = 64
    k = 2 * np.pi / nx
    x = np.arange(nx)
    rho = (1 + 1e-5 * np.cos(k * x))[None, :] * np.ones((2, 1))
    f = O.lb_equilibrium(rho, np.zeros((2, 2, nx)))
    F = np.zeros((2, 2, nx))
    T = nx / np.sqrt(O.CS2)  # one acoustic period, in steps
    E = []
    marks = (int(round(2 * T)), int(round(6 * T)))
    for t in range(marks[1]):
        f, r, u = O.lb_step_mrt(f, F, gs, gb, 0.0)
        if t + 1 in marks:
            E.append(np.sum(O.CS2 * (r - 1) ** 2 + r * (u[0] ** 2 + u[1] ** 2)))
    rate = np.log(E[0] / E[1]) / (marks[1] - marks[0]) / 2
    nu = 0.5 * O.CS2 * (1 + gs) / (1 - gs)
    nuB = 0.5 * O.CS2 * (1 + gb) / (1 - gb)
    gamma = 0.5 * k * k * (nu + nuB)
    assert abs(rate / gamma - 1) < 2e-2


def test_viscosity_relations_at_the_paper_parameters():
    """eta = eta_B = 1 R_G^2/tau rho with dx = R_G/3, dt = 0.002 tau: gamma_s = gamma_b,
    lattice nu = eta dt/(rho dx^2) = 0.018."""
    gs, gb = O.mrt_gammas(1.0, 1.0, 1.0, 1.0 / 3.0, 0.002)
    assert abs(gs - gb) < 1e-15
    assert abs(0.5 * O.CS2 * (1 + gs) / (1 - gs) - 0.018) < 1e-15
    p = dict(lb_mrt=1, lb_gamma_s=gs, lb_gamma_b=gb)
    assert abs(O.lb_viscosity(p) - 0.018) < 1e-15
