"""Pins of the three-dimensional lattice Boltzmann oracle (D3Q19, readings R26
and R27 in oracle/lb3d_oracle.py) against what fixes it independently:

* the lattice tensors of D3Q19: sum w = 1, sum w c = 0, sum w c c = I/3, odd
  moments zero, sum w c c c c = (delta delta + delta delta + delta delta)/9,
  which a wrong weight or velocity breaks;
* streaming moves a single population by its velocity;
* mass is conserved exactly and the total momentum grows by the total force
  each step (second-order forcing);
* the step commutes with a rotation of the axes;
* the hydrodynamic limit: a shear wave decays at nu k^2 with nu = (tau - 1/2)/3,
  and Kolmogorov flow F_x = F0 sin(k y) settles at u_x = F0 sin(k y) / (nu k^2),
  both to O(k^2) (Navier-Stokes solutions in closed form).
"""
import itertools

import numpy as np
import pytest

from oracle import lb3d_oracle as L


def _delta(a, b):
    return 1.0 if a == b else 0.0


def test_lattice_tensors():
    c = L.C19.astype(np.float64)
    w = L.W19
    assert len(c) == 19 and len({tuple(v) for v in L.C19}) == 19
    assert abs(w.sum() - 1) < 1e-15
    assert np.all(np.abs(w @ c) < 1e-15)
    for a, b in itertools.product(range(3), repeat=2):
        assert abs(np.sum(w * c[:, a] * c[:, b]) - _delta(a, b) / 3) < 1e-15
    for a, b, d in itertools.product(range(3), repeat=3):
        assert abs(np.sum(w * c[:, a] * c[:, b] * c[:, d])) < 1e-15
    for a, b, d, e in itertools.product(range(3), repeat=4):
        iso = (_delta(a, b) * _delta(d, e) + _delta(a, d) * _delta(b, e) + _delta(a, e) * _delta(b, d)) / 9
        assert abs(np.sum(w * c[:, a] * c[:, b] * c[:, d] * c[:, e]) - iso) < 1e-15, (a, b, d, e)
    # closed under negation; speeds 0, 1 and sqrt 2 with the weights 1/3, 1/18, 1/36
    for v in L.C19:
        assert any(np.array_equal(-v, u) for u in L.C19)
    sq = (c ** 2).sum(axis=1)
    assert np.all(w[sq == 0] == 1 / 3) and np.all(w[sq == 1] == 1 / 18) and np.all(w[sq == 2] == 1 / 36)
    assert (sq == 1).sum() == 6 and (sq == 2).sum() == 12


def test_equilibrium_moments():
    rng = np.random.default_rng(0)
    rho = 1 + 0.1 * rng.standard_normal((2, 3, 4))
    u = 0.05 * rng.standard_normal((3, 2, 3, 4))
    feq = L.equilibrium(rho, u)
    c = L.C19.astype(np.float64)
    assert np.allclose(feq.sum(axis=0), rho, rtol=0, atol=1e-15)
    for a in range(3):
        assert np.allclose(np.einsum("i,i...->...", c[:, a], feq), rho * u[a], rtol=0, atol=1e-15)
        for b in range(3):
            pi = np.einsum("i,i...->...", c[:, a] * c[:, b], feq)
            assert np.allclose(pi, rho * (_delta(a, b) / 3 + u[a] * u[b]), rtol=0, atol=1e-15)


@pytest.mark.parametrize("i", range(19))
def test_stream_moves_one_population_by_its_velocity(i):
    nz, ny, nx = 3, 4, 5
    fs = np.zeros((19, nz, ny, nx))
    z0, y0, x0 = 0, 3, 4  # at the box edge, so the move wraps where c_i points outwards
    fs[i, z0, y0, x0] = 1.0
    f = L.stream(fs)
    cx, cy, cz = L.C19[i]
    dest = ((z0 + cz) % nz, (y0 + cy) % ny, (x0 + cx) % nx)
    assert f[i][dest] == 1.0 and f.sum() == 1.0


def _random_state(shape, seed, amp=0.05):
    rng = np.random.default_rng(seed)
    rho = 1 + amp * rng.standard_normal(shape)
    u = amp * rng.standard_normal((3,) + shape)
    f = L.equilibrium(rho, u) + amp / 36 * rng.standard_normal((19,) + shape)
    F = 1e-3 * rng.standard_normal((3,) + shape)
    return f, F


@pytest.mark.parametrize("tau", [0.6, 1.0, 1.7])
def test_conservation_mass_and_momentum_gain(tau):
    f, F = _random_state((4, 6, 5), 1)
    out, rho, u = L.step(f, F, tau)
    c = L.C19.astype(np.float64)
    assert abs(out.sum() - f.sum()) < 1e-12
    for a in range(3):
        j0 = np.sum(np.einsum("i,i...->...", c[:, a], f))
        j1 = np.sum(np.einsum("i,i...->...", c[:, a], out))
        assert abs(j1 - (j0 + F[a].sum())) < 1e-12
    # the velocity includes half the force
    f_streamed = L.stream(f)
    for a in range(3):
        ja = np.einsum("i,i...->...", c[:, a], f_streamed)
        assert np.allclose(u[a] * rho, ja + 0.5 * F[a], rtol=0, atol=1e-14)


def test_relaxation_time_one_without_force_gives_equilibrium():
    f, F = _random_state((2, 3, 4), 2)
    fs = L.stream(f)
    out, rho, u = L.collide(fs, np.zeros_like(F), 1.0)
    assert np.allclose(out, L.equilibrium(rho, u), rtol=0, atol=1e-15)
    # and the equilibrium is a fixed point of the collision for any tau
    feq = L.equilibrium(rho, u)
    out2, _, _ = L.collide(feq, np.zeros_like(F), 0.73)
    assert np.allclose(out2, feq, rtol=0, atol=1e-15)


def test_step_commutes_with_axis_rotation():
    """Rotating the axes x -> y -> z -> x before the step gives the rotated
    result: a transposed shift or component anywhere breaks this."""
    f, F = _random_state((3, 4, 5), 3)
    # positions: B[z', y', x'] = A[z = x', y = z', x = y']
    rot = lambda A: np.transpose(A, (1, 2, 0))  # noqa: E731
    # velocities: (P c) = (c_z, c_x, c_y)
    pc = [tuple(v) for v in L.C19[:, [2, 0, 1]]]
    idx = [next(j for j in range(19) if tuple(L.C19[j]) == pc[i]) for i in range(19)]
    fr = np.empty((19,) + rot(f[0]).shape)
    for i in range(19):
        fr[idx[i]] = rot(f[i])
    Fr = np.stack([rot(F[2]), rot(F[0]), rot(F[1])])
    out, rho, u = L.step(f, F, 0.8)
    outr, rhor, ur = L.step(fr, Fr, 0.8)
    for i in range(19):
        assert np.allclose(outr[idx[i]], rot(out[i]), rtol=0, atol=1e-15)
    assert np.allclose(rhor, rot(rho), rtol=0, atol=1e-15)
    assert np.allclose(ur, np.stack([rot(u[2]), rot(u[0]), rot(u[1])]), rtol=0, atol=1e-15)


def test_site_matches_whole_lattice_step():
    f, F = _random_state((3, 4, 5), 4)
    out, rho, u = L.step(f, F, 0.9)
    for z, y, x in itertools.product(range(3), range(4), range(5)):
        o, r, v = L.site(f, F, 0.9, z, y, x)
        assert np.allclose(o, out[:, z, y, x], rtol=0, atol=1e-15)
        assert abs(r - rho[z, y, x]) < 1e-15 and np.allclose(v, u[:, z, y, x], rtol=0, atol=1e-15)


def _projection(v, k, coord):
    return 2 * np.mean(v * np.sin(k * coord))


@pytest.mark.parametrize("tau", [0.8, 1.3])
def test_shear_wave_decays_with_lattice_viscosity(tau):
    """u_x(y) = A sin(k y) decays as exp(-nu k^2 t), nu = (tau - 1/2)/3; the
    rate is taken between two times, so the start-up transient drops out."""
    ny = 64
    k = 2 * np.pi / ny
    y = np.arange(ny, dtype=np.float64)
    u = np.zeros((3, 1, ny, 1))
    u[0, 0, :, 0] = 1e-3 * np.sin(k * y)
    f = L.equilibrium(np.ones((1, ny, 1)), u)
    F = np.zeros((3, 1, ny, 1))
    amp = {}
    for t in range(1, 301):
        f, rho, uu = L.step(f, F, tau)
        if t in (50, 300):
            amp[t] = _projection(uu[0, 0, :, 0], k, y)
    rate = np.log(amp[50] / amp[300]) / 250
    nu = L.viscosity(tau)
    assert abs(rate / (nu * k * k) - 1) < 2e-3, rate / (nu * k * k)


@pytest.mark.parametrize("axis", ["x_along_y", "z_along_x"])
def test_kolmogorov_flow_steady_amplitude(axis):
    """F = F0 sin(k s) e_a settles at u_a = F0 sin(k s) / (nu k^2) (tau = 1);
    a dropped or mis-signed force term changes the amplitude by a factor."""
    n, tau, F0 = 32, 1.0, 1e-5
    k = 2 * np.pi / n
    s = np.arange(n, dtype=np.float64)
    if axis == "x_along_y":
        shape, comp = (1, n, 1), 0
        prof = np.sin(k * s)[None, :, None]
    else:
        shape, comp = (1, 1, n), 2
        prof = np.sin(k * s)[None, None, :]
    F = np.zeros((3,) + shape)
    F[comp] = F0 * prof
    f = L.equilibrium(np.ones(shape), np.zeros((3,) + shape))
    for _ in range(3000):
        f, rho, u = L.step(f, F, tau)
    got = _projection(u[comp].ravel(), k, s)
    want = F0 / (L.viscosity(tau) * k * k)
    assert abs(got / want - 1) < 5e-3, got / want
    others = [a for a in range(3) if a != comp]
    assert np.max(np.abs(u[others])) < 1e-12 * want
    assert np.max(np.abs(rho - 1)) < 1e-9


def _channel(ny, F0, steps):
    Y = np.arange(ny) + 0.5
    Fx = np.where(Y < ny / 2, -F0, F0)
    F = np.zeros((3, 1, ny, 1))
    F[0, 0, :, 0] = Fx
    f = L.equilibrium(np.ones((1, ny, 1)), np.zeros((3, 1, ny, 1)))
    for _ in range(steps):
        f, rho, u = L.step(f, F, 1.0)
    return u, Fx


def test_reverse_poiseuille_channel():
    """The paper's drive (force -F0 in the lower half of the box, +F0 in the
    upper) settles at the two parabolas of Eq. flow_field, with the
    second-order discretisation error of the two-dimensional lattice, and
    satisfies the lattice's discrete steady balance
    nu (u_{y+1} - 2 u_y + u_{y-1}) = -F_y - (F_{y+1} - 2 F_y + F_{y-1})/12."""
    from oracle import epdlb_oracle as O
    F0, errs = 1e-6, []
    for ny in (16, 32):
        u, Fx = _channel(ny, F0, 4000)
        ux = u[0, 0, :, 0]
        exact = O.poiseuille_profile(ny, F0, 1.0)
        errs.append(np.max(np.abs(ux - exact)) / np.max(np.abs(exact)))
        nu = L.viscosity(1.0)
        lhs = nu * (np.roll(ux, -1) - 2 * ux + np.roll(ux, 1))
        rhs = -Fx - (np.roll(Fx, -1) - 2 * Fx + np.roll(Fx, 1)) / 12.0
        assert np.max(np.abs(lhs - rhs)) < 1e-9 * F0
        assert np.max(np.abs(u[1:])) < 1e-14  # rounding of O(1) populations
    assert errs[0] < 6e-3 and errs[1] < 1.5e-3
    assert 3.0 < errs[0] / errs[1] < 5.0


# --- the multi-relaxation collision in three dimensions (reading R28) ---

@pytest.mark.parametrize("tau", [0.6, 1.0, 1.7])
def test_mrt_equal_rates_reduce_to_bgk(tau):
    """gamma_s = gamma_b = gamma_g = 1 - 1/tau gives the pinned BGK step with its
    second-order force term, population by population."""
    f, F = _random_state((3, 4, 5), 21)
    g = 1.0 - 1.0 / tau
    a = L.step_mrt(f, F, g, g, g)[0]
    b = L.step(f, F, tau)[0]
    assert np.max(np.abs(a - b)) < 1e-15


def test_hermite_expansion_carries_its_moments():
    rng = np.random.default_rng(4)
    shape = (2, 3, 4)
    rho = 1 + 0.1 * rng.standard_normal(shape)
    j = 0.05 * rng.standard_normal((3,) + shape)
    A = 0.02 * rng.standard_normal((3, 3) + shape)
    Pi = rho * L.CS2 * np.eye(3).reshape(3, 3, 1, 1, 1) + 0.5 * (A + A.transpose(1, 0, 2, 3, 4))
    r2, j2, P2 = L.stress_moments(L.hermite(rho, j, Pi))
    assert np.max(np.abs(r2 - rho)) < 1e-15 and np.max(np.abs(j2 - j)) < 1e-15
    assert np.max(np.abs(P2 - Pi)) < 1e-15


@pytest.mark.parametrize("gs,gb,gg", [(0.2, -0.5, 0.0), (-0.3, 0.6, 0.4)])
def test_mrt_conservation(gs, gb, gg):
    f, F = _random_state((4, 3, 5), 22)
    out, rho, u = L.step_mrt(f, F, gs, gb, gg)
    c = L.C19.astype(np.float64)
    assert abs(out.sum() - f.sum()) < 1e-12
    for a in range(3):
        j0 = np.sum(np.einsum("i,i...->...", c[:, a], f))
        j1 = np.sum(np.einsum("i,i...->...", c[:, a], out))
        assert abs(j1 - (j0 + F[a].sum())) < 1e-12


def _wave_rate(gs, gb, kind, n=64, T=1500, t0=200):
    """Decay rate of a shear wave (u_y(x)) or of a sound wave (rho(x)) along x."""
    k = 2 * np.pi / n
    x = np.arange(n, dtype=np.float64)
    rho0 = np.ones((1, 1, n))
    u0 = np.zeros((3, 1, 1, n))
    if kind == "shear":
        u0[1, 0, 0] = 1e-4 * np.sin(k * x)
    else:
        rho0[0, 0] += 1e-4 * np.sin(k * x)
    f = L.equilibrium(rho0, u0)
    F = np.zeros((3, 1, 1, n))
    E = []
    for _ in range(T):
        f, r, u = L.step_mrt(f, F, gs, gb, 0.0)
        if kind == "shear":
            E.append((2 * np.mean(u[1, 0, 0] * np.sin(k * x))) ** 2)
        else:  # density and momentum parts of the wave together decay smoothly
            rk = 2 * np.mean((r[0, 0] - 1) * np.sin(k * x))
            jk = 2 * np.mean(r[0, 0] * u[0, 0, 0] * np.cos(k * x))
            E.append(rk * rk + jk * jk / L.CS2)
    t = np.arange(T)
    return -np.polyfit(t[t0:], np.log(np.array(E)[t0:]), 1)[0] / 2, k


@pytest.mark.parametrize("gs,gb", [(0.2, -0.5), (-0.3, 0.5)])
def test_mrt_shear_wave_uses_gamma_s_only(gs, gb):
    rate, k = _wave_rate(gs, gb, "shear")
    nu, _ = L.mrt_viscosities(gs, gb)
    assert abs(rate / (nu * k * k) - 1) < 2e-3


def test_mrt_sound_attenuation_fixes_the_bulk_viscosity():
    """A sound wave decays at (k^2/2)(4 nu/3 + nu_B) (three-dimensional
    Navier-Stokes), with nu_B = (c_s^2/3)(1 + gamma_b)/(1 - gamma_b): the
    trace split of d = 3.  The difference between two gamma_b isolates nu_B
    (a d = 2 split would make it 3/2 as large)."""
    rates = {}
    for gb in (-0.5, 0.5):
        rate, k = _wave_rate(0.2, gb, "sound")
        nu, nuB = L.mrt_viscosities(0.2, gb)
        assert abs(rate / (k * k / 2 * (4 * nu / 3 + nuB)) - 1) < 1e-2
        rates[gb] = rate
    dB = L.mrt_viscosities(0.2, 0.5)[1] - L.mrt_viscosities(0.2, -0.5)[1]
    assert abs((rates[0.5] - rates[-0.5]) / (k * k / 2 * dB) - 1) < 3e-2


def test_site_mrt_matches_whole_lattice_step():
    f, F = _random_state((3, 4, 5), 23)
    out, rho, u = L.step_mrt(f, F, 0.2, -0.4, 0.3)
    for z, y, x in [(0, 0, 0), (2, 3, 4), (1, 2, 0), (0, 3, 2)]:
        o, r, v = L.site(f, F, 0.0, z, y, x, mrt=(0.2, -0.4, 0.3))
        assert np.allclose(o, out[:, z, y, x], rtol=0, atol=1e-15)
        assert abs(r - rho[z, y, x]) < 1e-15 and np.allclose(v, u[:, z, y, x], rtol=0, atol=1e-15)


@pytest.mark.parametrize("d", [2, 3])
def test_mrt_gammas_invert_the_pinned_viscosities(d):
    """The viscosity relations of Sec. II in d dimensions: the factors from
    mrt_gammas give back the lattice viscosities nu = eta dt/(rho dx^2) and
    nu_B = eta_B dt/(rho dx^2) through the shear (gamma_s) and bulk (gamma_b)
    relations that the shear-wave and sound-attenuation tests above fix (d = 3)
    and that the two-dimensional ones fix (d = 2: nu_B = (c_s^2/2)(1 + gamma_b)/(1 - gamma_b))."""
    from oracle import epdlb_oracle as O2
    dx, dt = 1.0 / 3.0, 0.002
    conv = dt / dx ** 2
    for eta, eta_B, rho in ((1.0, 1.0, 1.0), (0.7, 2.5, 1.0), (1.3, 0.4, 1.7)):
        gs, gb = O2.mrt_gammas(eta, eta_B, rho, dx, dt, d=d)
        if d == 3:
            nu, nuB = L.mrt_viscosities(gs, gb)
        else:
            nu = 0.5 * O2.CS2 * (1 + gs) / (1 - gs)
            nuB = 0.5 * O2.CS2 * (1 + gb) / (1 - gb)
        assert abs(nu - eta * conv / rho) < 1e-14 and abs(nuB - eta_B * conv / rho) < 1e-14, (eta, eta_B, rho)
