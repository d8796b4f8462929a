"""Pins of the oracle's LB (Eq. LB_prop, Eq. force_col, Eq. flow_field), force
reconstruction (k-space force, App. A), advection and EPD-update parts."""
import numpy as np

from oracle import epdlb_oracle as O
from seeded_inputs import preset


def test_d2q9_lattice_moments():
    """Isotropy of the D2Q9 set: sum w = 1, sum w c = 0, sum w c c = c_s^2 delta, third moment 0."""
    c, w = O.C9, O.W9
    assert abs(w.sum() - 1) < 1e-16
    assert np.allclose((w[:, None] * c).sum(0), 0)
    M2 = np.einsum("i,ia,ib->ab", w, c, c)
    assert np.allclose(M2, np.eye(2) / 3, atol=1e-16)
    M3 = np.einsum("i,ia,ib,ic->abc", w, c, c, c)
    assert np.allclose(M3, 0)


def test_lb_rest_state_fixed_point():
    rho = np.ones((6, 5))
    f = O.lb_equilibrium(rho, np.zeros((2, 6, 5)))
    out, r, u = O.lb_step(f, np.zeros((2, 6, 5)), 1.0)
    assert np.max(np.abs(out - f)) < 1e-15 and np.max(np.abs(u)) == 0


def test_lb_mass_and_momentum_balance():
    rng = np.random.default_rng(1)
    f = O.W9[:, None, None] * (1 + 0.1 * rng.standard_normal((9, 7, 9)))
    F = 1e-3 * rng.standard_normal((2, 7, 9))
    for tau in (1.0, 0.7):
        out, rho, u = O.lb_step(f, F, tau)
        assert abs(out.sum() - f.sum()) < 1e-13
        p0 = np.einsum("ia,iyx->a", O.C9.astype(float), f)
        p1 = np.einsum("ia,iyx->a", O.C9.astype(float), out)
        assert np.allclose(p1 - p0, F.sum(axis=(1, 2)), atol=1e-13)


def _run_channel(ny, F0, tau, steps, nx=2):
    Fx = np.where(np.arange(ny) < ny // 2, -F0, F0)
    F = np.zeros((2, ny, nx))
    F[0] = Fx[:, None]
    u = np.zeros((2, ny, nx))
    u[0] = O.poiseuille_profile(ny, F0, tau)[:, None]
    f = O.lb_equilibrium(np.ones((ny, nx)), u)
    for _ in range(steps):
        f, rho, u = O.lb_step(f, F, tau)
    return u[0, :, 0], Fx


def test_reverse_poiseuille_steady_state():
    """Steady LB flow under the reverse-Poiseuille force approaches Eq. flow_field
    (nu = (tau - 1/2)/3 in lattice units) with an O(L^-2) discretisation error."""
    F0 = 1e-6
    errs = []
    for ny in (16, 32):
        ux, Fx = _run_channel(ny, F0, 1.0, 6000)
        exact = O.poiseuille_profile(ny, F0, 1.0)
        errs.append(np.max(np.abs(ux - exact)) / np.max(np.abs(exact)))
        # discrete steady state of second-order forced LB (derived from the
        # Chapman-Enskog balance of the lattice equations):
        # nu (u_{y+1} - 2u_y + u_{y-1}) = -F_y - (1/12)(F_{y+1} - 2 F_y + F_{y-1})
        nu = 1.0 / 6.0
        lhs = nu * (np.roll(ux, -1) - 2 * ux + np.roll(ux, 1))
        rhs = -Fx - (np.roll(Fx, -1) - 2 * Fx + np.roll(Fx, 1)) / 12.0
        assert np.max(np.abs(lhs - rhs)) < 1e-10 * F0 * 1e4
    assert errs[0] < 6e-3 and errs[1] < 1.5e-3
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_shear_wave_viscosity():
    """A transverse shear wave decays at rate nu k^2 with nu = (tau - 1/2)/3 (the D2Q9
    value of the viscosity relation of Sec. II at gamma_s = 0)."""
    for tau in (1.0, 0.8):
        ny, nx = 64, 2
        k = 2 * np.pi / ny
        A = 1e-4
        u = np.zeros((2, ny, nx))
        u[0] = A * np.sin(k * (np.arange(ny) + 0.5))[:, None]
        f = O.lb_equilibrium(np.ones((ny, nx)), u)
        F = np.zeros((2, ny, nx))
        amps = []
        for t in range(400):
            f, rho, u = O.lb_step(f, F, tau)
            if t in (99, 399):
                amps.append(np.sum(u[0, :, 0] * np.sin(k * (np.arange(ny) + 0.5))) * 2 / ny)
        rate = np.log(amps[0] / amps[1]) / 300
        nu = (tau - 0.5) / 3
        assert abs(rate / (nu * k * k) - 1) < 1e-3


def test_force_single_mode_closed_form():
    """S = cos(k.r): f = -(kT/v)/dt k sin(k.r)/|k|^2, so -v beta D div f dt = S
    (Sec. II, k-space force)."""
    p = preset("cfg1")
    p.update(nx=16, ny=8, kT_over_v=1.7)
    x = (np.arange(16) + 0.5) * p["dx"]
    y = (np.arange(8) + 0.5) * p["dx"]
    X, Y = np.meshgrid(x, y)
    for mx, my in [(1, 0), (2, 3), (-3, 1)]:
        kx = 2 * np.pi * mx / (16 * p["dx"])
        ky = 2 * np.pi * my / (8 * p["dx"])
        S = np.cos(kx * X + ky * Y)
        f = O.polymer_force(S, p)
        pref = p["kT_over_v"] / p["dt"] / (kx * kx + ky * ky)
        assert np.max(np.abs(f[0] + pref * kx * np.sin(kx * X + ky * Y))) < 1e-12 * pref
        assert np.max(np.abs(f[1] + pref * ky * np.sin(kx * X + ky * Y))) < 1e-12 * pref


def test_force_irrotational_and_zero_mean():
    """App. A: the reconstructed force is irrotational; it has zero mean."""
    p = preset("cfg1")
    rng = np.random.default_rng(4)
    S = rng.standard_normal((32, 32))
    S -= S.mean()
    f = O.polymer_force(S, p)
    assert np.max(np.abs(f.mean(axis=(1, 2)))) < 1e-12
    fxh, fyh = np.fft.fft2(f[0]), np.fft.fft2(f[1])
    kx = O.wavenumbers(32, p["dx"])
    KX, KY = np.meshgrid(kx, kx)
    curl = KX * fyh - KY * fxh
    keep = np.ones((32, 32), bool)
    keep[:, 16] = False
    keep[16, :] = False
    assert np.max(np.abs(curl[keep])) < 1e-9 * np.max(np.abs(fxh))
    div = 1j * (KX * fxh + KY * fyh)
    Sh = np.fft.fft2(S)
    ref = -p["kT_over_v"] / p["dt"] * Sh
    keep[0, 0] = False
    assert np.max(np.abs(div[keep] - ref[keep])) < 1e-9 * np.max(np.abs(ref))


def test_force_dense_dft_8x8():
    """8x8: the force from explicit DFT sums (no FFT) equals the oracle's."""
    p = preset("cfg1")
    p.update(nx=8, ny=8)
    rng = np.random.default_rng(8)
    S = rng.standard_normal((8, 8))
    n = 8
    idx = np.arange(n)
    F = np.exp(-2j * np.pi * np.outer(idx, idx) / n)
    Sh = F @ S @ F.T
    m = np.where(idx < 4, idx, idx - 8)
    k = 2 * np.pi * m / (8 * p["dx"])
    fx = np.zeros((8, 8), complex)
    fy = np.zeros((8, 8), complex)
    for a in range(8):      # y index
        for b in range(8):  # x index
            k2 = k[a] ** 2 + k[b] ** 2
            if k2 == 0:
                continue
            c = p["kT_over_v"] / p["dt"] * Sh[a, b] * 1j / k2
            fx[a, b] = 0 if b == 4 else c * k[b]
            fy[a, b] = 0 if a == 4 else c * k[a]
    Fi = np.conj(F) / n
    ref = np.stack([(Fi @ fx @ Fi.T).real, (Fi @ fy @ Fi.T).real])
    assert np.max(np.abs(O.polymer_force(S, p) - ref)) < 1e-10


def test_lattice_force_units_and_external():
    p = preset("cfg1")
    S = np.zeros((32, 32))
    F = O.lattice_force(S, p)
    conv = p["dt"] ** 2 / p["dx"]
    assert abs(conv - 1.2e-5) < 1e-18
    assert np.allclose(F[0, :16], -p["g"] * conv, rtol=1e-15)
    assert np.allclose(F[0, 16:], p["g"] * conv, rtol=1e-15)
    assert np.all(F[1] == 0)


def test_advection_conservation_and_shift():
    rng = np.random.default_rng(2)
    phi = rng.random((3, 8, 10))
    w = rng.standard_normal((3, 8, 10))
    u = 0.1 * rng.standard_normal((2, 8, 10))
    pt, wt = O.advect(phi, w, u)
    assert np.allclose(pt.sum(axis=(1, 2)), phi.sum(axis=(1, 2)), rtol=1e-14)
    # uniform fields are invariant under any flow
    c = np.full((3, 8, 10), 0.3)
    pc, wc = O.advect(c, c, u)
    assert np.max(np.abs(wc - 0.3)) < 1e-15
    # a uniform Courant-1 flow in +x shifts by exactly one cell; -y likewise
    one = np.zeros((2, 8, 10)); one[0] = 1.0
    ps, ws = O.advect(phi, w, one)
    assert np.max(np.abs(ps - np.roll(phi, 1, axis=2))) < 1e-15
    assert np.max(np.abs(ws - np.roll(w, 1, axis=2))) < 1e-15
    down = np.zeros((2, 8, 10)); down[1] = -1.0
    ps, ws = O.advect(phi, w, down)
    assert np.max(np.abs(ps - np.roll(phi, -1, axis=1))) < 1e-15
    assert np.max(np.abs(ws - np.roll(w, -1, axis=1))) < 1e-15


def test_field_update_fixed_point_and_mean():
    p = preset("cfg1")
    shape = (3, 32, 32)
    phi = np.stack([np.full(shape[1:], v) for v in (0.05, 0.05, 0.9)])
    w = np.stack([np.full(shape[1:], v) for v in (0.2, -0.1, 0.4)])
    assert np.max(np.abs(O.field_update(phi, w, p) - w)) < 1e-16
    rng = np.random.default_rng(3)
    phi = phi + 0.01 * rng.standard_normal(shape)
    w = w + 0.1 * rng.standard_normal(shape)
    out = O.field_update(phi, w, p)
    assert np.allclose(out.mean(axis=(1, 2)), w.mean(axis=(1, 2)), atol=1e-15)


def test_full_step_homogeneous_start():
    """Noise-free start: the EPD fields stay uniform and the flow stays at the LB
    steady state; mass and the composition means are conserved."""
    p = preset("cfg1")
    p.update(g=1e-3)
    s = O.init_state(p, np.zeros((3, 32, 32)))
    phi0 = s["phi"].copy()
    m0 = s["fstar"].sum()
    for _ in range(20):
        s = O.step(s, p)
    assert np.max(np.abs(s["phi"] - phi0)) < 1e-14
    assert np.max(np.abs(s["omega"])) < 1e-13
    assert abs(s["fstar"].sum() - m0) < 1e-11
    prof = O.poiseuille_profile(32, O.external_force_lattice_amplitude(p), 1.0)
    assert np.max(np.abs(s["u"][0, :, 0] - prof)) < 5e-3 * np.max(np.abs(prof))


def test_full_step_noisy_conservation():
    p = preset("cfg1")
    from seeded_inputs import initial_omega
    s = O.init_state(p, initial_omega(32, 32, 1001, 1e-3))
    for _ in range(5):
        s = O.step(s, p)
    assert abs(s["phi"][0].mean() - 0.5 * p["phi_P"]) < 1e-15
    assert abs(s["phi"].sum(axis=0).mean() - 1) < 1e-14
    assert abs(s["fstar"].sum() - 32 * 32) < 1e-10
