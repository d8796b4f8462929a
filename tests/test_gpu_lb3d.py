"""GPU parity of the three-dimensional fluid (D3Q19, epdlb_lb3_* in the C ABI)
against the FP64 oracle oracle/lb3d_oracle.py on the same seeded inputs.

Bars: FP64 storage agrees with the oracle to 1e-13 (rounding order only);
FP32 storage keeps the deviations f_i - w_i, whose size here is at most
about 0.05, to a few ulps per step: 5e-7 absolute on populations and
velocities after a few steps.  Boxes are ragged against the kernel's tiling
(64-site row chunks, 4 rows per block) and include the degenerate widths 1.
At the benchmark's size (256^3, FP32) one step is checked at sampled sites
(including the faces, where the streaming wraps) with the oracle's per-site
step, and the exact balances (mass, momentum gain = total force) over the
whole box after further steps.
"""
import sys

import numpy as np
import pytest

from oracle import lb3d_oracle as L

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _fluid(nx, ny, nz, tau, precision):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1804_02883_amd import Fluid3D
    return Fluid3D(nx, ny, nz, tau, precision)


def _state(shape, seed, amp=0.05, famp=1e-3):
    rng = np.random.default_rng(seed)
    rho = 1 + amp * rng.standard_normal(shape)
    u = amp * rng.standard_normal((3,) + shape)
    f = L.equilibrium(rho, u) + amp / 36 * rng.standard_normal((19,) + shape)
    F = famp * rng.standard_normal((3,) + shape)
    return f, F


SHAPES = [(6, 10, 40), (3, 5, 130), (1, 1, 1), (2, 3, 1), (1, 7, 64), (5, 4, 65)]


@pytest.mark.parametrize("prec,tol", [(0, 1e-13), (1, 5e-7)])
@pytest.mark.parametrize("shape", SHAPES)
def test_steps_vs_oracle(shape, prec, tol):
    nz, ny, nx = shape
    say(f"[lb3] {nz}x{ny}x{nx} precision={prec} 4 steps")
    tau = 0.8
    f, F = _state(shape, nx * 7 + ny * 3 + nz)
    fl = _fluid(nx, ny, nz, tau, prec)
    fl.set_populations(f)
    fl.set_force(F)
    if prec == 1:  # the device holds FP32 deviations: start the oracle from those
        w = L.W19[:, None, None, None]
        f = w + (f - w).astype(np.float32).astype(np.float64)
        F = F.astype(np.float32).astype(np.float64)
    fl.step(4)
    for _ in range(4):
        f, rho, u = L.step(f, F, tau)
    got = fl.populations()
    grho, gu = fl.velocity()
    err = np.max(np.abs(got - f))
    say(f"  max |f - oracle| {err:.2e}, u {np.max(np.abs(gu - u)):.2e}")
    assert err < tol
    assert np.max(np.abs(grho - rho)) < tol and np.max(np.abs(gu - u)) < tol
    fl.close()


def test_equilibrium_and_rest_start():
    nz, ny, nx = 3, 6, 70
    rng = np.random.default_rng(5)
    rho = 1 + 0.1 * rng.standard_normal((nz, ny, nx))
    u = 0.05 * rng.standard_normal((3, nz, ny, nx))
    fl = _fluid(nx, ny, nz, 1.0, 0)
    # a new context is at rest: f = w everywhere
    assert np.max(np.abs(fl.populations() - L.W19[:, None, None, None])) == 0.0
    fl.set_equilibrium(rho, u)
    assert np.max(np.abs(fl.populations() - L.equilibrium(rho, u))) < 1e-15
    fl.set_equilibrium(None, u)
    assert np.max(np.abs(fl.populations() - L.equilibrium(np.ones_like(rho), u))) < 1e-15
    fl.set_equilibrium(rho, None)
    assert np.max(np.abs(fl.populations() - L.equilibrium(rho, np.zeros_like(u)))) < 1e-15
    fl.close()


def test_argument_and_state_errors():
    from paper_1804_02883_amd import EpdlbError, Fluid3D
    _fluid(4, 4, 4, 1.0, 0).close()  # skips without a GPU
    for args in [(0, 4, 4, 1.0), (4, 4, 5000, 1.0), (4, 4, 4, 0.5), (4, 4, 4, float("nan"))]:
        with pytest.raises(EpdlbError):
            Fluid3D(*args)
    with pytest.raises(EpdlbError):
        Fluid3D(4, 4, 4, 1.0, precision=2)
    fl = _fluid(4, 4, 4, 1.0, 1)
    with pytest.raises(EpdlbError):  # no step yet
        fl.velocity()
    bad = np.tile(L.W19[:, None, None, None], (1, 4, 4, 4))
    bad[3, 1, 2, 3] = np.inf
    with pytest.raises(EpdlbError):
        fl.set_populations(bad)
    with pytest.raises(EpdlbError):
        fl.set_equilibrium(np.zeros((4, 4, 4)), None)
    with pytest.raises(EpdlbError):
        fl.set_force(np.full((3, 4, 4, 4), np.nan))
    fl.step(0)
    with pytest.raises(EpdlbError):
        fl.velocity()
    fl.step(1)
    rho, u = fl.velocity()
    assert np.all(rho == 1.0) and np.all(u == 0.0)
    fl.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_kolmogorov_flow_on_the_gpu(prec):
    """F_x = F0 sin(k y) on a 64 x 32 x 2 box settles at F0 sin(k y)/(nu k^2)
    (to O(k^2), as in the oracle's pin), uniform in x and z."""
    nz, ny, nx, tau, F0 = 2, 32, 64, 1.0, 1e-5
    k = 2 * np.pi / ny
    y = np.arange(ny, dtype=np.float64)
    F = np.zeros((3, nz, ny, nx))
    F[0] = F0 * np.sin(k * y)[None, :, None]
    fl = _fluid(nx, ny, nz, tau, prec)
    fl.set_force(F)
    fl.step(3000)
    rho, u = fl.velocity()
    prof = u[0].mean(axis=(0, 2))
    got = 2 * np.mean(prof * np.sin(k * y))
    want = F0 / (L.viscosity(tau) * k * k)
    say(f"  precision {prec}: amplitude / closed form {got / want:.5f}")
    assert abs(got / want - 1) < 5e-3
    assert np.max(np.abs(u[0] - prof[None, :, None])) < 1e-6 * want
    # no cross flow: exact in FP64, FP32 rounding relaxes over about 1/(nu k^2) steps
    assert np.max(np.abs(u[1:])) < (1e-9 if prec == 0 else 1e-4) * want
    fl.close()


def test_full_size_sampled_step_and_balances():
    """256^3, FP32, tau = 0.8: one step at 4000 sampled sites (and all 8
    corners) against the oracle's per-site step; then 3 more steps and the
    balances over the whole box."""
    n = 256
    shape = (n, n, n)
    say("[lb3] 256^3 FP32: generating the seeded state")
    rng = np.random.default_rng(2024)
    w = L.W19[:, None, None, None]
    dev = (0.01 * rng.standard_normal((19,) + shape, dtype=np.float32)) * w.astype(np.float32)
    f = dev.astype(np.float64) + w
    del dev
    F = (1e-4 * rng.standard_normal((3,) + shape, dtype=np.float32)).astype(np.float64)
    tau = 0.8
    fl = _fluid(n, n, n, tau, 1)
    fl.set_populations(f)
    fl.set_force(F)
    ms = fl.profile(1)
    say(f"  one launch {ms[0]:.3f} ms")
    got = fl.populations()
    rho_g, u_g = fl.velocity()
    sites = [tuple(int(v) for v in rng.integers(0, n, 3)) for _ in range(4000)]
    sites += [(z, y, x) for z in (0, n - 1) for y in (0, n - 1) for x in (0, n - 1)]
    worst = 0.0
    for (z, y, x) in sites:
        o, r, v = L.site(f, F, tau, z, y, x)
        worst = max(worst, np.max(np.abs(got[:, z, y, x] - o)), abs(rho_g[z, y, x] - r),
                    np.max(np.abs(u_g[:, z, y, x] - v)))
    say(f"  sampled max error {worst:.2e}")
    assert worst < 5e-7
    # balances of the GPU's own steps: mass exact, momentum grows by the total force
    c = L.C19.astype(np.float64)

    def totals(a):
        sums = [float(a[i].sum(dtype=np.float64)) for i in range(19)]
        return sum(sums), [sum(c[i, d] * sums[i] for i in range(19)) for d in range(3)]

    m0, j0 = totals(got)
    del f
    fl.step(3)
    m1, j1 = totals(fl.populations())
    N = float(n ** 3)
    say(f"  mass change per site {(m1 - m0) / N:.2e}")
    assert abs(m1 - m0) / N < 1e-9
    for d in range(3):
        gain = (j1[d] - j0[d]) - 3 * F[d].sum()
        assert abs(gain) / N < 1e-9, (d, gain / N)
    fl.close()


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 1e-4)])
def test_reverse_poiseuille_channel_on_the_gpu(prec, tol):
    """A 48 x 32 x 3 box under the paper's drive (-F0 below the middle in y,
    +F0 above) for 4000 steps: uniform in x and z, equal to the oracle's
    channel of one column (relative to the peak speed), and within the
    lattice's 1.5e-3 of Eq. flow_field."""
    from oracle import epdlb_oracle as O
    nz, ny, nx, F0, steps = 3, 32, 48, 1e-6, 4000
    Y = np.arange(ny) + 0.5
    Fx = np.where(Y < ny / 2, -F0, F0)
    F = np.zeros((3, nz, ny, nx))
    F[0] = Fx[None, :, None]
    fl = _fluid(nx, ny, nz, 1.0, prec)
    fl.set_force(F)
    fl.step(steps)
    rho, u = fl.velocity()
    fl.close()
    f = L.equilibrium(np.ones((1, ny, 1)), np.zeros((3, 1, ny, 1)))
    F1 = np.zeros((3, 1, ny, 1))
    F1[0, 0, :, 0] = Fx
    for _ in range(steps):
        f, _, u1 = L.step(f, F1, 1.0)
    ref = u1[0, 0, :, 0]
    peak = np.max(np.abs(ref))
    err = np.max(np.abs(u[0] - ref[None, :, None])) / peak
    exact = O.poiseuille_profile(ny, F0, 1.0)
    say(f"  precision {prec}: |u - oracle| / peak {err:.2e}, "
        f"|u - Eq. flow_field| / peak {np.max(np.abs(u[0, 0, :, 0] - exact)) / peak:.2e}")
    assert err < tol
    assert np.max(np.abs(u[0, 1, :, 7] - exact)) / np.max(np.abs(exact)) < 1.5e-3
    # no cross flow beyond the rounding of the stored populations
    assert np.max(np.abs(u[1:])) < (1e-14 if prec == 0 else 1e-9)


# --- the multi-relaxation collision (epdlb_lb3_set_collision) ---

GAMMAS = [(0.2, -0.5, 0.0), (-0.3, 0.6, 0.4)]


@pytest.mark.parametrize("gam", GAMMAS)
@pytest.mark.parametrize("prec,tol", [(0, 1e-13), (1, 5e-7)])
@pytest.mark.parametrize("shape", [(6, 10, 40), (3, 5, 130), (1, 1, 1), (5, 4, 65)])
def test_mrt_steps_vs_oracle(shape, prec, tol, gam):
    nz, ny, nx = shape
    say(f"[lb3 mrt] {nz}x{ny}x{nx} precision={prec} gammas={gam} 4 steps")
    f, F = _state(shape, nx * 5 + ny + nz)
    fl = _fluid(nx, ny, nz, 1.0, prec)
    fl.set_collision(1, *gam)
    fl.set_populations(f)
    fl.set_force(F)
    if prec == 1:
        w = L.W19[:, None, None, None]
        f = w + (f - w).astype(np.float32).astype(np.float64)
        F = F.astype(np.float32).astype(np.float64)
    fl.step(4)
    for _ in range(4):
        f, rho, u = L.step_mrt(f, F, *gam)
    got = fl.populations()
    grho, gu = fl.velocity()
    err = np.max(np.abs(got - f))
    say(f"  max |f - oracle| {err:.2e}")
    assert err < tol
    assert np.max(np.abs(grho - rho)) < tol and np.max(np.abs(gu - u)) < tol
    fl.close()


def test_mrt_equal_rates_match_bgk_kernel_and_errors():
    """Factors 1 - 1/tau reproduce the BGK kernel at tau (FP64, to rounding);
    factors outside (-1, 1) are rejected; mrt = 0 returns to BGK."""
    from paper_1804_02883_amd import EpdlbError
    shape = (4, 6, 70)
    f, F = _state(shape, 99)
    out = []
    for mrt in (0, 1):
        fl = _fluid(70, 6, 4, 0.8, 0)
        if mrt:
            fl.set_collision(1, 1 - 1 / 0.8, 1 - 1 / 0.8, 1 - 1 / 0.8)
        fl.set_populations(f)
        fl.set_force(F)
        fl.step(3)
        out.append(fl.populations())
        for bad in [(1.0, 0.0, 0.0), (0.0, -1.0, 0.0), (0.0, 0.0, float("nan"))]:
            with pytest.raises(EpdlbError):
                fl.set_collision(1, *bad)
        with pytest.raises(EpdlbError):
            fl.set_collision(2)
        fl.close()
    assert np.max(np.abs(out[0] - out[1])) < 1e-15


def test_mrt_full_size_sampled_step():
    """256^3 FP32 with the multi-relaxation collision: one step at 2000 sampled
    sites and the 8 corners against the oracle's per-site step."""
    n = 256
    shape = (n, n, n)
    gam = (0.2, -0.5, 0.1)
    rng = np.random.default_rng(2025)
    w = L.W19[:, None, None, None]
    dev = (0.01 * rng.standard_normal((19,) + shape, dtype=np.float32)) * w.astype(np.float32)
    f = dev.astype(np.float64) + w
    del dev
    F = (1e-4 * rng.standard_normal((3,) + shape, dtype=np.float32)).astype(np.float64)
    fl = _fluid(n, n, n, 1.0, 1)
    fl.set_collision(1, *gam)
    fl.set_populations(f)
    fl.set_force(F)
    ms = fl.profile(1)
    say(f"  one multi-relaxation launch {ms[0]:.3f} ms")
    got = fl.populations()
    rho_g, u_g = fl.velocity()
    fl.close()
    sites = [tuple(int(v) for v in rng.integers(0, n, 3)) for _ in range(2000)]
    sites += [(z, y, x) for z in (0, n - 1) for y in (0, n - 1) for x in (0, n - 1)]
    worst = 0.0
    for (z, y, x) in sites:
        o, r, v = L.site(f, F, 0.0, z, y, x, mrt=gam)
        worst = max(worst, np.max(np.abs(got[:, z, y, x] - o)), abs(rho_g[z, y, x] - r),
                    np.max(np.abs(u_g[:, z, y, x] - v)))
    say(f"  sampled max error {worst:.2e}")
    assert worst < 5e-7


def test_mrt_channel_uses_the_shear_viscosity():
    """The reverse-Poiseuille drive with the multi-relaxation collision
    (gamma_s = 0.2, gamma_b = -0.5, gamma_g = 0), FP64, 4000 steps: equal to the
    oracle's one-column channel, and Eq. flow_field with
    nu = (1/6)(1 + gamma_s)/(1 - gamma_s) within 5e-3 (the oracle's own
    discretisation error here is 3.9e-3)."""
    from oracle import epdlb_oracle as O
    nz, ny, nx, F0, steps = 2, 32, 64, 1e-6, 4000
    gs, gb = 0.2, -0.5
    Y = np.arange(ny) + 0.5
    Fx = np.where(Y < ny / 2, -F0, F0)
    F = np.zeros((3, nz, ny, nx))
    F[0] = Fx[None, :, None]
    fl = _fluid(nx, ny, nz, 1.0, 0)
    fl.set_collision(1, gs, gb, 0.0)
    fl.set_force(F)
    fl.step(steps)
    _, u = fl.velocity()
    fl.close()
    f = L.equilibrium(np.ones((1, ny, 1)), np.zeros((3, 1, ny, 1)))
    F1 = np.zeros((3, 1, ny, 1))
    F1[0, 0, :, 0] = Fx
    for _ in range(steps):
        f, _, u1 = L.step_mrt(f, F1, gs, gb, 0.0)
    ref = u1[0, 0, :, 0]
    peak = np.max(np.abs(ref))
    err = np.max(np.abs(u[0] - ref[None, :, None])) / peak
    nu = L.mrt_viscosities(gs, gb)[0]
    exact = O.poiseuille_profile(ny, F0, 1.0, nu=nu)
    err_ex = np.max(np.abs(u[0, 1, :, 5] - exact)) / np.max(np.abs(exact))
    say(f"  |u - oracle| / peak {err:.2e}, |u - Eq. flow_field| / peak {err_ex:.2e}")
    assert err < 1e-10
    assert err_ex < 5e-3


@pytest.mark.parametrize("shape", [(1, 1, 4096), (1, 4096, 1), (4096, 1, 1), (2, 3, 4096)])
def test_maximum_side_vs_oracle(shape):
    """A side at the 4096 limit: a wave walking 64 chunks of one row, a grid of
    1024 row blocks, or 4096 z-planes (the grid's second dimension); FP64,
    both collisions, 2 steps."""
    nz, ny, nx = shape
    say(f"[lb3] maximum side {nz}x{ny}x{nx}")
    f0, F = _state(shape, 4096 + nx + 2 * ny)
    for gam in (None, (0.2, -0.5, 0.3)):
        fl = _fluid(nx, ny, nz, 0.9, 0)
        if gam:
            fl.set_collision(1, *gam)
        fl.set_populations(f0)
        fl.set_force(F)
        fl.step(2)
        f = f0
        for _ in range(2):
            f = (L.step(f, F, 0.9) if gam is None else L.step_mrt(f, F, *gam))[0]
        assert np.max(np.abs(fl.populations() - f)) < 1e-13
        fl.close()


@pytest.mark.parametrize("mrt", [0, 1])
def test_fp32_long_run_balances(mrt):
    """48^3 FP32 under a zero-mean random force, 500 steps: no systematic mass
    drift (below 1e-7 per site, against 500 steps of single-precision rounding
    of deviations near 1e-3), and the momentum gain equals 500 times the total
    force to the same order."""
    n, steps = 48, 500
    shape = (n, n, n)
    rng = np.random.default_rng(48)
    F = 1e-6 * rng.standard_normal((3,) + shape)
    F -= F.mean(axis=(1, 2, 3), keepdims=True)
    F = F.astype(np.float32).astype(np.float64)
    fl = _fluid(n, n, n, 0.8, 1)
    if mrt:
        fl.set_collision(1, 1 - 1 / 0.8, 0.3, 0.0)
    fl.set_equilibrium(1 + 1e-3 * rng.standard_normal(shape), 1e-3 * rng.standard_normal((3,) + shape))
    c = L.C19.astype(np.float64)

    def totals(a):
        sums = [float(a[i].sum(dtype=np.float64)) for i in range(19)]
        return sum(sums), np.array([sum(c[i, d] * sums[i] for i in range(19)) for d in range(3)])

    m0, j0 = totals(fl.populations())
    fl.step(steps)
    m1, j1 = totals(fl.populations())
    fl.close()
    N = float(n ** 3)
    drift = (m1 - m0) / N
    dj = (j1 - j0 - steps * F.reshape(3, -1).sum(axis=1)) / N
    say(f"  collision {'mrt' if mrt else 'bgk'}: mass drift per site {drift:.2e}, momentum {np.max(np.abs(dj)):.2e}")
    assert abs(drift) < 1e-7
    assert np.max(np.abs(dj)) < 1e-7
