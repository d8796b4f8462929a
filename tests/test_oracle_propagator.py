"""Pins of the oracle's chain-statistics part (Sec. II: modified diffusion
equation, split step, density integrals and Eq. phi_s) against facts fixed by
the paper and by mathematics, not by the oracle itself."""
import numpy as np
import pytest
import scipy.linalg

from oracle import epdlb_oracle as O
from seeded_inputs import preset


def small_params(nx=16, ny=12, N=10, f_A=0.37, **kw):
    p = preset("cfg1")
    p.update(nx=nx, ny=ny, n_contour=N, f_A=f_A)
    p.update(kw)
    return p


def rand_omega(p, seed=3, amp=0.4):
    rng = np.random.default_rng(seed)
    return amp * rng.standard_normal((3, p["ny"], p["nx"]))


def test_node_weights_sum_to_block_fractions():
    for N, fA in [(16, 0.5), (64, 0.3), (32, 0.3), (17, 0.882), (10, 0.37)]:
        wA, wB = O.node_weights(N, fA)
        assert abs(wA.sum() - fA) < 1e-15
        assert abs(wB.sum() - (1 - fA)) < 1e-15
        assert np.all(wA >= 0) and np.all(wB >= 0)


def test_homogeneous_closed_form():
    """Constant fields: q_j = exp(-ds N sum_{i<j} w_i), Q_P/V = exp(-N(f_A a + (1-f_A) b)),
    Phi_A = f_A phibar_P, Phi_B = (1-f_A) phibar_P, Phi_S = 1 - phibar_P."""
    p = small_params(N=16, f_A=0.3)  # f_A N = 4.8: junction segment
    alpha, beta, gam = 0.7, -0.4, 0.25
    shape = (p["ny"], p["nx"])
    wA, wB = np.full(shape, alpha), np.full(shape, beta)
    q, qb = O.propagate(wA, wB, p, gauge=(0.0, 0.0))
    N = p["n_contour"]
    f_A = p["f_A"]
    # segment fields written out directly from the block structure
    acc = 0.0
    for j in range(N + 1):
        assert np.allclose(q[j], np.exp(-acc), rtol=1e-14, atol=0)
        if j < N:
            lo, hi = j / N, (j + 1) / N
            frac_A = max(0.0, min(hi, f_A) - lo) * N
            acc += frac_A * alpha + (1 - frac_A) * beta
    d = O.densities(np.stack([wA, wB, np.full(shape, gam)]), p, gauge=(0.0, 0.0, 0.0))
    V = p["nx"] * p["ny"] * p["dx"] ** 2
    assert abs(d["Q_P"] / V - np.exp(-N * (f_A * alpha + (1 - f_A) * beta))) < 1e-14 * np.exp(
        -N * (f_A * alpha + (1 - f_A) * beta))
    assert abs(d["Q_S"] / V - np.exp(-gam)) < 1e-15
    assert np.allclose(d["phi"][0], f_A * p["phi_P"], rtol=1e-14, atol=0)
    assert np.allclose(d["phi"][1], (1 - f_A) * p["phi_P"], rtol=1e-14, atol=0)
    assert np.allclose(d["phi"][2], 1 - p["phi_P"], rtol=1e-14, atol=0)


def test_heat_kernel_plane_wave():
    """A lattice plane wave cos(k.r) is an eigenfunction: K cos = exp(-R_G^2 |k|^2 ds) cos,
    with k = 2 pi m / (n dx) at cell centres (x + 1/2) dx."""
    p = small_params(nx=16, ny=12, N=8, R_G=1.3)
    x = (np.arange(p["nx"]) + 0.5) * p["dx"]
    y = (np.arange(p["ny"]) + 0.5) * p["dx"]
    X, Y = np.meshgrid(x, y)
    for mx, my in [(1, 0), (0, 1), (3, 2), (-5, 4), (8, 6)]:
        kx = 2 * np.pi * mx / (p["nx"] * p["dx"])
        ky = 2 * np.pi * my / (p["ny"] * p["dx"])
        g = np.cos(kx * X + ky * Y)
        expect = np.exp(-p["R_G"] ** 2 * (kx ** 2 + ky ** 2) / p["n_contour"]) * g
        assert np.max(np.abs(O.apply_heat_kernel(g, p) - expect)) < 1e-14


def test_split_step_constant_field_plane_wave():
    """One split step on cos(k.r) in a constant field w: exp(-N w ds) exp(-R_G^2 k^2 ds) cos."""
    p = small_params(nx=8, ny=8, N=4, f_A=1.0)
    x = (np.arange(8) + 0.5) * p["dx"]
    X, Y = np.meshgrid(x, x)
    k = 2 * np.pi * 2 / (8 * p["dx"])
    g0 = np.cos(k * X)
    w = 0.9
    ds = 1.0 / p["n_contour"]
    E = np.exp(-p["n_contour"] * w * ds / 2)
    g1 = E * O.apply_heat_kernel(E * g0, p)
    assert np.max(np.abs(g1 - np.exp(-p["n_contour"] * w * ds) * np.exp(-k * k * ds) * g0)) < 1e-15


def test_adjoint_symmetry_and_Q_fwd_equals_bwd():
    p = small_params()
    w = rand_omega(p)
    q, qb = O.propagate(w[0], w[1], p)
    N = p["n_contour"]
    ref = np.sum(q[N])
    for j in range(N + 1):
        assert abs(np.sum(q[j] * qb[N - j]) - ref) < 2e-14 * abs(ref)
    assert abs(np.sum(qb[N]) - ref) < 2e-14 * abs(ref)


def test_density_is_log_derivative_of_QP():
    """Phi_A(r) = -(V phibar_P / (N dA)) d ln Q_P / d w_A(r), by central differences
    with the gauge constants held fixed; likewise Phi_B."""
    p = small_params(nx=8, ny=6, N=7, f_A=0.45)
    w = rand_omega(p, seed=11, amp=0.5)
    gauge = (0.1, -0.2, 0.0)
    d = O.densities(w, p, gauge=gauge)
    dA = p["dx"] ** 2
    V = p["nx"] * p["ny"] * dA
    N = p["n_contour"]
    h = 1e-5
    for species in (0, 1):
        for (yy, xx) in [(0, 0), (2, 5), (5, 7)]:
            wp = w.copy(); wp[species, yy, xx] += h
            wm = w.copy(); wm[species, yy, xx] -= h
            lp = np.log(O.densities(wp, p, gauge=gauge)["Q_P"])
            lm = np.log(O.densities(wm, p, gauge=gauge)["Q_P"])
            fd = -(V * p["phi_P"] / (N * dA)) * (lp - lm) / (2 * h)
            assert abs(fd - d["phi"][species, yy, xx]) < 1e-8 * abs(d["phi"][species, yy, xx])


def test_solvent_density_is_log_derivative_of_QS():
    p = small_params(nx=8, ny=6, N=4)
    w = rand_omega(p, seed=5)
    gauge = (0.0, 0.0, 0.3)
    d = O.densities(w, p, gauge=gauge)
    dA = p["dx"] ** 2
    V = p["nx"] * p["ny"] * dA
    h = 1e-6
    wp = w.copy(); wp[2, 3, 4] += h
    wm = w.copy(); wm[2, 3, 4] -= h
    fd = -(V * (1 - p["phi_P"]) / dA) * (np.log(O.densities(wp, p, gauge=gauge)["Q_S"]) -
                                         np.log(O.densities(wm, p, gauge=gauge)["Q_S"])) / (2 * h)
    assert abs(fd - d["phi"][2, 3, 4]) < 1e-8


def test_gauge_translation_reflection_invariance():
    p = small_params()
    w = rand_omega(p, seed=7)
    d0 = O.densities(w, p)["phi"]
    # gauge: shifts of each species' potential leave all densities unchanged
    d1 = O.densities(w + np.array([0.3, -1.1, 0.7])[:, None, None], p)["phi"]
    assert np.max(np.abs(d1 - d0)) < 1e-14
    d2 = O.densities(w, p, gauge=(0.5, -0.5, 0.2))["phi"]
    assert np.max(np.abs(d2 - d0)) < 1e-14
    # lattice translation
    wt = np.roll(w, (3, -5), axis=(1, 2))
    assert np.max(np.abs(O.densities(wt, p)["phi"] - np.roll(d0, (3, -5), axis=(1, 2)))) < 1e-14
    # reflection x -> -x about the box centre maps cell x to nx-1-x
    wr = w[:, :, ::-1]
    assert np.max(np.abs(O.densities(wr, p)["phi"] - d0[:, :, ::-1])) < 1e-14


def test_compressibility_means():
    p = small_params()
    w = rand_omega(p, seed=9, amp=0.8)
    phi = O.densities(w, p)["phi"]
    assert abs(phi[0].mean() - p["f_A"] * p["phi_P"]) < 1e-15
    assert abs(phi[1].mean() - (1 - p["f_A"]) * p["phi_P"]) < 1e-15
    assert abs(phi[2].mean() - (1 - p["phi_P"])) < 1e-15
    assert abs(phi.sum(axis=0).mean() - 1.0) < 1e-15


def _dft_matrix(n):
    m = np.arange(n)
    return np.exp(-2j * np.pi * np.outer(m, m) / n)


def test_brute_force_8x8_dense():
    """8x8 grid: K = expm(R_G^2 ds L), L the spectral Laplacian built from explicit
    DFT matrices (no FFT); dense chain products and dense density sums."""
    p = small_params(nx=8, ny=8, N=6, f_A=0.4)
    n = 8
    F = _dft_matrix(n)
    Finv = np.conj(F) / n
    m = np.arange(n)
    m = np.where(m < n // 2, m, m - n)
    k = 2 * np.pi * m / (n * p["dx"])
    L1 = (Finv @ np.diag(-k ** 2) @ F).real
    I8 = np.eye(n)
    Lap = np.kron(I8, L1) + np.kron(L1, I8)  # index y*8 + x
    N = p["n_contour"]
    ds = 1.0 / N
    K = scipy.linalg.expm(p["R_G"] ** 2 * ds * Lap)
    w = rand_omega(p, seed=21, amp=0.6)
    gauge = (0.05, -0.1, 0.2)
    wA = w[0].reshape(-1) - gauge[0]
    wB = w[1].reshape(-1) - gauge[1]
    # segment A-content from the block picture: share of [j/N, (j+1)/N] below f_A
    segs = []
    for j in range(N):
        a = max(0.0, min((j + 1) / N, p["f_A"]) - j / N) * N
        segs.append(np.diag(np.exp(-(a * wA + (1 - a) * wB) / 2)))
    q = [np.ones(64)]
    qb = [np.ones(64)]
    for j in range(N):
        q.append(segs[j] @ K @ segs[j] @ q[-1])
        qb.append(segs[N - 1 - j] @ K @ segs[N - 1 - j] @ qb[-1])
    qo, qbo = O.propagate(w[0], w[1], p, gauge=gauge[:2])
    for j in range(N + 1):
        assert np.max(np.abs(qo[j].reshape(-1) - q[j])) < 1e-12 * np.max(np.abs(q[j]))
        assert np.max(np.abs(qbo[j].reshape(-1) - qb[j])) < 1e-12 * np.max(np.abs(qb[j]))
    # densities from the trapezoid rule over each block, written out per segment
    dA = p["dx"] ** 2
    V = 64 * dA
    QP = dA * q[N].sum()
    phiA = np.zeros(64)
    phiB = np.zeros(64)
    for j in range(N):
        a = max(0.0, min((j + 1) / N, p["f_A"]) - j / N) * N
        trap = 0.5 * ds * (q[j] * qb[N - j] + q[j + 1] * qb[N - j - 1])
        phiA += a * trap
        phiB += (1 - a) * trap
    phiA *= V * p["phi_P"] / QP
    phiB *= V * p["phi_P"] / QP
    d = O.densities(w, p, gauge=gauge)
    assert np.max(np.abs(d["phi"][0].reshape(-1) - phiA)) < 1e-12
    assert np.max(np.abs(d["phi"][1].reshape(-1) - phiB)) < 1e-12
    assert abs(d["Q_P"] - QP) < 1e-12 * QP
