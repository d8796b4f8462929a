"""Pins of the oracle's chemical potential, EPD field update and advection
against what the paper and the mathematics fix.

* The chemical potential is the derivative of the free energy of Sec. II
  (Eq. free_energy): checked against central differences of the local free
  energy density at fixed potentials, and against the derivative of the whole
  functional (with its ln Q_P and ln Q_S terms) along a path of potentials,
  where the potentials' own derivative cancels against the density integrals.
  Distinct chi_AB, chi_AS, chi_BS, a non-zero kappa_H and distinct
  diffusivities make a sign, a swapped pair or a wrong species visible.
* One field update (Eq. diff_w with the 5-point Laplacian) of a single
  Fourier mode has a closed-form response per species.
* Advection: a hand-computed 3 x 3 case (tests/golden/advect_3x3.json) whose
  velocity varies along its own axis fixes the face-velocity average and the
  donor cell of the flux form, and the upwind rule of the potentials' step.
"""
import json
import os

import numpy as np
import pytest

from oracle import epdlb_oracle as O
from seeded_inputs import preset

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def distinct_params(**kw):
    p = preset("cfg1", nx=8, ny=8, n_contour=6, f_A=0.4, phi_P=0.2)
    p.update(chi_AB=0.9, chi_AS=1.7, chi_BS=-0.35, kappa_H=2.3, D_A=0.11, D_B=0.23, D_S=0.71)
    p.update(kw)
    return p


def local_free_energy(phi, omega, p):
    """Integrand of Eq. free_energy, written from the printed functional:
    1/2 sum_{I, J != I} chi_IJ Phi_I Phi_J - sum_I w_I Phi_I + kappa_H/2 (sum_I Phi_I - 1)^2."""
    A, B, S = phi
    pair = p["chi_AB"] * A * B + p["chi_AS"] * A * S + p["chi_BS"] * B * S  # each unordered pair once
    lin = omega[0] * A + omega[1] * B + omega[2] * S
    return pair - lin + 0.5 * p["kappa_H"] * (A + B + S - 1.0) ** 2


def test_mu_is_the_local_free_energy_derivative():
    p = distinct_params()
    rng = np.random.default_rng(11)
    phi = 0.2 + 0.6 * rng.random((3, 5, 7))
    omega = rng.standard_normal((3, 5, 7))
    mu = O.chemical_potential(phi, omega, p)
    h = 1e-6
    for I in range(3):
        e = np.zeros_like(phi)
        e[I] = h
        fd = (local_free_energy(phi + e, omega, p) - local_free_energy(phi - e, omega, p)) / (2 * h)
        assert np.max(np.abs(mu[I] - fd)) < 1e-8, I
    # the three species see clearly different potentials here
    assert np.mean(np.abs(mu[0] - mu[1])) > 0.1 and np.mean(np.abs(mu[1] - mu[2])) > 0.1


def total_free_energy(omega, p):
    """Eq. free_energy at Phi = Phi[omega] (gauge constants zero):
    -phibar_S V ln(Q_S/(V phibar_S)) - (phibar_P/N) V ln(Q_P N/(V phibar_P)) + dA sum_r f(Phi, omega)."""
    d = O.densities(omega, p, gauge=(0.0, 0.0, 0.0))
    dA = p["dx"] ** 2
    V = p["nx"] * p["ny"] * dA
    N = p["n_contour"]
    phiP = p["phi_P"]
    phiS = 1.0 - phiP
    Fid = -phiS * V * np.log(d["Q_S"] / (V * phiS)) - phiP / N * V * np.log(d["Q_P"] * N / (V * phiP))
    return Fid + dA * float(np.sum(local_free_energy(d["phi"], omega, p))), d["phi"]


def test_mu_is_the_derivative_of_the_whole_functional():
    """dF/de along omega + e v equals dA sum_r mu . dPhi/de: the explicit omega
    dependence of the ln Q terms cancels the -sum w Phi term exactly on the
    grid (trapezoid contour weights), so mu alone carries the derivative."""
    p = distinct_params()
    rng = np.random.default_rng(5)
    omega = 0.3 * rng.standard_normal((3, 8, 8))
    v = rng.standard_normal((3, 8, 8))
    h = 1e-5
    Fp, phip = total_free_energy(omega + h * v, p)
    Fm, phim = total_free_energy(omega - h * v, p)
    dF = (Fp - Fm) / (2 * h)
    F0, phi0 = total_free_energy(omega, p)
    mu = O.chemical_potential(phi0, omega, p)
    dphi = (phip - phim) / (2 * h)
    rhs = p["dx"] ** 2 * float(np.sum(mu * dphi))
    assert abs(dF - rhs) < 1e-8 * max(1.0, abs(dF)), (dF, rhs)
    assert abs(dF) > 1e-3


def lap_eigenvalue(mx, my, nx, ny):
    """-Lambda of the 5-point Laplacian on the mode cos(2 pi (mx x/nx + my y/ny))."""
    return -(4.0 - 2.0 * np.cos(2 * np.pi * mx / nx) - 2.0 * np.cos(2 * np.pi * my / ny))


@pytest.mark.parametrize("I", [0, 1, 2])
def test_field_update_single_mode_in_omega(I):
    """Uniform Phi, a single mode a cos(k.r) in omega_I only: mu_I = const - omega_I,
    so Eq. diff_w gives omega_I' = const + a (1 - D_I dt Lambda / dx^2) cos(k.r);
    the other potentials are untouched."""
    p = distinct_params(nx=16, ny=8)
    ny, nx = 8, 16
    y, x = np.mgrid[0:ny, 0:nx]
    mode = np.cos(2 * np.pi * (3 * x / nx + 1 * y / ny))
    phi = np.stack([np.full((ny, nx), v) for v in (0.07, 0.11, 0.8)])
    base = np.array([0.4, -0.2, 0.1])
    omega = base[:, None, None] * np.ones((3, ny, nx))
    a = 0.05
    omega[I] += a * mode
    out = O.field_update(phi, omega, p)
    D = (p["D_A"], p["D_B"], p["D_S"])[I]
    lam = -lap_eigenvalue(3, 1, nx, ny)
    expect = base[I] + a * (1.0 - D * p["dt"] * lam / p["dx"] ** 2) * mode
    assert np.max(np.abs(out[I] - expect)) < 1e-14
    for J in range(3):
        if J != I:
            assert np.max(np.abs(out[J] - base[J])) < 1e-15


@pytest.mark.parametrize("J", [0, 1, 2])
def test_field_update_single_mode_in_phi(J):
    """Uniform omega, a single mode b cos(k.r) in Phi_J only: mu_I gains
    (chi_IJ [I != J] + kappa_H) b cos(k.r), so omega_I' = omega_I
    + D_I dt Lambda (chi_IJ [I != J] + kappa_H) b cos(k.r) / dx^2."""
    p = distinct_params(nx=8, ny=16)
    ny, nx = 16, 8
    y, x = np.mgrid[0:ny, 0:nx]
    mode = np.cos(2 * np.pi * (1 * x / nx + 2 * y / ny))
    phi = np.stack([np.full((ny, nx), v) for v in (0.07, 0.11, 0.8)])
    b = 0.01
    phi[J] += b * mode
    base = np.array([0.4, -0.2, 0.1])
    omega = base[:, None, None] * np.ones((3, ny, nx))
    out = O.field_update(phi, omega, p)
    chi = {(0, 1): p["chi_AB"], (0, 2): p["chi_AS"], (1, 2): p["chi_BS"]}
    lam = -lap_eigenvalue(1, 2, nx, ny)
    for I in range(3):
        c = p["kappa_H"] + (chi[tuple(sorted((I, J)))] if I != J else 0.0)
        D = (p["D_A"], p["D_B"], p["D_S"])[I]
        expect = base[I] + D * p["dt"] * lam * c * b * mode / p["dx"] ** 2
        assert np.max(np.abs(out[I] - expect)) < 1e-15, (I, J)


def test_advect_hand_computed_3x3():
    g = json.load(open(os.path.join(GOLDEN, "advect_3x3.json")))
    phi = np.array(g["phi"], dtype=np.float64)
    omega = np.array(g["omega"], dtype=np.float64)
    u = np.array(g["u"], dtype=np.float64)
    pt, wt = O.advect(phi, omega, u)
    assert np.max(np.abs(pt - np.array(g["phi_advected"]))) < 1e-14
    assert np.max(np.abs(wt - np.array(g["omega_advected"]))) < 1e-14
    assert np.allclose(pt.sum(axis=(1, 2)), phi.sum(axis=(1, 2)), rtol=0, atol=1e-14)
