"""Pins of the three-dimensional propagator and density oracle (reading R29 in
oracle/epd3d_oracle.py), against what fixes it from outside:

* a field uniform along z gives, in every z-plane, the pinned two-dimensional
  oracle's densities;
* the densities commute with a rotation of the axes;
* uniform fields give the closed forms Phi_A = f_A phibar_P,
  Phi_B = (1 - f_A) phibar_P, Phi_S = 1 - phibar_P;
* cos(k z) is an eigenfunction of the heat kernel with eigenvalue
  exp(-R_G^2 k^2 ds);
* Phi_A = -(V phibar_P / (N dV)) d ln Q_P / d omega_A at a site (central
  differences), and the forward and backward chains give the same Q_P.
"""
import numpy as np
import pytest

from oracle import epd3d_oracle as E3
from oracle import epdlb_oracle as O
from seeded_inputs import preset


def _p(**kw):
    return preset("cfg1", **kw)


def _omega(shape, seed, sigma=0.1):
    return sigma * np.random.default_rng(seed).standard_normal((3,) + shape)


def test_uniform_along_z_equals_two_dimensional_oracle():
    p = _p(nx=16, ny=8, n_contour=8, f_A=0.3)
    w2 = _omega((8, 16), 1)
    w3 = np.repeat(w2[:, None], 4, axis=1)
    d3 = E3.densities3(w3, p)
    d2 = O.densities(w2, p)
    for z in range(4):
        assert np.max(np.abs(d3["phi"][:, z] - d2["phi"])) < 1e-13
    assert abs(d3["Q_P"] / (d2["Q_P"] * 4 * p["dx"]) - 1) < 1e-12


def test_rotation_of_the_axes():
    p = _p(n_contour=6, f_A=0.5)
    w = _omega((4, 6, 8), 2)
    rot = lambda A: np.transpose(A, (1, 2, 0))  # noqa: E731
    d = E3.densities3(w, p)["phi"]
    dr = E3.densities3(np.stack([rot(x) for x in w]), p)["phi"]
    for I in range(3):
        assert np.max(np.abs(dr[I] - rot(d[I]))) < 1e-13


@pytest.mark.parametrize("fA", [0.3, 0.5, 0.82])
def test_uniform_fields_closed_form(fA):
    p = _p(n_contour=10, f_A=fA, phi_P=0.15)
    w = np.stack([np.full((4, 4, 8), 0.3), np.full((4, 4, 8), -0.2), np.full((4, 4, 8), 0.7)])
    phi = E3.densities3(w, p)["phi"]
    assert np.max(np.abs(phi[0] - fA * 0.15)) < 1e-14
    assert np.max(np.abs(phi[1] - (1 - fA) * 0.15)) < 1e-14
    assert np.max(np.abs(phi[2] - 0.85)) < 1e-14


def test_plane_wave_along_z_is_an_eigenfunction():
    p = _p(n_contour=16)
    nz = 16
    z = np.arange(nz)
    for m in (1, 3):
        k = 2 * np.pi * m / (nz * p["dx"])
        g = np.broadcast_to(np.cos(k * z * p["dx"])[:, None, None], (nz, 2, 4)).copy()
        out = E3.apply_heat_kernel3(g, p)
        lam = np.exp(-p["R_G"] ** 2 * k * k / p["n_contour"])
        assert np.max(np.abs(out - lam * g)) < 1e-14


def test_density_is_derivative_of_log_partition_function():
    p = _p(n_contour=8, f_A=0.4)
    w = _omega((4, 4, 8), 3, 0.05)
    g = tuple(float(np.mean(x)) for x in w)
    d = E3.densities3(w, p, g)
    assert abs(d["Q_P_bwd"] / d["Q_P"] - 1) < 1e-12
    V = w[0].size * p["dx"] ** 3
    h = 1e-5
    for (z, y, x) in [(0, 1, 2), (3, 3, 7)]:
        wp, wm = w.copy(), w.copy()
        wp[0, z, y, x] += h
        wm[0, z, y, x] -= h
        dl = (np.log(E3.densities3(wp, p, g)["Q_P"]) - np.log(E3.densities3(wm, p, g)["Q_P"])) / (2 * h)
        fd = -V * p["phi_P"] / (p["n_contour"] * p["dx"] ** 3) * dl
        assert abs(fd - d["phi"][0, z, y, x]) < 1e-7 * abs(d["phi"][0, z, y, x]) + 1e-12
