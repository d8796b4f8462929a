"""Plain FP64 CPU oracle of the three-dimensional lattice Boltzmann fluid.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  The GPU library shares no code with
it.

Source: Heuser, Sevink, Schmid, arXiv:1804.02883.  The paper runs its method
in two dimensions with D2Q9 and names D3Q19 as the scheme that replaces it in
three dimensions (end of Sec. II, before Sec. III).  The collision and the
body force are those of the two-dimensional fluid (Sec. II, Eq. LB_prop and
Eq. force_col) at gamma_s = gamma_b = 0, written for 19 velocities.

Readings (labels continue the list of epdlb_oracle.READINGS):

R26  D3Q19 velocity set and weights as in Qian, d'Humieres and Lallemand
     (1992): the rest velocity (weight 1/3), the six axis velocities (1/18)
     and the twelve face diagonals (1/36); c_s^2 = 1/3.  Populations are
     indexed 0 rest, 1-6 (+x, -x, +y, -y, +z, -z), 7-18 the diagonals in the
     order of C19 below.  Arrays are [i][z][y][x] with x fastest; vectors
     (force, velocity) are planes (x, y, z).
R27  The step is the two-dimensional one (reading R12) in three dimensions:
     pull streaming f_i(x) = f*_i(x - c_i) on the periodic box, moments
     rho = sum f_i and u = (sum f_i c_i + F/2) / rho, BGK collision towards
     the second-order equilibrium with relaxation time tau, plus the
     second-order force term (1 - 1/(2 tau)) w_i [3 (c_i - u).F + 9 (c_i.u)(c_i.F)].
     Kinematic viscosity nu = (tau - 1/2)/3 in lattice units.
R28  The multi-relaxation collision (the paper's, Sec. II, Eq. force_col) in
     three dimensions, as the two-dimensional one (reading R17) with the trace
     split of d = 3, where the printed 2/3 and 1/3 apply as printed: the
     non-equilibrium stress keeps gamma_s of its traceless part and gamma_b of
     its trace tr/3 I; the forcing stress is
     Sigma = (1 + gamma_s)/2 [u F + F u - (2/3)(u.F) I] + (1 + gamma_b)/3 (u.F) I;
     the nine non-hydrodynamic modes are scaled by gamma_g.  Shear viscosity
     nu = (c_s^2/2)(1 + gamma_s)/(1 - gamma_s), bulk viscosity
     nu_B = (c_s^2/3)(1 + gamma_b)/(1 - gamma_b) (the paper's relations with d = 3,
     rho = 1, lattice units).
"""
import numpy as np

C19 = np.array([[0, 0, 0],
                [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
                [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0],
                [1, 0, 1], [-1, 0, -1], [1, 0, -1], [-1, 0, 1],
                [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]], dtype=np.int64)
W19 = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12, dtype=np.float64)
CS2 = 1.0 / 3.0


def viscosity(tau):
    """nu = c_s^2 (tau - 1/2) (reading R27)."""
    return CS2 * (tau - 0.5)


def equilibrium(rho, u):
    """Second-order equilibrium f^eq_i = w_i rho (1 + 3 c.u + 4.5 (c.u)^2 - 1.5 u^2),
    shape (19,) + rho.shape; u has shape (3,) + rho.shape."""
    usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2]
    feq = np.empty((19,) + np.shape(rho))
    for i in range(19):
        cu = C19[i, 0] * u[0] + C19[i, 1] * u[1] + C19[i, 2] * u[2]
        feq[i] = W19[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq)
    return feq


def stream(fstar):
    """Pull streaming f_i(x) = f*_i(x - c_i) on the periodic box (axes z, y, x)."""
    f = np.empty_like(fstar)
    for i in range(19):
        f[i] = np.roll(fstar[i], shift=(C19[i, 2], C19[i, 1], C19[i, 0]), axis=(0, 1, 2))
    return f


def moments(f):
    """rho = sum f_i, j = sum f_i c_i (shapes (nz, ny, nx) and (3, nz, ny, nx))."""
    rho = f.sum(axis=0)
    j = np.stack([sum(C19[i, a] * f[i] for i in range(19)) for a in range(3)])
    return rho, j


def collide(f, F, tau):
    """BGK collision with the second-order force term (reading R27) of streamed
    populations f; returns (f*, rho, u)."""
    rho, j = moments(f)
    u = (j + 0.5 * F) / rho
    feq = equilibrium(rho, u)
    out = np.empty_like(f)
    for i in range(19):
        c = C19[i]
        cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2]
        cF = c[0] * F[0] + c[1] * F[1] + c[2] * F[2]
        cmuF = (c[0] - u[0]) * F[0] + (c[1] - u[1]) * F[1] + (c[2] - u[2]) * F[2]
        src = W19[i] * (3.0 * cmuF + 9.0 * cu * cF)
        out[i] = f[i] - (f[i] - feq[i]) / tau + (1.0 - 0.5 / tau) * src
    return out, rho, u


def step(fstar, F, tau):
    """One step (Eq. LB_prop with the force of Eq. force_col, reading R27):
    stream, then collide.  Returns (f*_new, rho, u)."""
    return collide(stream(fstar), F, tau)


def site(fstar, F, tau, z, y, x, mrt=None):
    """The step at one site, from the pre-streaming populations: the 19
    post-collision values and (rho, u) there.  Gathers the neighbours by index
    (not by rolling whole planes), for sampled checks of large lattices.
    mrt = (gamma_s, gamma_b, gamma_g) selects the multi-relaxation collision."""
    nz, ny, nx = fstar.shape[1:]
    f = np.array([fstar[i, (z - C19[i, 2]) % nz, (y - C19[i, 1]) % ny, (x - C19[i, 0]) % nx]
                  for i in range(19)], dtype=np.float64).reshape(19, 1, 1, 1)
    Fs = np.array([F[a, z, y, x] for a in range(3)], dtype=np.float64).reshape(3, 1, 1, 1)
    if mrt is None:
        out, rho, u = collide(f, Fs, tau)
    else:
        out, rho, u = collide_mrt(f, Fs, *mrt)
    return out[:, 0, 0, 0], float(rho[0, 0, 0]), u[:, 0, 0, 0]


def stress_moments(f):
    """rho, j and Pi = sum f_i c_i c_i (shapes (...), (3, ...), (3, 3, ...))."""
    c = C19.astype(np.float64)
    rho = f.sum(axis=0)
    j = np.einsum("ia,i...->a...", c, f)
    Pi = np.einsum("ia,ib,i...->ab...", c, c, f)
    return rho, j, Pi


def hermite(rho, j, Pi):
    """Populations carrying the moments (rho, j, Pi) and nothing else:
    n_i = w_i [rho + j.c_i/c_s^2 + (Pi - rho c_s^2 I):(c_i c_i - c_s^2 I)/(2 c_s^4)]."""
    out = np.empty((19,) + np.shape(rho))
    for i in range(19):
        c = C19[i].astype(np.float64)
        h = 0.0
        for a in range(3):
            for b in range(3):
                h = h + (Pi[a, b] - (rho * CS2 if a == b else 0.0)) * (c[a] * c[b] - (CS2 if a == b else 0.0))
        out[i] = W19[i] * (rho + (j[0] * c[0] + j[1] * c[1] + j[2] * c[2]) / CS2 + h / (2.0 * CS2 * CS2))
    return out


def collide_mrt(f, F, gamma_s, gamma_b, gamma_g):
    """Multi-relaxation collision with the force term of Eq. force_col in three
    dimensions (reading R28).  u = (j + F/2)/rho; Pi_eq = rho c_s^2 I + rho u u;
    the non-equilibrium stress keeps gamma_s of its traceless part and gamma_b
    of its trace; post-collision moments (rho, j + F, Pi_eq + relaxed + Sigma);
    the remainder f - hermite(moments of f) is scaled by gamma_g.
    Returns (f*, rho, u)."""
    rho, j, Pi = stress_moments(f)
    u = (j + 0.5 * F) / rho
    eye = np.eye(3).reshape((3, 3) + (1,) * np.ndim(rho))
    Pi_eq = rho * CS2 * eye + rho * np.einsum("a...,b...->ab...", u, u)
    neq = Pi - Pi_eq
    tr = neq[0, 0] + neq[1, 1] + neq[2, 2]
    relaxed = gamma_s * (neq - tr / 3.0 * eye) + gamma_b * tr / 3.0 * eye
    uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2]
    sym = np.einsum("a...,b...->ab...", u, F) + np.einsum("a...,b...->ab...", F, u)
    Sigma = 0.5 * (1.0 + gamma_s) * (sym - (2.0 / 3.0) * uF * eye) + (1.0 + gamma_b) / 3.0 * uF * eye
    post = hermite(rho, j + F, Pi_eq + relaxed + Sigma)
    ghost = f - hermite(rho, j, Pi)
    return post + gamma_g * ghost, rho, u


def step_mrt(fstar, F, gamma_s, gamma_b, gamma_g):
    """Stream, then the multi-relaxation collision.  Returns (f*, rho, u)."""
    return collide_mrt(stream(fstar), F, gamma_s, gamma_b, gamma_g)


def mrt_viscosities(gamma_s, gamma_b):
    """(nu, nu_B) of reading R28."""
    return (0.5 * CS2 * (1.0 + gamma_s) / (1.0 - gamma_s),
            CS2 / 3.0 * (1.0 + gamma_b) / (1.0 - gamma_b))
