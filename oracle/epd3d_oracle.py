"""Plain FP64 CPU oracle of the chain propagators and densities on a
three-dimensional grid.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  The GPU library shares no code with
it.

Source: Heuser, Sevink, Schmid, arXiv:1804.02883.  The paper computes in two
dimensions and states that the method is not restricted to them (end of
Sec. II).  The propagators and densities here are those of Sec. II (the split
step, the density integrals and Eq. phi_s), read as in the two-dimensional
oracle (readings R4-R7, R14 of epdlb_oracle.READINGS), on a periodic
nx x ny x nz grid with volume element dV = dx^3 and V = nx ny nz dV:

R29  In three dimensions the heat kernel of the split step is
     exp(-R_G^2 |k|^2 ds) with |k|^2 = kx^2 + ky^2 + kz^2, and every
     normalisation carries dV and V in place of dA and the area.  Arrays are
     [z][y][x], x fastest.
"""
import numpy as np

from oracle.epdlb_oracle import node_weights, segment_fractions, wavenumbers


def heat_multiplier3(shape, p):
    """exp(-R_G^2 |k|^2 ds) on the grid of shape (nz, ny, nx), FFT storage order."""
    nz, ny, nx = shape
    ds = 1.0 / p["n_contour"]
    kx = wavenumbers(nx, p["dx"])
    ky = wavenumbers(ny, p["dx"])
    kz = wavenumbers(nz, p["dx"])
    k2 = kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2
    return np.exp(-p["R_G"] ** 2 * k2 * ds)


def apply_heat_kernel3(g, p):
    """exp(R_G^2 Laplacian ds) g in Fourier space."""
    return np.fft.ifftn(heat_multiplier3(g.shape, p) * np.fft.fftn(g)).real


def propagate3(wA, wB, p, gauge):
    """Forward and backward chain propagators on nodes 0..N, shape (N+1, nz, ny, nx):
    q_{j+1} = E_j K (E_j q_j), E_j = exp(-(w_j - c_j)/2) with the segment field
    w_j = a_j wA + (1 - a_j) wB (Sec. II split step; q_0 = 1; the backward
    chain takes the segments in reverse order)."""
    N = p["n_contour"]
    cA, cB = gauge
    a = segment_fractions(N, p["f_A"])
    mult = heat_multiplier3(wA.shape, p)
    E = [np.exp(-(a[j] * (wA - cA) + (1.0 - a[j]) * (wB - cB)) / 2.0) for j in range(N)]
    q = np.empty((N + 1,) + wA.shape)
    qb = np.empty((N + 1,) + wA.shape)
    q[0] = 1.0
    qb[0] = 1.0
    for j in range(N):
        q[j + 1] = E[j] * np.fft.ifftn(mult * np.fft.fftn(E[j] * q[j])).real
        e = E[N - 1 - j]
        qb[j + 1] = e * np.fft.ifftn(mult * np.fft.fftn(e * qb[j])).real
    return q, qb


def densities3(omega, p, gauge=None):
    """Phi_A, Phi_B (the density integrals of Sec. II), Phi_S (Eq. phi_s), Q_P
    and Q_S on the grid of omega (3, nz, ny, nx); gauge (cA, cB, cS) defaults
    to the site means."""
    wA, wB, wS = omega
    N = p["n_contour"]
    if gauge is None:
        gauge = tuple(float(np.mean(w)) for w in omega)
    cA, cB, cS = gauge
    q, qb = propagate3(wA, wB, p, (cA, cB))
    dV = p["dx"] ** 3
    V = wA.size * dV
    QP = dV * float(np.sum(q[N]))
    wAn, wBn = node_weights(N, p["f_A"])
    sA = np.zeros_like(wA)
    sB = np.zeros_like(wA)
    for j in range(N + 1):
        prod = q[j] * qb[N - j]
        sA += wAn[j] * prod
        sB += wBn[j] * prod
    eS = np.exp(-(wS - cS))
    QS = dV * float(np.sum(eS))
    phiP = p["phi_P"]
    phi = np.stack([V * phiP / QP * sA, V * phiP / QP * sB, V * (1.0 - phiP) * eS / QS])
    return dict(phi=phi, Q_P=QP, Q_P_bwd=dV * float(np.sum(qb[N])), Q_S=QS, gauge=(cA, cB, cS))
