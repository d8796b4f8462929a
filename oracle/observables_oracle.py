"""Plain FP64 CPU oracle for the paper's observables of a density state.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  The GPU library shares no code with
it.

Source: Heuser, Sevink, Schmid, arXiv:1804.02883.  Each function names the
equation it follows.  Readings where the paper is silent (labels continue the
list of epdlb_oracle.READINGS):

R18  Particles are the connected clusters of sites with Phi_P >= threshold
     under nearest-neighbour (4-) connectivity on the periodic grid; the
     comparison is made in the precision the densities are stored in.
R19  Positions in the gyration tensor: each site of a particle is placed at
     its minimum-image offset from the particle's lowest site index (the
     particle's label).  A particle whose offsets reach half the box in x or
     y is flagged as wrapping; its tensor is then not meaningful.
R20  Y_2^P: y is measured from the box centre at cell centres, y = j + 1/2 -
     L_y/2, and the integrals are the sums over rows of the x-averaged Phi_P.
R24  Nucleation events (Sec. IV, nucleation stage): sampled every few steps,
     a particle of the current sample none of whose sites was a particle
     site (Phi_P >= threshold) at the previous sample is a new nucleus; its
     time is the sample's and its position the centroid.  At the first sample
     every particle counts.  The sampling interval must be short against the
     time a particle takes to move by its own size, or a moving particle is
     counted again.  The particle density n_p is the particle count over the
     system size V = nx ny dx^2.
"""
from collections import deque

import numpy as np


def sigma(phi, phibar_P):
    """Eq. for sigma(t) (Sec. III): (1/V) int |Phi_P - phibar_P|, Phi_P = Phi_A + Phi_B."""
    phiP = np.asarray(phi[0], dtype=np.float64) + np.asarray(phi[1], dtype=np.float64)
    return float(np.mean(np.abs(phiP - phibar_P)))


def sigma_delta(phiP_a, phiP_b):
    """Eq. for sigma_Delta (Sec. III): (1/V) int |Phi_P^LB - Phi_P^NLB|."""
    return float(np.mean(np.abs(np.asarray(phiP_a, dtype=np.float64) - np.asarray(phiP_b, dtype=np.float64))))


def y2p(phiP, phibar_P):
    """Eq. width (Sec. IV): sqrt(int y^2 Phi_P(y) dy / (phibar_P int y^2 dy)) with the
    x-averaged profile Phi_P(y) (reading R20)."""
    phiP = np.asarray(phiP, dtype=np.float64)
    ny = phiP.shape[0]
    y = np.arange(ny) + 0.5 - ny / 2.0
    prof = phiP.mean(axis=1)
    return float(np.sqrt(np.sum(y * y * prof) / (phibar_P * np.sum(y * y))))


def label_particles(phiP, threshold=0.5):
    """Connected clusters of sites with phiP >= threshold, 4-connectivity, periodic
    (reading R18), by breadth-first search.  Returns an int64 array of labels:
    -1 off the particles, else the lowest flat site index (y * nx + x) of the
    site's particle."""
    ny, nx = phiP.shape
    fg = phiP >= threshold
    lab = np.full((ny, nx), -1, dtype=np.int64)
    for start in range(nx * ny):
        y0, x0 = divmod(start, nx)
        if not fg[y0, x0] or lab[y0, x0] >= 0:
            continue
        # start is the lowest index of its cluster: all lower foreground sites
        # already belong to labelled clusters
        lab[y0, x0] = start
        q = deque([(y0, x0)])
        while q:
            y, x = q.popleft()
            for dy, dx in ((0, 1), (0, -1), (1, 0), (-1, 0)):
                yy, xx = (y + dy) % ny, (x + dx) % nx
                if fg[yy, xx] and lab[yy, xx] < 0:
                    lab[yy, xx] = start
                    q.append((yy, xx))
    return lab


def particle_table(phiP, threshold=0.5):
    """Per particle, in increasing label order: dict(label, area, content N,
    centroid (x, y) in the box, G (Gxx, Gxy, Gyy), R, c_rel, wraps).

    G follows Eq. gyration_tensor as written, the double sum
    G_nm = (1/(2 N^2)) sum_i sum_j Phi_i Phi_j (r_n^i - r_n^j)(r_m^i - r_m^j)
    over the particle's sites, with positions per reading R19; c = lambda_+ -
    lambda_-, R = sqrt(lambda_+ + lambda_-) (Eq. asph), c_rel = c^2/R^4
    (Eq. rel_asph)."""
    phiP = np.asarray(phiP, dtype=np.float64)
    ny, nx = phiP.shape
    lab = label_particles(phiP, threshold)
    out = []
    for L in np.unique(lab[lab >= 0]):
        ys, xs = np.nonzero(lab == L)
        w = phiP[ys, xs]
        ly, lx = divmod(int(L), nx)
        dx = (xs - lx + nx // 2) % nx - nx // 2
        dy = (ys - ly + ny // 2) % ny - ny // 2
        wraps = bool(np.any(np.abs(dx) >= nx // 2) or np.any(np.abs(dy) >= ny // 2))
        N = float(w.sum())
        r = np.stack([dx, dy]).astype(np.float64)
        G = np.zeros((2, 2))
        for a in range(2):
            for b in range(2):
                d_a = r[a][:, None] - r[a][None, :]
                d_b = r[b][:, None] - r[b][None, :]
                G[a, b] = np.sum(w[:, None] * w[None, :] * d_a * d_b) / (2.0 * N * N)
        lam = np.linalg.eigvalsh(G)
        c = lam[1] - lam[0]
        R = np.sqrt(lam[0] + lam[1])
        c_rel = c * c / R ** 4 if R > 0 else 0.0
        cx = (lx + np.sum(w * dx) / N) % nx
        cy = (ly + np.sum(w * dy) / N) % ny
        out.append(dict(label=int(L), area=int(len(xs)), content=N, centroid=(float(cx), float(cy)),
                        G=(float(G[0, 0]), float(G[0, 1]), float(G[1, 1])), R=float(R), c_rel=float(c_rel),
                        wraps=wraps))
    return out


def nucleation_events(phiP_prev, phiP, threshold=0.5):
    """Particles of phiP that are new since the sample phiP_prev (reading R24),
    as particle_table entries in label order; phiP_prev None: every particle."""
    table = particle_table(phiP, threshold)
    if phiP_prev is None:
        return table
    was = np.asarray(phiP_prev, dtype=np.float64) >= threshold
    lab = label_particles(phiP, threshold)
    return [t for t in table if not np.any(was[lab == t["label"]])]


def particle_density(n_particles, nx, ny, dx):
    """n_p (Sec. IV, nucleation stage): particles per unit area of the system (reading R24)."""
    return n_particles / (nx * ny * dx * dx)
