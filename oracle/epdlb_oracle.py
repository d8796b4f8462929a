"""Plain, slow, FP64 CPU oracle for the hybrid LB/EPD time step.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  The GPU library shares no code with
it; both consume the seeded inputs in `seeded_inputs`.

Source: Heuser, Sevink, Schmid, "Self-assembly of polymeric particles in
Poiseuille flow: a hybrid Lattice Boltzmann / External Potential Dynamics
simulation study" (arXiv:1804.02883).  Each function names the passage it
follows.  Where the paper is silent, the reading taken is stated in the
function's docstring (readings R1-R14, listed together in `READINGS`).

Grid: nx x ny sites, arrays indexed [y, x]; site (x, y) is the cell centre
((x + 1/2) dx, (y + 1/2) dx); periodic in both directions.

Every function here has a pin in tests/test_oracle_*.py except the ones named
in PARITY_UNPINNED (none): the chemical potential and the field update are
pinned to the free energy of Sec. II and to closed-form single-mode updates,
the advection to a hand-computed case (tests/test_oracle_epd_update.py).
"""
import numpy as np

READINGS = {
    "R1": "One propagator evaluation per step; omega after convection comes from the "
          "auxiliary omega-convection (App. C comment 1) instead of a Phi->omega CG solve "
          "(cg_invert = 0, the default; cg_invert = 1 runs the solve, readings R21-R23).",
    "R2": "Step order: advection -> mu at the advected composition -> omega update -> "
          "densities -> force from the diffusive change -> LB; advection uses the "
          "previous LB velocity.",
    "R3": "Diffusive composition change = Phi(omega^{n+1}) - advected Phi.",
    "R4": "Backward propagator g' starts at the B end: field omega(r, 1 - s).",
    "R5": "g(r, 0) = g'(r, 0) = 1.",
    "R6": "Segment-constant field with a fractional junction segment a_j = clip(f_A N - j, 0, 1).",
    "R7": "Contour integrals by trapezoid-consistent node weights w_A, w_B.",
    "R8": "N = number of chain segments; ds = 1/N; the same N multiplies omega.",
    "R9": "kT/v = 1 in rho R_G^2 tau^-2 (the paper leaves 1/(beta v) unspecified).",
    "R10": "Donor-cell (upwind) advection: flux form for Phi, upwind form for omega; "
           "5-point Laplacian for the omega update.",
    "R11": "Force in k-space with continuous k; zero at k = 0 and on the Nyquist line of "
           "each odd derivative.",
    "R12": "LB at gamma_s = gamma_b = 0 (BGK, tau = 1) with second-order forcing "
           "(Guo form, which equals the Duenweg force term there); u includes F/2.",
    "R13": "Lattice force F = f dt^2/dx with rho_0 = 1; g in units f* = rho R_G tau^-2.",
    "R14": "Gauge: omega_I shifted by constants c_I inside the propagator "
           "(densities are invariant under such shifts).",
    "R17": "Multi-relaxation LB (lb_mrt = 1): collision in moment space; the traceless "
           "non-equilibrium stress is scaled by gamma_s, its trace by gamma_b, the three "
           "non-hydrodynamic modes by gamma_g (not stated in the paper; default 0). The "
           "forcing stress Sigma of Eq. force_col uses the trace split of d = 2 "
           "(the printed 2/3 and 1/3 are the d = 3 values; the bulk-viscosity relation of "
           "the same passage carries d). u includes F/2; the momentum gains F.",
    "R21": "Phi->omega inversion (App. C comments 2 and 3): Fletcher-Reeves conjugate "
           "gradients on G(omega) = (V phibar_P/N) ln Q_P + V phibar_S ln Q_S + dA sum_I "
           "sum_r omega_I Phi~_I, whose gradient is dA (Phi~ - Phi[omega]) exactly for the "
           "trapezoid contour weights (the paper names the method, not the functional).",
    "R22": "Line search: one secant step on the directional derivative from a trial point "
           "at the previous step length (1 at the first iteration); a direction that is no "
           "descent direction is replaced by the steepest descent; when the curvature along "
           "the direction is not positive the trial step is taken.",
    "R23": "Stopping: sqrt(sum_I sum_r (Phi~_I - Phi_I[omega])^2 / (nx ny)) < N_tr (1e-8), the "
           "three fields together; start from the auxiliary-convected omega (comment 1); "
           "after cg_max_iter iterations the last iterate is used unconverged.",
    "R25": "Optional diagonal preconditioning of the inversion (cg_precond = 1; the paper's "
           "iteration is plain): directions from s divided by the local response "
           "(N Phi_A, N Phi_B, Phi_S) at the current iterate; same fixed point and stopping test.",
}

PARITY_UNPINNED = ()

# D2Q9 velocity set and weights (lattice Boltzmann model statement, Sec. II).
C9 = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1],
               [1, 1], [-1, 1], [-1, -1], [1, -1]], dtype=np.int64)
W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, dtype=np.float64)
CS2 = 1.0 / 3.0


# --------------------------------------------------------------------------
# Chain statistics: modified diffusion equation, split step, densities
# (Sec. II, Eqs. mod_diff1/mod_diff2, the Tzeremes split step, Eq. phi_s)
# --------------------------------------------------------------------------

def segment_fractions(N, f_A):
    """A-content a_j of contour segment j = 0..N-1 (reading R6).

    Segment j covers s in [j/N, (j+1)/N]; the field omega(r, s) is omega_A for
    s < f_A and omega_B otherwise (Sec. II), so a_j is the A-covered share of
    the segment.
    """
    j = np.arange(N, dtype=np.float64)
    return np.clip(f_A * N - j, 0.0, 1.0)


def node_weights(N, f_A):
    """Contour weights for int ds over the A and B parts at nodes 0..N (reading R7)."""
    a = segment_fractions(N, f_A)
    ds = 1.0 / N
    wA = np.zeros(N + 1)
    wB = np.zeros(N + 1)
    for j in range(N + 1):
        if j >= 1:
            wA[j] += 0.5 * ds * a[j - 1]
            wB[j] += 0.5 * ds * (1.0 - a[j - 1])
        if j <= N - 1:
            wA[j] += 0.5 * ds * a[j]
            wB[j] += 0.5 * ds * (1.0 - a[j])
    return wA, wB


def wavenumbers(n, dx):
    """k_m = 2 pi m / (n dx), m in [-n/2, n/2), in FFT storage order."""
    return 2.0 * np.pi * np.fft.fftfreq(n, d=dx)


def heat_multiplier(p):
    """Fourier multiplier of exp(R_G^2 Laplacian ds) on the grid (Sec. II split step)."""
    ds = 1.0 / p["n_contour"]
    kx = wavenumbers(p["nx"], p["dx"])
    ky = wavenumbers(p["ny"], p["dx"])
    k2 = ky[:, None] ** 2 + kx[None, :] ** 2
    return np.exp(-p["R_G"] ** 2 * k2 * ds)


def apply_heat_kernel(g, p):
    """exp(R_G^2 Laplacian ds) g, evaluated in Fourier space (Sec. II)."""
    return np.fft.ifft2(heat_multiplier(p) * np.fft.fft2(g)).real


def field_means(omega):
    """FP64 site averages of each field plane."""
    return np.array([float(np.mean(w)) for w in omega])


def propagate(wA, wB, p, gauge=None):
    """Forward and backward chain propagators on nodes 0..N.

    Split step (Sec. II, Tzeremes scheme), with the segment field of reading R6:
        q_{j+1} = E_j  K  (E_j q_j),   E_j = exp(-N ds (w_j - c_j) / 2),
        w_j = a_j wA + (1 - a_j) wB,   c_j = a_j cA + (1 - a_j) cB,
    K = exp(R_G^2 Laplacian ds).  q_0 = 1 (reading R5).  The backward chain
    q' uses the segments in reverse order (reading R4).  `gauge` = (cA, cB)
    (reading R14); default: the site means of wA and wB.
    Returns arrays of shape (N+1, ny, nx).
    """
    N = p["n_contour"]
    ds = 1.0 / N
    if gauge is None:
        gauge = (float(np.mean(wA)), float(np.mean(wB)))
    cA, cB = gauge
    a = segment_fractions(N, p["f_A"])
    mult = heat_multiplier(p)
    E = []
    for j in range(N):
        wj = a[j] * (wA - cA) + (1.0 - a[j]) * (wB - cB)
        E.append(np.exp(-N * ds * wj / 2.0))
    shape = wA.shape
    q = np.empty((N + 1,) + shape)
    qb = np.empty((N + 1,) + shape)
    q[0] = 1.0
    qb[0] = 1.0
    for j in range(N):
        q[j + 1] = E[j] * np.fft.ifft2(mult * np.fft.fft2(E[j] * q[j])).real
        e = E[N - 1 - j]
        qb[j + 1] = e * np.fft.ifft2(mult * np.fft.fft2(e * qb[j])).real
    return q, qb


def densities(omega, p, gauge=None):
    """Composition fields from the potentials (Sec. II, the density integrals and Eq. phi_s).

    Phi_A = (V phibar_P / Q_P) sum_j w_A(j) q_j q'_{N-j}, likewise Phi_B;
    Q_P = dA sum_r q_N; Phi_S = V phibar_S exp(-(w_S - c_S)) / Q_S with
    Q_S = dA sum_r exp(-(w_S - c_S)).  `gauge` = (cA, cB, cS), default the
    site means (reading R14).  Returns a dict with phi (3, ny, nx), Q_P,
    Q_P_bwd (from the backward chain), Q_S and the gauge used.
    """
    wA, wB, wS = omega
    N = p["n_contour"]
    if gauge is None:
        gauge = tuple(field_means(omega))
    cA, cB, cS = gauge
    q, qb = propagate(wA, wB, p, (cA, cB))
    dA = p["dx"] ** 2
    V = p["nx"] * p["ny"] * dA
    QP = dA * float(np.sum(q[N]))
    QPb = dA * float(np.sum(qb[N]))
    wAn, wBn = node_weights(N, p["f_A"])
    sA = np.zeros_like(wA)
    sB = np.zeros_like(wA)
    for j in range(N + 1):
        prod = q[j] * qb[N - j]
        sA += wAn[j] * prod
        sB += wBn[j] * prod
    phiP = p["phi_P"]
    phiS_bar = 1.0 - phiP
    eS = np.exp(-(wS - cS))
    QS = dA * float(np.sum(eS))
    phi = np.stack([V * phiP / QP * sA, V * phiP / QP * sB, V * phiS_bar * eS / QS])
    return dict(phi=phi, Q_P=QP, Q_P_bwd=QPb, Q_S=QS, gauge=(cA, cB, cS))


# --------------------------------------------------------------------------
# Convection and EPD diffusion (Eq. conv_diff, Eq. diff_w, App. C comments 1 and 4)
# --------------------------------------------------------------------------

def advect(phi, omega, u):
    """One Euler-forward convection step in lattice units (reading R10).

    Phi (conservative flux form): face velocity u_{x+1/2} = (u(x) + u(x+1))/2,
    flux J_{x+1/2} = u_{x+1/2} Phi(upwind cell), upwind = x if u_{x+1/2} >= 0
    else x+1; Phi~ = Phi - (J_{x+1/2} - J_{x-1/2}) - (same in y).
    omega (auxiliary convection step of App. C, comment 1): upwind
    omega~ = omega - [u+ (w - w_{x-1}) + u- (w_{x+1} - w)] - (same in y),
    with u+ = max(u, 0), u- = min(u, 0) at the cell centre.
    """
    ux, uy = u
    out_phi = phi.copy()
    out_w = omega.copy()
    for axis, uc in ((-1, ux), (-2, uy)):
        ax2 = axis + 2  # axis within a single (ny, nx) plane
        uf = 0.5 * (uc + np.roll(uc, -1, axis=ax2))
        for I in range(phi.shape[0]):
            f = phi[I]
            J = np.where(uf >= 0.0, uf * f, uf * np.roll(f, -1, axis=ax2))
            out_phi[I] -= J - np.roll(J, 1, axis=ax2)
        up = np.maximum(uc, 0.0)
        um = np.minimum(uc, 0.0)
        for I in range(omega.shape[0]):
            w = omega[I]
            out_w[I] -= up * (w - np.roll(w, 1, axis=ax2)) + um * (np.roll(w, -1, axis=ax2) - w)
    return out_phi, out_w


def chi_matrix(p):
    c = np.zeros((3, 3))
    c[0, 1] = c[1, 0] = p["chi_AB"]
    c[0, 2] = c[2, 0] = p["chi_AS"]
    c[1, 2] = c[2, 1] = p["chi_BS"]
    return c


def chemical_potential(phi, omega, p):
    """mu_I = dF/dPhi_I from Eq. free_energy: sum_{J!=I} chi_IJ Phi_J - w_I + kappa_H (sum Phi - 1)."""
    chi = chi_matrix(p)
    tot = phi.sum(axis=0)
    mu = np.empty_like(phi)
    for I in range(3):
        acc = np.zeros_like(tot)
        for J in range(3):
            if J != I:
                acc += chi[I, J] * phi[J]
        mu[I] = acc - omega[I] + p["kappa_H"] * (tot - 1.0)
    return mu


def laplacian5(f):
    """5-point periodic Laplacian in lattice units (reading R10)."""
    return (np.roll(f, 1, -1) + np.roll(f, -1, -1) + np.roll(f, 1, -2) + np.roll(f, -1, -2) - 4.0 * f)


def diffusivities(p):
    return np.array([p["D_A"], p["D_B"], p["D_S"]])


def field_update(phi_t, omega_t, p):
    """EPD diffusion step, Eq. diff_w: w^{n+1} = w~ - (D_I dt / dx^2) Lap mu~ (App. C comment 4)."""
    mu = chemical_potential(phi_t, omega_t, p)
    D = diffusivities(p)
    out = np.empty_like(omega_t)
    for I in range(3):
        out[I] = omega_t[I] - D[I] * p["dt"] / p["dx"] ** 2 * laplacian5(mu[I])
    return out


# --------------------------------------------------------------------------
# Force reconstruction (Sec. II, k-space force; App. A) and the external force (Eq. force_field_2)
# --------------------------------------------------------------------------

def polymer_force(S, p):
    """Physical force f = sum_I f_I from S = sum_I dPhi_I^D / D_I (readings R3, R9, R11).

    f^(k) = (kT/v) S^(k) i k / (dt |k|^2); f^(0) = 0; the x component is
    zeroed on the k_x Nyquist line and the y component on the k_y Nyquist line.
    Returns (2, ny, nx).
    """
    ny, nx = S.shape
    kx = wavenumbers(nx, p["dx"])
    ky = wavenumbers(ny, p["dx"])
    KX, KY = np.meshgrid(kx, ky)
    k2 = KX ** 2 + KY ** 2
    Sh = np.fft.fft2(S)
    inv = np.zeros_like(k2)
    nz = k2 > 0
    inv[nz] = 1.0 / k2[nz]
    pref = p["kT_over_v"] / p["dt"]
    fx_h = pref * Sh * 1j * KX * inv
    fy_h = pref * Sh * 1j * KY * inv
    fx_h[:, nx // 2] = 0.0
    fy_h[ny // 2, :] = 0.0
    return np.stack([np.fft.ifft2(fx_h).real, np.fft.ifft2(fy_h).real])


def external_force_x(p):
    """Reverse-Poiseuille driving, Eq. force_field_2: -g for y < L_y/2, +g otherwise (per row)."""
    ny = p["ny"]
    y = np.arange(ny)
    return np.where(y < ny // 2, -p["g"], p["g"])


def lattice_force(S, p):
    """Body force in lattice units, F = (f + f_ext) dt^2/dx (reading R13), shape (2, ny, nx)."""
    ny, nx = p["ny"], p["nx"]
    conv = p["dt"] ** 2 / p["dx"]
    if p.get("couple_lb", 1):
        f = polymer_force(S, p) * conv
    else:
        f = np.zeros((2, ny, nx))
    fext = external_force_x(p)
    if p.get("g_units", 0) == 0:
        fext = fext * conv
    f[0] += fext[:, None]
    return f


# --------------------------------------------------------------------------
# D2Q9 lattice Boltzmann (Eq. LB_prop, Eq. force_col)
# --------------------------------------------------------------------------

def lb_equilibrium(rho, u):
    """Second-order D2Q9 equilibrium, shape (9, ny, nx)."""
    ux, uy = u
    usq = ux * ux + uy * uy
    feq = np.empty((9,) + rho.shape)
    for i in range(9):
        cu = C9[i, 0] * ux + C9[i, 1] * uy
        feq[i] = W9[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq)
    return feq


def lb_stream(fstar):
    """Streaming of Eq. LB_prop as a pull: f_i(x) = f*_i(x - c_i), periodic."""
    f = np.empty_like(fstar)
    for i in range(9):
        f[i] = np.roll(fstar[i], shift=(C9[i, 1], C9[i, 0]), axis=(0, 1))
    return f


def lb_step(fstar, F, tau):
    """Stream then collide with body force (reading R12).

    Streaming of Eq. LB_prop as a pull: f_i(x) = f*_i(x - c_i).  Moments
    rho = sum f_i, u = (sum f_i c_i + F/2)/rho.  Collision:
    f*_i = f_i - (f_i - feq_i)/tau + (1 - 1/(2 tau)) w_i [3 (c_i - u).F + 9 (c_i.u)(c_i.F)].
    Returns (f*_new, rho, u).
    """
    f = lb_stream(fstar)
    rho = f.sum(axis=0)
    jx = sum(C9[i, 0] * f[i] for i in range(9))
    jy = sum(C9[i, 1] * f[i] for i in range(9))
    ux = (jx + 0.5 * F[0]) / rho
    uy = (jy + 0.5 * F[1]) / rho
    u = np.stack([ux, uy])
    feq = lb_equilibrium(rho, u)
    out = np.empty_like(f)
    for i in range(9):
        cu = C9[i, 0] * ux + C9[i, 1] * uy
        cF = C9[i, 0] * F[0] + C9[i, 1] * F[1]
        cmuF = (C9[i, 0] - ux) * F[0] + (C9[i, 1] - uy) * F[1]
        src = W9[i] * (3.0 * cmuF + 9.0 * cu * cF)
        out[i] = f[i] - (f[i] - feq[i]) / tau + (1.0 - 0.5 / tau) * src
    return out, rho, u


def lb_moments(f):
    """rho = sum f_i, j = sum f_i c_i, Pi = sum f_i c_i c_i (shapes (), (2,), (2, 2))."""
    c = C9.astype(np.float64)
    rho = f.sum(axis=0)
    j = np.einsum("ia,i...->a...", c, f)
    Pi = np.einsum("ia,ib,i...->ab...", c, c, f)
    return rho, j, Pi


def lb_hermite(rho, j, Pi):
    """Populations carrying the moments (rho, j, Pi) and nothing else: the
    second-order Hermite expansion in the D2Q9 weights,
    n_i = w_i [rho + j.c_i/c_s^2 + (Pi - rho c_s^2 I):(c_i c_i - c_s^2 I)/(2 c_s^4)]."""
    out = np.empty((9,) + np.shape(rho))
    for i in range(9):
        cx, cy = float(C9[i, 0]), float(C9[i, 1])
        h = ((Pi[0, 0] - rho * CS2) * (cx * cx - CS2) + (Pi[1, 1] - rho * CS2) * (cy * cy - CS2)
             + 2.0 * Pi[0, 1] * cx * cy)
        out[i] = W9[i] * (rho + (j[0] * cx + j[1] * cy) / CS2 + h / (2.0 * CS2 * CS2))
    return out


def lb_collide_mrt(f, F, gamma_s, gamma_b, gamma_g):
    """Multi-relaxation collision with the force term of Eq. force_col (reading R17).

    u = (j + F/2)/rho; Pi_eq = rho c_s^2 I + rho u u; the non-equilibrium stress
    Pi - Pi_eq keeps gamma_s of its traceless part and gamma_b of its trace;
    Sigma = (1 + gamma_s)/2 [u F + F u - (u.F) I] + (1 + gamma_b)/2 (u.F) I;
    post-collision moments (rho, j + F, Pi_eq + relaxed + Sigma); the
    non-hydrodynamic remainder f - hermite(moments of f) is scaled by gamma_g.
    Returns (f*, rho, u)."""
    rho, j, Pi = lb_moments(f)
    u = (j + 0.5 * F) / rho
    eye = np.eye(2)[:, :, None, None]
    uu = np.einsum("a...,b...->ab...", u, u)
    Pi_eq = rho * CS2 * eye + rho * uu
    neq = Pi - Pi_eq
    tr = neq[0, 0] + neq[1, 1]
    relaxed = gamma_s * (neq - 0.5 * tr * eye) + gamma_b * 0.5 * tr * eye
    uF = u[0] * F[0] + u[1] * F[1]
    sym = np.einsum("a...,b...->ab...", u, F) + np.einsum("a...,b...->ab...", F, u)
    Sigma = 0.5 * (1.0 + gamma_s) * (sym - uF * eye) + 0.5 * (1.0 + gamma_b) * uF * eye
    post = lb_hermite(rho, j + F, Pi_eq + relaxed + Sigma)
    ghost = f - lb_hermite(rho, j, Pi)
    return post + gamma_g * ghost, rho, u


def lb_step_mrt(fstar, F, gamma_s, gamma_b, gamma_g):
    """Stream (Eq. LB_prop) then the multi-relaxation collision.  Returns (f*, rho, u)."""
    return lb_collide_mrt(lb_stream(fstar), F, gamma_s, gamma_b, gamma_g)


def mrt_gammas(eta, eta_B, rho, dx, dt, d=2):
    """gamma_s, gamma_b from the viscosity relations of Sec. II:
    eta = (dt rho c_s^2/2)(1 + gamma_s)/(1 - gamma_s),
    eta_B = (dt rho c_s^2/d)(1 + gamma_b)/(1 - gamma_b), c_s^2 = dx^2/(3 dt^2)."""
    cs2 = dx * dx / (3.0 * dt * dt)
    a = 2.0 * eta / (dt * rho * cs2)
    b = d * eta_B / (dt * rho * cs2)
    return (a - 1.0) / (a + 1.0), (b - 1.0) / (b + 1.0)


def lb_viscosity(p):
    """Lattice kinematic shear viscosity of the configured collision (rho = 1):
    BGK (tau - 1/2)/3; multi-relaxation (c_s^2/2)(1 + gamma_s)/(1 - gamma_s)."""
    if p.get("lb_mrt", 0):
        gs = p["lb_gamma_s"]
        return 0.5 * CS2 * (1.0 + gs) / (1.0 - gs)
    return (p["lb_tau"] - 0.5) / 3.0


def lb_advance(fstar, F, p):
    """The configured LB step: BGK (lb_mrt = 0) or multi-relaxation (lb_mrt = 1)."""
    if p.get("lb_mrt", 0):
        return lb_step_mrt(fstar, F, p["lb_gamma_s"], p["lb_gamma_b"], p.get("lb_gamma_g", 0.0))
    return lb_step(fstar, F, p["lb_tau"])


def poiseuille_profile(ny, F0, tau, nu=None):
    """Eq. flow_field in lattice units at cell centres y + 1/2, rho = 1, with
    nu = (tau - 1/2)/3 unless the viscosity nu is given."""
    if nu is None:
        nu = (tau - 0.5) / 3.0
    Y = np.arange(ny) + 0.5
    Ly = float(ny)
    return -(F0 / (2.0 * nu)) * (Y - Ly / 2) * (np.abs(Y - Ly / 2) - Ly / 2)


def external_force_lattice_amplitude(p):
    return p["g"] * (p["dt"] ** 2 / p["dx"] if p.get("g_units", 0) == 0 else 1.0)


# --------------------------------------------------------------------------
# State, initialisation and the hybrid step (App. C)
# --------------------------------------------------------------------------

def init_state(p, omega0):
    """Initial state from the potentials omega0 (3, ny, nx).

    Phi^0 = Phi[omega0]; LB starts from f^eq(1, u_init) with u_init the
    analytic profile (Sec. IV: runs start from the flow of Eq. flow_field) when
    init_flow = 1, else at rest.
    """
    ny, nx = p["ny"], p["nx"]
    omega = np.array(omega0, dtype=np.float64, copy=True)
    d = densities(omega, p)
    u = np.zeros((2, ny, nx))
    if p.get("init_flow", 1):
        prof = poiseuille_profile(ny, external_force_lattice_amplitude(p), p["lb_tau"], nu=lb_viscosity(p))
        u[0] = prof[:, None]
    rho = np.ones((ny, nx))
    fstar = lb_equilibrium(rho, u)
    return dict(omega=omega, phi=d["phi"], fstar=fstar, u=u, rho=rho, n=0,
                Q_P=d["Q_P"], Q_S=d["Q_S"], S=np.zeros((ny, nx)), F=np.zeros((2, ny, nx)))


# --------------------------------------------------------------------------
# Phi -> omega inversion (App. C comments 1-3; readings R21-R23)
# --------------------------------------------------------------------------

def legendre_objective(omega, phi_target, p, gauge):
    """G(omega) of reading R21 at a fixed gauge (cA, cB, cS).

    G = (V phibar_P / N) ln Q_P + V phibar_S ln Q_S + dA sum_I sum_r omega_I Phi~_I.
    Since Phi_I(r) = -(dA)^-1 dG_0/d omega_I(r) for the first two terms (the
    density integrals are the derivatives of the log partition functions),
    dG/d omega_I(r) = dA (Phi~_I(r) - Phi_I[omega](r)); G is convex, so its
    minimisers are the fields that reproduce Phi~.
    """
    d = densities(omega, p, gauge)
    dA = p["dx"] ** 2
    V = p["nx"] * p["ny"] * dA
    phiP = p["phi_P"]
    return (V * phiP / p["n_contour"] * np.log(d["Q_P"]) + V * (1.0 - phiP) * np.log(d["Q_S"])
            + dA * float(np.sum(omega * phi_target)))


def secant_root(alpha_t, delta0, delta_t):
    """Step length of the line search (reading R22): the root of the directional
    derivative along the direction, linear through (0, delta0) and
    (alpha_t, delta_t); the trial length itself when the slope is not negative."""
    curv = delta0 - delta_t
    return alpha_t * delta0 / curv if curv > 0.0 else alpha_t


def local_response(phi, p):
    """Diagonal of the density response used to precondition the inversion
    (reading R25): N Phi_A, N Phi_B for the chain (the potential enters the
    propagator multiplied by N) and Phi_S for the solvent (Eq. phi_s)."""
    N = p["n_contour"]
    return np.stack([N * phi[0], N * phi[1], phi[2]])


def invert_densities(phi_target, omega0, p, tol=1e-8, max_iter=1000, precond=0):
    """Potentials reproducing the composition phi_target (App. C comments 2 and 3).

    Nonlinear conjugate gradients with the Fletcher-Reeves factor on the
    functional of reading R21: the descent direction at omega is
    s = Phi[omega] - Phi~ (minus the gradient over dA); directions
    d_0 = s_0, d_{k+1} = s_{k+1} + (|s_{k+1}|^2 / |s_k|^2) d_k.  Each line search
    (reading R22) evaluates the directional derivative d . s at a trial point
    omega + alpha_t d and takes the secant root
    alpha = alpha_t (d . s) / (d . s - d . s_t).  Stops when the RMS residual
    over the three fields (reading R23) is below tol.
    precond = 1 (reading R25): the directions are built from z = s / m, m the
    local response at the current iterate, and the factor is (s.z)_{k+1} /
    (s.z)_k; the line search and the stopping test are unchanged.
    Returns dict(omega, phi, iters, evals, restarts, resid0, resid, converged).
    """
    n = p["nx"] * p["ny"]
    x = np.array(omega0, dtype=np.float64, copy=True)

    def descent(w):
        ph = densities(w, p)["phi"]
        return ph - phi_target, ph

    def scaled(s, ph):
        if not precond:
            return s
        m = local_response(ph, p)
        return np.where(m > 0.0, s / np.where(m > 0.0, m, 1.0), s)  # a density rounded to zero keeps s

    s, ph = descent(x)
    evals = 1
    r2 = float(np.sum(s * s))
    resid0 = np.sqrt(r2 / n)
    out = dict(iters=0, restarts=0, resid0=resid0, resid=resid0, converged=resid0 < tol)
    if out["converged"]:
        return dict(out, omega=x, phi=ph, evals=evals)
    z = scaled(s, ph)
    sz = float(np.sum(s * z))
    d = z.copy()
    alpha_t = 1.0
    for it in range(1, max_iter + 1):
        delta0 = float(np.sum(d * s))
        if not delta0 > 0.0:
            d = z.copy()
            delta0 = sz
            out["restarts"] += 1
        delta_t = float(np.sum(d * descent(x + alpha_t * d)[0]))
        evals += 1
        alpha = secant_root(alpha_t, delta0, delta_t)
        x = x + alpha * d
        s, ph = descent(x)
        evals += 1
        out["iters"] = it
        out["resid"] = np.sqrt(float(np.sum(s * s)) / n)
        if out["resid"] < tol:
            out["converged"] = True
            break
        if not np.isfinite(out["resid"]):
            break  # a state that blew up: stop, unconverged
        z = scaled(s, ph)
        sz_new = float(np.sum(s * z))
        d = z + (sz_new / sz) * d
        sz, alpha_t = sz_new, alpha
    return dict(out, omega=x, phi=ph, evals=evals)


def step(state, p):
    """One hybrid LB/EPD step (App. C flow, readings R1-R3).

    1. advect Phi^n and omega^n with u^{n-1};
    1b. (cg_invert = 1) replace the advected omega by the potentials that
        reproduce the advected composition (invert_densities, tolerance
        cg_tol, at most cg_max_iter iterations);
    2. mu at the advected composition, omega^{n+1} by the EPD diffusion step;
    3. Phi^{n+1} = Phi[omega^{n+1}];
    4. S = sum_I (Phi_I^{n+1} - Phi~_I)/D_I, lattice force F;
    5. LB stream + collide with F, giving u^n.
    """
    couple = p.get("couple_lb", 1)
    u_adv = state["u"] if couple else np.zeros_like(state["u"])
    phi_t, omega_t = advect(state["phi"], state["omega"], u_adv)
    inv = None
    if p.get("cg_invert", 0):
        inv = invert_densities(phi_t, omega_t, p, p.get("cg_tol", 1e-8), p.get("cg_max_iter", 1000),
                               p.get("cg_precond", 0))
        omega_t = inv["omega"]
    omega_new = field_update(phi_t, omega_t, p)
    d = densities(omega_new, p)
    D = diffusivities(p)
    S = sum((d["phi"][I] - phi_t[I]) / D[I] for I in range(3))
    F = lattice_force(S, p)
    fstar, rho, u = lb_advance(state["fstar"], F, p)
    return dict(omega=omega_new, phi=d["phi"], fstar=fstar, u=u, rho=rho, n=state["n"] + 1,
                Q_P=d["Q_P"], Q_S=d["Q_S"], S=S, F=F, phi_t=phi_t, omega_t=omega_t, cg=inv)


def run(p, omega0, nsteps):
    s = init_state(p, omega0)
    for _ in range(nsteps):
        s = step(s, p)
    return s
