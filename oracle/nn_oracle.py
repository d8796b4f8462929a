"""FP64 CPU oracle of the density surrogate -- test infrastructure only.

The learned part is not in the paper; it stands in for the chain-propagator
step (Sec. II: modified diffusion equations, split step, density integrals)
between exact evaluations.  Network (one sample, periodic grid ny x nx):

  x   = (w_A - <w_A>, w_B - <w_B>, w_S - <w_S>, f_A, 1/N)       5 channels
  z_l = b_l + sum_{t in taps} sum_ci a_{l-1}[r + d_l t, ci] W_l[t, ci, co]
        taps t = (ty, tx) in {-1,0,1}^2 (index (ty+1)*3 + (tx+1)), dilations d = (1, 2, 4, 8)
  a_l = SiLU(z_l) = z_l * sigmoid(z_l)     l = 1, 2, 3;   o = z_4 (2 channels)
  Phi_hat_c = softplus(o_c)                c = A, B
  loss = mean over sites and c of ((Phi_hat_c - Phi_c) / phibar_P)^2

Inference renormalises Phi_hat to the exact means (<Phi_A> = f_A phibar_P,
<Phi_B> = (1 - f_A) phibar_P, which the exact densities satisfy, see the
compressibility pins) and takes Phi_S from its closed form (Eq. phi_s).
Adam: Kingma and Ba, "Adam: a method for stochastic optimization" (2015).
Arrays are [y, x, channel] (channels last).

`rnd` arguments (default: none) round the values a BF16 implementation
stores between its steps -- network input, weights, hidden activations,
pre-activations kept for the backward pass, and the propagated gradients --
so that the oracle takes the same rounding decisions as such an
implementation; every sum is still taken in FP64.

surrogate_run() is the hybrid step of the main oracle with these densities
between exact steps (an exact step every `fallback_every` steps): the force
source S always differences network densities (at an exact step the exact
densities become the state and S~ of the next step is corrected by the
difference of the two estimators at this step).
"""
import numpy as np

from oracle import epdlb_oracle as O

DILATIONS = (1, 2, 4, 8)
TAPS = [(ty, tx) for ty in (-1, 0, 1) for tx in (-1, 0, 1)]


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def softplus(z):
    return np.logaddexp(0.0, z)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def conv(a, W, b, d):
    """Periodic dilated 3x3 convolution: a [ny, nx, ci], W [9, ci, co], b [co]."""
    out = np.broadcast_to(b, a.shape[:2] + (W.shape[2],)).astype(np.float64).copy()
    for t, (ty, tx) in enumerate(TAPS):
        sh = np.roll(a, shift=(-ty * d, -tx * d), axis=(0, 1))  # sh[r] = a[r + d t]
        out += sh @ W[t]
    return out


def conv_input_grad(g, W, d):
    """d/d a of sum(g * conv(a)): sum_t g[r - d t] W[t]^T."""
    out = np.zeros(g.shape[:2] + (W.shape[1],))
    for t, (ty, tx) in enumerate(TAPS):
        sh = np.roll(g, shift=(ty * d, tx * d), axis=(0, 1))  # sh[r] = g[r - d t]
        out += sh @ W[t].T
    return out


def conv_weight_grad(a, g, d):
    """d/d W[t] of sum(g * conv(a)) = sum_r a[r + d t]^T g[r]."""
    ci, co = a.shape[2], g.shape[2]
    out = np.zeros((9, ci, co))
    for t, (ty, tx) in enumerate(TAPS):
        sh = np.roll(a, shift=(-ty * d, -tx * d), axis=(0, 1))
        out[t] = sh.reshape(-1, ci).T @ g.reshape(-1, co)
    return out


def make_input(omega, f_A, N):
    """5-channel input from the potentials (3, ny, nx)."""
    ny, nx = omega.shape[1:]
    x = np.empty((ny, nx, 5))
    for I in range(3):
        x[..., I] = omega[I] - np.mean(omega[I])
    x[..., 3] = f_A
    x[..., 4] = 1.0 / N
    return x


def bf16_round(a):
    """Nearest bfloat16 (ties to even) of float32(a), returned as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def _ident(a):
    return a


def forward(params, x, rnd=None):
    """params: list of (W [9, ci, co], b [co]).  Returns (o, cache)."""
    rnd = rnd or _ident
    a = x
    cache = []
    for l, (W, b) in enumerate(params):
        z = conv(a, W, b, DILATIONS[l])
        cache.append((a, z))
        a = rnd(silu(z)) if l < len(params) - 1 else z
    return a, cache


def loss_and_grad_output(o, phi_ab, phiP):
    """MSE of softplus(o) against the exact (Phi_A, Phi_B) [ny, nx, 2]; returns (loss, dL/do)."""
    r = (softplus(o) - phi_ab) / phiP
    M = r.size
    loss = float(np.sum(r * r) / M)
    return loss, 2.0 * r / phiP * sigmoid(o) / M


def backward(params, cache, go, rnd=None):
    """Gradients [(dW, db)] of the loss given dL/do."""
    rnd = rnd or _ident
    grads = [None] * len(params)
    g = rnd(go)
    for l in range(len(params) - 1, -1, -1):
        W, b = params[l]
        a_in, z = cache[l]
        if l < len(params) - 1:
            g = rnd(g * silu_grad(rnd(z)))
        grads[l] = (conv_weight_grad(a_in, g, DILATIONS[l]), g.sum(axis=(0, 1)))
        if l > 0:
            g = conv_input_grad(g, W, DILATIONS[l])
    return grads


def predict_densities(params, omega, p, gauge_S=None, rnd=None):
    """Surrogate densities (3, ny, nx): renormalised NN output plus exact Phi_S."""
    x = make_input(omega, p["f_A"], p["n_contour"])
    if rnd:
        x = rnd(x)
    o, _ = forward(params, x, rnd)
    ph = softplus(o)
    phiA = ph[..., 0] * (p["f_A"] * p["phi_P"] / np.mean(ph[..., 0]))
    phiB = ph[..., 1] * ((1 - p["f_A"]) * p["phi_P"] / np.mean(ph[..., 1]))
    wS = omega[2]
    c = np.mean(wS) if gauge_S is None else gauge_S
    e = np.exp(-(wS - c))
    phiS = (1 - p["phi_P"]) * e / np.mean(e)
    return np.stack([phiA, phiB, phiS])


def adam_update(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def round_params(params, rnd):
    """Weights as a BF16 implementation holds them (biases stay FP32)."""
    return [(rnd(W), np.asarray(b, dtype=np.float32).astype(np.float64)) for W, b in params]


def surrogate_run(p, params, omega0, nsteps, fallback_every, rnd=None, dens_fn=None, history=False):
    """Hybrid steps with network densities between exact steps.

    Returns the final state (as the main oracle's step) plus 'errs': the max
    over sites and species A, B of |Phi_NN - Phi_exact| at the seed and at
    every exact step.  dens_fn(omega) replaces the network (for pins);
    history=True adds the lists 'omegas' (seed first) and 'Ss'."""
    D = O.diffusivities(p)
    if dens_fn is None:
        def dens_fn(w):
            return predict_densities(params, w, p, rnd=rnd)
    s = O.init_state(p, omega0)
    omegas, Ss = [s["omega"]], []
    nn0 = dens_fn(s["omega"])
    corr = sum((nn0[I] - s["phi"][I]) / D[I] for I in (0, 1))
    errs = [float(np.max(np.abs(nn0[:2] - s["phi"][:2])))]
    last_exact = True
    couple = p.get("couple_lb", 1)
    for k in range(nsteps):
        exact = k % fallback_every == 0
        u_adv = s["u"] if couple else np.zeros_like(s["u"])
        phi_t, omega_t = O.advect(s["phi"], s["omega"], u_adv)
        omega_new = O.field_update(phi_t, omega_t, p)
        nn = dens_fn(omega_new)
        S = sum((nn[I] - phi_t[I]) / D[I] for I in range(3))
        if last_exact:
            S = S - corr
        if exact:
            phi_new = O.densities(omega_new, p)["phi"]
            corr = sum((nn[I] - phi_new[I]) / D[I] for I in (0, 1))
            errs.append(float(np.max(np.abs(nn[:2] - phi_new[:2]))))
        else:
            phi_new = nn
        F = O.lattice_force(S, p)
        fstar, rho, u = O.lb_step(s["fstar"], F, p["lb_tau"])
        s = dict(omega=omega_new, phi=phi_new, fstar=fstar, u=u, rho=rho, n=s["n"] + 1, S=S, F=F)
        last_exact = exact
        if history:
            omegas.append(omega_new)
            Ss.append(S)
    s["errs"] = errs
    if history:
        s["omegas"], s["Ss"] = omegas, Ss
    return s
