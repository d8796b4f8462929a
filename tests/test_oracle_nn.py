"""Pins of the surrogate oracle: gradients by central differences, the
dilated periodic convolution by brute-force loops, Adam by its definition on a
quadratic, and the renormalised densities' exact means."""
import numpy as np

from oracle import epdlb_oracle as O
from oracle import nn_oracle as NN


def small_params(rng, chans=(5, 4, 4, 3, 2)):
    ps = []
    for ci, co in zip(chans[:-1], chans[1:]):
        ps.append((0.4 * rng.standard_normal((9, ci, co)), 0.1 * rng.standard_normal(co)))
    return ps


def test_conv_matches_loops():
    rng = np.random.default_rng(0)
    a = rng.standard_normal((6, 7, 3))
    W = rng.standard_normal((9, 3, 2))
    b = rng.standard_normal(2)
    for d in (1, 2, 4):
        out = NN.conv(a, W, b, d)
        ref = np.zeros((6, 7, 2))
        for y in range(6):
            for x in range(7):
                acc = b.copy()
                for t, (ty, tx) in enumerate(NN.TAPS):
                    acc += a[(y + ty * d) % 6, (x + tx * d) % 7] @ W[t]
                ref[y, x] = acc
        assert np.max(np.abs(out - ref)) < 1e-13


def test_gradients_by_central_differences():
    rng = np.random.default_rng(1)
    params = small_params(rng)
    x = rng.standard_normal((8, 8, 5))
    target = 0.05 + 0.01 * rng.random((8, 8, 2))

    def loss(ps):
        o, _ = NN.forward(ps, x)
        return NN.loss_and_grad_output(o, target, 0.1)[0]

    o, cache = NN.forward(params, x)
    _, go = NN.loss_and_grad_output(o, target, 0.1)
    grads = NN.backward(params, cache, go)
    h = 1e-6
    for l in range(4):
        W, b = params[l]
        for idx in [(0, 0, 0), (4, W.shape[1] - 1, W.shape[2] - 1), (7, 1, 0)]:
            Wp = W.copy(); Wp[idx] += h
            Wm = W.copy(); Wm[idx] -= h
            pp = list(params); pp[l] = (Wp, b)
            pm = list(params); pm[l] = (Wm, b)
            fd = (loss(pp) - loss(pm)) / (2 * h)
            assert abs(fd - grads[l][0][idx]) < 1e-6 * max(1.0, abs(fd)), (l, idx, fd, grads[l][0][idx])
        bp = b.copy(); bp[0] += h
        bm = b.copy(); bm[0] -= h
        pp = list(params); pp[l] = (W, bp)
        pm = list(params); pm[l] = (W, bm)
        fd = (loss(pp) - loss(pm)) / (2 * h)
        assert abs(fd - grads[l][1][0]) < 1e-6 * max(1.0, abs(fd))


def test_input_gradient_is_adjoint():
    """<g, conv(a)> = <conv_input_grad(g), a> + <g, bias> for random a, g (adjoint identity)."""
    rng = np.random.default_rng(2)
    a = rng.standard_normal((8, 6, 3))
    g = rng.standard_normal((8, 6, 4))
    W = rng.standard_normal((9, 3, 4))
    for d in (1, 2, 8):
        lhs = np.sum(g * NN.conv(a, W, np.zeros(4), d))
        rhs = np.sum(NN.conv_input_grad(g, W, d) * a)
        assert abs(lhs - rhs) < 1e-10 * abs(lhs)
        gw = NN.conv_weight_grad(a, g, d)
        assert abs(np.sum(gw * W) - lhs) < 1e-10 * abs(lhs)


def test_adam_on_quadratic():
    """Adam's first step moves each coordinate by lr against the gradient sign
    (bias-corrected m/sqrt(v) = g/|g|); many steps reach the minimum."""
    theta = np.array([3.0, -2.0])
    m = np.zeros(2)
    v = np.zeros(2)
    t1, m, v = NN.adam_update(theta, 2 * theta, m, v, 1, 0.1)
    assert np.allclose(t1, theta - 0.1 * np.sign(theta), atol=1e-7)
    th = t1
    for t in range(2, 600):
        th, m, v = NN.adam_update(th, 2 * th, m, v, t, 0.05)
    assert np.max(np.abs(th)) < 1e-2


def test_surrogate_densities_have_exact_means():
    rng = np.random.default_rng(3)
    params = small_params(rng)
    omega = 0.3 * rng.standard_normal((3, 8, 8))
    p = dict(f_A=0.3, phi_P=0.15, n_contour=16)
    phi = NN.predict_densities(params, omega, p)
    assert abs(phi[0].mean() - 0.3 * 0.15) < 1e-15
    assert abs(phi[1].mean() - 0.7 * 0.15) < 1e-15
    assert abs(phi[2].mean() - 0.85) < 1e-15
    assert np.all(phi > 0)


def test_bf16_rounding_values():
    r = NN.bf16_round(np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, np.pi, -2.5, 0.0, 65280.0 + 128]))
    # ties go to the even mantissa: 1 + 2^-8 -> 1, 1 + 3*2^-8 -> 1 + 2^-6
    assert list(r) == [1.0, 1.0, 1 + 2.0 ** -6, 3.140625, -2.5, 0.0, 65536.0]
    x = np.random.default_rng(4).standard_normal(10000) * 10.0 ** np.random.default_rng(5).integers(-5, 5, 10000)
    rel = np.abs(NN.bf16_round(x) - x) / np.abs(x)
    assert rel.max() <= 2.0 ** -8 * (1 + 1e-6)


def _small_p(**kw):
    p = dict(O_defaults())
    p.update(kw)
    return p


def O_defaults():
    from seeded_inputs import preset
    return preset("cfg1", nx=16, ny=16, n_contour=8)


def test_surrogate_run_with_exact_densities_is_the_exact_run():
    """A 'network' that returns the exact densities reproduces the plain hybrid step."""
    p = _small_p()
    w0 = 0.2 * np.random.default_rng(6).standard_normal((3, p["ny"], p["nx"]))
    ref = O.init_state(p, w0)
    for _ in range(5):
        ref = O.step(ref, p)
    s = NN.surrogate_run(p, None, w0, 5, 2, dens_fn=lambda w: O.densities(w, p)["phi"])
    for k in ("omega", "phi", "fstar", "u", "S"):
        assert np.max(np.abs(s[k] - ref[k])) <= 1e-13 * max(1.0, np.max(np.abs(ref[k]))), k
    assert max(s["errs"]) < 1e-15


def test_surrogate_force_differences_one_estimator():
    """Frozen flow (no advection): with a biased estimator f = exact + delta,
    S at every step, including those after exact steps, equals
    sum_I (f(omega_k) - f(omega_{k-1}))/D_I: the estimator's bias cancels."""
    p = _small_p(couple_lb=0)
    rng = np.random.default_rng(7)
    w0 = 0.2 * rng.standard_normal((3, p["ny"], p["nx"]))
    delta = 1e-3 * rng.standard_normal((3, p["ny"], p["nx"]))
    delta[2] = 0.0

    def f(w):
        return O.densities(w, p)["phi"] + delta

    s = NN.surrogate_run(p, None, w0, 7, 3, dens_fn=f, history=True)
    D = O.diffusivities(p)
    for k in range(1, 8):
        ref = sum((f(s["omegas"][k])[I] - f(s["omegas"][k - 1])[I]) / D[I] for I in range(3))
        assert np.max(np.abs(s["Ss"][k - 1] - ref)) < 1e-12, k
    assert np.allclose(s["errs"], np.max(np.abs(delta[:2])), rtol=0, atol=1e-16)


def test_activation_closed_forms():
    """softplus(z) = ln(1 + e^z), sigmoid its derivative, SiLU z sigmoid(z) with
    derivative sigmoid(z)(1 + z(1 - sigmoid(z))), at points with closed values."""
    z = np.array([0.0, np.log(np.e - 1.0), -np.log(3.0), 40.0, -40.0])
    assert np.allclose(NN.softplus(z), [np.log(2.0), 1.0, np.log(4.0 / 3.0), 40.0, np.exp(-40.0)],
                       rtol=1e-15, atol=1e-300)
    assert np.allclose(NN.sigmoid(np.array([0.0, np.log(3.0)])), [0.5, 0.75], rtol=1e-15)
    assert np.allclose(NN.silu(np.array([0.0, np.log(3.0)])), [0.0, 0.75 * np.log(3.0)], rtol=1e-15)
    h = 1e-6
    zz = np.linspace(-4, 4, 17)
    assert np.max(np.abs((NN.softplus(zz + h) - NN.softplus(zz - h)) / (2 * h) - NN.sigmoid(zz))) < 1e-9
    assert np.max(np.abs((NN.silu(zz + h) - NN.silu(zz - h)) / (2 * h) - NN.silu_grad(zz))) < 1e-9


def test_input_channels_and_gauge_invariance():
    """The network sees w_I - <w_I> and the constant channels f_A and 1/N, so its
    densities, like the exact ones (Sec. II: the potentials enter only up to a
    constant per species), do not change when a constant is added to a field."""
    rng = np.random.default_rng(9)
    omega = 0.3 * rng.standard_normal((3, 8, 8))
    x = NN.make_input(omega, 0.3, 32)
    assert np.all(x[..., 3] == 0.3) and np.all(x[..., 4] == 0.03125)
    assert np.max(np.abs(x[..., :3].mean(axis=(0, 1)))) < 1e-16
    params = small_params(rng)
    p = dict(f_A=0.3, phi_P=0.15, n_contour=32)
    a = NN.predict_densities(params, omega, p)
    b = NN.predict_densities(params, omega + np.array([0.7, -1.2, 2.5])[:, None, None], p)
    assert np.max(np.abs(a - b)) < 1e-14
    ex_a = O.densities(omega, dict(O_defaults(), nx=8, ny=8, n_contour=32, f_A=0.3, phi_P=0.15))["phi"]
    ex_b = O.densities(omega + np.array([0.7, -1.2, 2.5])[:, None, None],
                       dict(O_defaults(), nx=8, ny=8, n_contour=32, f_A=0.3, phi_P=0.15))["phi"]
    assert np.max(np.abs(ex_a - ex_b)) < 1e-14


def test_exact_steps_fall_on_multiples_of_the_fallback_interval():
    """Step k (counted from 0 after seeding) is exact when k % fallback_every == 0:
    the first step is exact, and with a biased estimator the state's densities
    carry the bias exactly after the other steps."""
    p = _small_p(couple_lb=0)
    rng = np.random.default_rng(12)
    w0 = 0.2 * rng.standard_normal((3, p["ny"], p["nx"]))
    delta = 1e-3 * rng.standard_normal((3, p["ny"], p["nx"]))
    delta[2] = 0.0

    def f(w):
        return O.densities(w, p)["phi"] + delta

    for n in range(1, 8):
        s = NN.surrogate_run(p, None, w0, n, 3, dens_fn=f)
        assert len(s["errs"]) == 1 + len(range(0, n, 3)), n
        last_exact = (n - 1) % 3 == 0
        dev = np.max(np.abs(s["phi"] - O.densities(s["omega"], p)["phi"]))
        assert (dev < 1e-15) if last_exact else abs(dev - np.max(np.abs(delta))) < 1e-15, n
