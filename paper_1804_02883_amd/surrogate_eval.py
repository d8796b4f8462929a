"""Plain versus surrogate hybrid steps on one workload (library calls only).

Both runs start from the same seeded potentials.  The surrogate run takes an
exact step every `fallback_every` steps (and when its residual test fires);
at each of them the library records max |Phi_NN - Phi_exact| over sites and
species A, B, which is the error reported here.  Timing: HIP events around
the stepped region on the runs' stream, after a warm-up that also captures
the step graphs.
"""
import time

import numpy as np


def _timed_steps(sim, steps, stream):
    import torch
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    sim.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1)


def compare(params, seed, sigma, weights, steps, fallback_every=50, check_every=10, resid_tol=1e-3,
            err_tol=9e-4, warmup=None, tune_cache=None):
    """Returns a dict: plain and surrogate site-updates/s, speedup, errors.  With
    `tune_cache` both runs use the autotuned FFT launch shapes (read from the
    cache, tuned and appended when missing)."""
    from paper_1804_02883_amd import Simulation
    n = params["nx"] * params["ny"]
    warm = fallback_every if warmup is None else warmup
    out = {}
    # plain
    pp = dict(params, density_mode=0)
    sim = Simulation(pp)
    sim.seed(seed, sigma)
    if tune_cache:
        sim.autotune(20, tune_cache)
    sim.step(2)
    ms_warm = _timed_steps(sim, warm - 2, sim.stream)
    ms = _timed_steps(sim, steps, sim.stream)
    sim.sync()
    phi_plain = sim.densities()
    out["plain"] = dict(value=n * steps / (ms / 1e3), ms_per_step=ms / steps)
    sim.close()
    # surrogate
    ps = dict(params, density_mode=1, fallback_every=fallback_every, check_every=check_every,
              resid_tol=resid_tol, err_tol=err_tol)
    sim = Simulation(ps)
    sim.surrogate_set_weights(weights)
    sim.seed(seed, sigma)
    if tune_cache:
        sim.autotune(20, tune_cache)
    sim.step(2)
    _timed_steps(sim, warm - 2, sim.stream)
    ms_s = _timed_steps(sim, steps, sim.stream)
    sim.sync()
    d = sim.diag()
    phi_sur = sim.densities()
    sim.close()
    out["surrogate"] = dict(value=n * steps / (ms_s / 1e3), ms_per_step=ms_s / steps, n_exact=d["n_exact"],
                            n_triggered=d["n_triggered"], density_err_in_use=d["nn_err_in_use"],
                            max_density_err=d["nn_err_max"],
                            last_density_err=d["nn_err_last"], resid_max=d["resid_nn_max"],
                            resid_exact=d["resid_exact"])
    out["speedup"] = out["surrogate"]["value"] / out["plain"]["value"]
    # trajectory difference after warm-up + steps, and the size of the density
    # fluctuations (the error of predicting uniform densities)
    phiP_s, phiP_p = phi_sur[0] + phi_sur[1], phi_plain[0] + phi_plain[1]
    out["sigma_delta"] = float(np.mean(np.abs(phiP_s - phiP_p)))
    out["fluct_max"] = float(np.max(np.abs(phi_plain[:2] - phi_plain[:2].mean(axis=(1, 2), keepdims=True))))
    out["steps"] = steps + warm
    return out


def error_trace(params, seed, sigma, weights, steps, fallback_every=50):
    """Surrogate error at every exact step of one run (host reads after each interval; not timed)."""
    from paper_1804_02883_amd import Simulation
    ps = dict(params, density_mode=1, fallback_every=fallback_every, check_every=10, resid_tol=1e-3, err_tol=0.0)
    sim = Simulation(ps)
    sim.surrogate_set_weights(weights)
    sim.seed(seed, sigma)
    errs, fluct = [], []
    for k in range(steps // fallback_every):
        sim.step(fallback_every)
        d = sim.diag()
        errs.append(d["nn_err_last"])
        if k % 20 == 0:
            phi = sim.densities()
            fluct.append(float(np.max(np.abs(phi[:2] - phi[:2].mean(axis=(1, 2), keepdims=True)))))
    sim.close()
    e = np.array(errs)
    return dict(every=fallback_every, err_first10=[round(x, 6) for x in e[:10]],
                err_max=float(e.max()), err_argmax_step=int(e.argmax()) * fallback_every,
                steps_over_1e3=int(np.sum(e > 1e-3)) * fallback_every, err_p50=float(np.median(e)),
                fluct_every_1000=[round(x, 5) for x in fluct])
