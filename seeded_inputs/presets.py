"""Named workloads: grid shapes, chain and interaction parameters, seeds.

Defaults follow the paper's unit system and parameter set (Sec. III): R_G = 1,
D_S = 1, D_A = D_B = D_S/N, grid spacing R_G/3, time step 0.002 tau.  The
Helfand parameter is kappa_H = 20/N (1.176 at the paper's N = 17), and the
Flory-Huggins parameters follow one of two readings:

* "L": chi_AB = chi_AS = 1.5/N, chi_BS = 0 (homogeneous state stable);
* "Q": chi_AB = 1.05*17/N, chi_AS = 1.20*17/N, chi_BS = 0 (the paper's values
  rescaled to fixed chi*N; a quench into the unstable region).

The body-force amplitude g is given in the paper's force unit
f* = rho R_G tau^-2 (Sec. IV) unless g_units = 1 (lattice units).
"""

SIZES_BATCH = [(64, 64), (128, 128), (256, 128), (512, 256)]


def base_params(nx, ny, N, f_A=0.5, phi_P=0.1, chi="L", g=1e-5, precision=1):
    if chi == "L":
        chi_AB, chi_AS, chi_BS = 1.5 / N, 1.5 / N, 0.0
    elif chi == "Q":
        chi_AB, chi_AS, chi_BS = 1.05 * 17.0 / N, 1.20 * 17.0 / N, 0.0
    else:
        raise ValueError("chi reading must be 'L' or 'Q'")
    return dict(
        nx=nx, ny=ny, n_contour=N, f_A=f_A, phi_P=phi_P,
        chi_AB=chi_AB, chi_AS=chi_AS, chi_BS=chi_BS, kappa_H=20.0 / N,
        D_S=1.0, D_A=1.0 / N, D_B=1.0 / N,
        R_G=1.0, dx=1.0 / 3.0, dt=0.002, kT_over_v=1.0,
        lb_tau=1.0, g=g, g_units=0,
        precision=precision, init_flow=1, couple_lb=1,
    )


PRESETS = {
    "cfg1": dict(params=base_params(32, 32, 16, 0.5, 0.1, "L", 1e-5, precision=0),
                 steps=200, seed=1001, sigma=1e-3,
                 name="32x32 FP64 N=16 f_A=0.5 phi_P=0.1"),
    "cfg2": dict(params=base_params(256, 256, 32, 0.5, 0.1, "L", 1e-5),
                 steps=10000, seed=1002, sigma=1e-3,
                 name="256x256 FP32 N=32 f_A=0.5 phi_P=0.1"),
    "cfg3": dict(params=base_params(1024, 512, 64, 0.3, 0.15, "L", 1e-5),
                 steps=50000, seed=1003, sigma=1e-3, g_values=(1e-6, 1e-5, 5e-5),
                 name="1024x512 FP32 N=64 f_A=0.3 phi_P=0.15"),
    "cfg5": dict(params=base_params(512, 512, 32, 0.5, 0.1, "L", 1e-5),
                 steps=20000, seed=1005, sigma=1e-3,
                 name="512x512 FP32 N=32 f_A=0.5 phi_P=0.1"),
    # the surrogate comparison: a quench (reading Q) from a stronger seeded
    # noise, so that the density fluctuations exceed the 1e-3 error bar
    "cfg5q": dict(params=base_params(512, 512, 32, 0.5, 0.1, "Q", 1e-5),
                  steps=20000, seed=1005, sigma=0.05,
                  name="512x512 FP32 N=32 f_A=0.5 phi_P=0.1, chi reading Q, noise 0.05"),
}


def preset(name, **overrides):
    """A copy of the named workload's parameter dict with overrides applied."""
    p = dict(PRESETS[name]["params"])
    p.update(overrides)
    return p


def replica_manifest(n_replicas=64, manifest_seed=4242, N=32, phi_P=0.1):
    """The batched workload: uneven grids, own seed, force and A fraction each.

    Replica r draws three SplitMix64 uniforms (u0, u1, u2) from `manifest_seed`:
    grid = SIZES_BATCH[min(int(4 u0), 3)], g = 5e-5 u1, f_A = 0.3 if u2 <= 0.5
    else 0.5; its noise seed is 4000 + r.
    """
    from .noise import splitmix64_uniforms
    u = splitmix64_uniforms(manifest_seed, 3 * n_replicas)
    out = []
    for r in range(n_replicas):
        nx, ny = SIZES_BATCH[min(int(4.0 * u[3 * r]), 3)]
        g = 5e-5 * float(u[3 * r + 1])
        f_A = 0.3 if u[3 * r + 2] <= 0.5 else 0.5
        out.append(dict(params=base_params(nx, ny, N, f_A, phi_P, "L", g),
                        seed=4000 + r, sigma=1e-3))
    return out
