"""ctypes binding of libepdlb.so: the C ABI's functions under the same names,
plus a small `Simulation` convenience wrapper.

Argument marshalling only: every step of the simulation runs in the HIP
kernels of the library.  PyTorch supplies device memory (the context's
workspace is a torch uint8 tensor) and the stream (`work_stream`: torch's
current stream, or a torch stream of its own when that is the legacy default
stream), so torch's allocator and events see the library's work.  Without a GPU the host
entry points (params, validation, workspace size, noise) still work.
"""
import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libepdlb.so")

EPDLB_ABI_VERSION = 1
EPDLB_OK = 0
EPDLB_EINVAL = -1
EPDLB_ENOMEM = -2
EPDLB_EHIP = -3
EPDLB_ENONFINITE = -4
EPDLB_EUNSTABLE = -5
EPDLB_ESTATE = -6
EPDLB_ENODEV = -7

EPDLB_STAGE_ADVECT_UPDATE = 1
EPDLB_STAGE_DENSITIES = 2
EPDLB_STAGE_FORCE = 3
EPDLB_STAGE_LB = 4

EPDLB_AUX_STILDE = 1
EPDLB_AUX_S = 2
EPDLB_AUX_FORCE = 3

EPDLB_NN_PARAMS = 77954


class epdlb_params(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("n_contour", ctypes.c_int32),
        ("f_A", ctypes.c_double), ("phi_P", ctypes.c_double),
        ("chi_AB", ctypes.c_double), ("chi_AS", ctypes.c_double), ("chi_BS", ctypes.c_double),
        ("kappa_H", ctypes.c_double),
        ("D_S", ctypes.c_double), ("D_A", ctypes.c_double), ("D_B", ctypes.c_double),
        ("R_G", ctypes.c_double), ("dx", ctypes.c_double), ("dt", ctypes.c_double),
        ("kT_over_v", ctypes.c_double),
        ("lb_tau", ctypes.c_double), ("g", ctypes.c_double),
        ("g_units", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("init_flow", ctypes.c_int32), ("couple_lb", ctypes.c_int32),
        ("density_mode", ctypes.c_int32), ("fallback_every", ctypes.c_int32),
        ("check_every", ctypes.c_int32), ("resid_tol", ctypes.c_double), ("err_tol", ctypes.c_double),
        ("lb_mrt", ctypes.c_int32),
        ("lb_gamma_s", ctypes.c_double), ("lb_gamma_b", ctypes.c_double), ("lb_gamma_g", ctypes.c_double),
        ("cg_invert", ctypes.c_int32), ("cg_max_iter", ctypes.c_int32), ("cg_tol", ctypes.c_double),
        ("cg_precond", ctypes.c_int32),
        ("mach_max", ctypes.c_double),
    ]


class epdlb_diag(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64),
        ("Q_P", ctypes.c_double), ("Q_P_bwd", ctypes.c_double),
        ("Q_S", ctypes.c_double), ("gauge_S", ctypes.c_double),
        ("mean_omega", ctypes.c_double * 3),
        ("n_exact", ctypes.c_int64), ("n_triggered", ctypes.c_int64),
        ("nn_err_last", ctypes.c_double), ("nn_err_max", ctypes.c_double),
        ("resid_nn_max", ctypes.c_double), ("resid_exact", ctypes.c_double),
        ("nn_err_in_use", ctypes.c_double),
    ]


class epdlb_kernel_stat(ctypes.Structure):
    _fields_ = [
        ("name", ctypes.c_char * 32),
        ("launches", ctypes.c_int64),
        ("total_ms", ctypes.c_double), ("min_ms", ctypes.c_double), ("max_ms", ctypes.c_double),
    ]


class epdlb_shape(ctypes.Structure):
    _fields_ = [("family", ctypes.c_char * 16), ("R", ctypes.c_int32), ("nf", ctypes.c_int32),
                ("us", ctypes.c_double)]


class epdlb_dev_views(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("plane", ctypes.c_int64),
                ("omega", ctypes.c_void_p), ("phi", ctypes.c_void_p),
                ("rho", ctypes.c_void_p), ("u", ctypes.c_void_p)]


class epdlb_obs(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_double), ("y2p", ctypes.c_double),
                ("n_particles", ctypes.c_int32), ("n_wrapping", ctypes.c_int32)]


class epdlb_particle(ctypes.Structure):
    _fields_ = [("label", ctypes.c_int32), ("area", ctypes.c_int32), ("wraps", ctypes.c_int32),
                ("born", ctypes.c_int32), ("content", ctypes.c_double), ("cx", ctypes.c_double),
                ("cy", ctypes.c_double), ("gxx", ctypes.c_double), ("gxy", ctypes.c_double),
                ("gyy", ctypes.c_double), ("R", ctypes.c_double), ("c_rel", ctypes.c_double)]


class epdlb_cg_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("evals", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("resid0", ctypes.c_double), ("resid", ctypes.c_double)]


class EpdlbError(RuntimeError):
    def __init__(self, code, fn, msg):
        super().__init__(f"{fn} failed ({code}): {msg}")
        self.code = code


_lib = None

_P = ctypes.POINTER
_dp = _P(ctypes.c_double)
_fp = _P(ctypes.c_float)
_ip = _P(ctypes.c_int32)
_vp = ctypes.c_void_p

SIGNATURES = {
    "epdlb_params_default": (ctypes.c_int, [_P(epdlb_params)]),
    "epdlb_validate": (ctypes.c_int, [_P(epdlb_params)]),
    "epdlb_mrt_gammas": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_int32, _dp, _dp]),
    "epdlb_workspace_bytes": (ctypes.c_int, [_P(epdlb_params), _P(ctypes.c_size_t)]),
    "epdlb_noise_fill": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_double, ctypes.c_int32,
                                        ctypes.c_int32, _dp]),
    "epdlb_create": (ctypes.c_int, [_P(epdlb_params), ctypes.c_int, _vp, _vp, ctypes.c_size_t,
                                    _P(_vp)]),
    "epdlb_seed": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.c_double]),
    "epdlb_set_fields": (ctypes.c_int, [_vp, _dp]),
    "epdlb_set_state": (ctypes.c_int, [_vp, _dp, _dp, _dp, _dp]),
    "epdlb_get_state": (ctypes.c_int, [_vp, _dp, _dp, _dp, _dp]),
    "epdlb_device_views": (ctypes.c_int, [_vp, _P(epdlb_dev_views)]),
    "epdlb_step": (ctypes.c_int, [_vp, ctypes.c_int64]),
    "epdlb_run_stage": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "epdlb_sync": (ctypes.c_int, [_vp]),
    "epdlb_read_densities": (ctypes.c_int, [_vp, _dp, _dp, _dp]),
    "epdlb_read_fields": (ctypes.c_int, [_vp, _dp, _dp, _dp]),
    "epdlb_read_velocity": (ctypes.c_int, [_vp, _dp, _dp, _dp]),
    "epdlb_read_populations": (ctypes.c_int, [_vp, _dp]),
    "epdlb_read_aux": (ctypes.c_int, [_vp, ctypes.c_int32, _dp]),
    "epdlb_write_aux": (ctypes.c_int, [_vp, ctypes.c_int32, _dp]),
    "epdlb_read_diag": (ctypes.c_int, [_vp, _P(epdlb_diag)]),
    "epdlb_autotune": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_char_p]),
    "epdlb_get_shapes": (ctypes.c_int, [_vp, _P(epdlb_shape), ctypes.c_int32, _P(ctypes.c_int32)]),
    "epdlb_set_shape": (ctypes.c_int, [_vp, ctypes.c_char_p, ctypes.c_int32, ctypes.c_int32]),
    "epdlb_profile_start": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "epdlb_profile_read": (ctypes.c_int, [_vp, _P(epdlb_kernel_stat), ctypes.c_int32,
                                          _P(ctypes.c_int32)]),
    "epdlb_destroy": (None, [_vp]),
    "epdlb_batch_create": (ctypes.c_int, [_P(epdlb_params), ctypes.c_int32, ctypes.c_int, _vp, _P(_vp)]),
    "epdlb_batch_seed": (ctypes.c_int, [_vp, _P(ctypes.c_uint64), ctypes.c_double]),
    "epdlb_batch_set_fields": (ctypes.c_int, [_vp, ctypes.c_int32, _dp]),
    "epdlb_batch_step": (ctypes.c_int, [_vp, ctypes.c_int64]),
    "epdlb_batch_sync": (ctypes.c_int, [_vp]),
    "epdlb_batch_read_densities": (ctypes.c_int, [_vp, ctypes.c_int32, _dp, _dp, _dp]),
    "epdlb_batch_read_fields": (ctypes.c_int, [_vp, ctypes.c_int32, _dp, _dp, _dp]),
    "epdlb_batch_read_velocity": (ctypes.c_int, [_vp, ctypes.c_int32, _dp, _dp, _dp]),
    "epdlb_batch_read_diag": (ctypes.c_int, [_vp, ctypes.c_int32, _P(epdlb_diag)]),
    "epdlb_batch_autotune": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_char_p]),
    "epdlb_batch_info": (ctypes.c_int, [_vp, _P(ctypes.c_int32), _P(ctypes.c_int64)]),
    "epdlb_batch_profile_start": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "epdlb_batch_profile_read": (ctypes.c_int, [_vp, _P(epdlb_kernel_stat), ctypes.c_int32,
                                                _P(ctypes.c_int32)]),
    "epdlb_batch_destroy": (None, [_vp]),
    "epdlb_surrogate_set_weights": (ctypes.c_int, [_vp, _fp, ctypes.c_int64]),
    "epdlb_nn_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int, _vp, _P(_vp)]),
    "epdlb_nn_set_weights": (ctypes.c_int, [_vp, _fp, ctypes.c_int64]),
    "epdlb_nn_get_weights": (ctypes.c_int, [_vp, _fp, ctypes.c_int64]),
    "epdlb_nn_set_pair": (ctypes.c_int, [_vp, ctypes.c_int32, _dp, _dp, ctypes.c_double, ctypes.c_int32]),
    "epdlb_nn_capture": (ctypes.c_int, [_vp, ctypes.c_int32, _vp]),
    "epdlb_nn_evaluate": (ctypes.c_int, [_vp, _ip, ctypes.c_int32, ctypes.c_double, _dp, _dp, _fp]),
    "epdlb_nn_train_step": (ctypes.c_int, [_vp, _ip, ctypes.c_int32, ctypes.c_double, ctypes.c_double]),
    "epdlb_nn_last_loss": (ctypes.c_int, [_vp, _dp, _dp]),
    "epdlb_nn_predict": (ctypes.c_int, [_vp, ctypes.c_int32, _dp]),
    "epdlb_nn_destroy": (None, [_vp]),
    "epdlb_observables": (ctypes.c_int, [_vp, ctypes.c_double, _P(epdlb_obs), _P(epdlb_particle), ctypes.c_int32,
                                         _P(ctypes.c_int32)]),
    "epdlb_sigma_delta": (ctypes.c_int, [_vp, _vp, _dp]),
    "epdlb_sigma_delta_noalloc": (ctypes.c_int, [_vp, _vp, _dp]),
    "epdlb_track_particles": (ctypes.c_int, [_vp, ctypes.c_double, _P(epdlb_obs), _P(epdlb_particle), ctypes.c_int32,
                                             _P(ctypes.c_int32)]),
    "epdlb_track_reset": (ctypes.c_int, [_vp]),
    "epdlb_batch_observables": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_double, _P(epdlb_obs),
                                               _P(epdlb_particle), ctypes.c_int32, _P(ctypes.c_int32)]),
    "epdlb_batch_track_particles": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_double, _P(epdlb_obs),
                                                   _P(epdlb_particle), ctypes.c_int32, _P(ctypes.c_int32)]),
    "epdlb_batch_track_reset": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "epdlb_invert_densities": (ctypes.c_int, [_vp, _dp, ctypes.c_int32, ctypes.c_double, _P(epdlb_cg_info)]),
    "epdlb_cg_stats": (ctypes.c_int, [_vp, _P(epdlb_cg_info), _P(ctypes.c_int64)]),
    "epdlb_lb3_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                        ctypes.c_int32, ctypes.c_int, _vp, _P(_vp)]),
    "epdlb_lb3_set_populations": (ctypes.c_int, [_vp, _dp]),
    "epdlb_lb3_set_equilibrium": (ctypes.c_int, [_vp, _dp, _dp]),
    "epdlb_lb3_set_force": (ctypes.c_int, [_vp, _dp]),
    "epdlb_lb3_set_collision": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                               ctypes.c_double]),
    "epdlb_lb3_step": (ctypes.c_int, [_vp, ctypes.c_int64]),
    "epdlb_lb3_profile": (ctypes.c_int, [_vp, ctypes.c_int32, _dp]),
    "epdlb_lb3_sync": (ctypes.c_int, [_vp]),
    "epdlb_lb3_read_populations": (ctypes.c_int, [_vp, _dp]),
    "epdlb_lb3_read_velocity": (ctypes.c_int, [_vp, _dp, _dp]),
    "epdlb_lb3_destroy": (None, [_vp]),
    "epdlb_epd3_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_int32, ctypes.c_int, _vp, _P(_vp)]),
    "epdlb_epd3_densities": (ctypes.c_int, [_vp, _dp, _dp, _dp, _dp]),
    "epdlb_epd3_time": (ctypes.c_int, [_vp, ctypes.c_int32, _dp]),
    "epdlb_epd3_profile": (ctypes.c_int, [_vp, _dp, _P(ctypes.c_int32)]),
    "epdlb_epd3_destroy": (None, [_vp]),
    "epdlb_last_error": (ctypes.c_char_p, []),
}


def load_library(path=LIB_PATH):
    """Load libepdlb.so (built in-tree by paper_1804_02883_amd.build); raise if missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: run `python -m paper_1804_02883_amd.build` first")
    try:  # bind to the HIP runtime torch already loaded, if any
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(code, fn):
    if code != EPDLB_OK:
        msg = load_library().epdlb_last_error().decode()
        raise EpdlbError(code, fn, msg)


def _ptr(a):
    return a.ctypes.data_as(_dp)


def _f64(a, count):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.size != count:
        raise ValueError(f"expected {count} values, got {a.size}")
    return a



def work_stream(device):
    """The stream a context queues its work on: torch's current stream of
    `device`, or a new torch stream (default priority) when the current one is
    the legacy default stream, whose null handle the library would read as "no
    stream" and answer with a private stream that torch events cannot see.
    Events that time a context's work are recorded on this stream."""
    import torch
    dev = torch.device("cuda", device) if isinstance(device, int) else device
    s = torch.cuda.current_stream(dev)
    if s.cuda_stream == 0:
        s = torch.cuda.Stream(dev)
    return s


def make_params(d=None, **kw):
    """epdlb_params from the library defaults, updated by a dict and keywords."""
    p = epdlb_params()
    _check(load_library().epdlb_params_default(ctypes.byref(p)), "epdlb_params_default")
    for k, v in dict(d or {}, **kw).items():
        if not hasattr(p, k):
            raise KeyError(f"unknown parameter {k}")
        setattr(p, k, v)
    return p


def epdlb_mrt_gammas(eta, eta_B, rho, dx, dt, dim):
    gs, gb = ctypes.c_double(), ctypes.c_double()
    _check(load_library().epdlb_mrt_gammas(eta, eta_B, rho, dx, dt, dim, ctypes.byref(gs), ctypes.byref(gb)),
           "epdlb_mrt_gammas")
    return gs.value, gb.value


def mrt_gammas(eta, eta_B, rho=1.0, dx=1.0 / 3.0, dt=0.002, d=2):
    """(gamma_s, gamma_b) of the multi-relaxation LB from the shear and bulk
    viscosities (epdlb_mrt_gammas, Sec. II viscosity relations)."""
    return epdlb_mrt_gammas(eta, eta_B, rho, dx, dt, d)


# ---- functions with the C ABI's names --------------------------------------------------

def epdlb_params_default():
    return make_params()


def epdlb_validate(p):
    return load_library().epdlb_validate(ctypes.byref(p))


def epdlb_workspace_bytes(p):
    n = ctypes.c_size_t(0)
    _check(load_library().epdlb_workspace_bytes(ctypes.byref(p), ctypes.byref(n)), "epdlb_workspace_bytes")
    return n.value


def epdlb_noise_fill(seed, sigma, nx, ny):
    out = np.empty(3 * nx * ny, dtype=np.float64)
    _check(load_library().epdlb_noise_fill(seed, sigma, nx, ny, _ptr(out)), "epdlb_noise_fill")
    return out.reshape(3, ny, nx)


def epdlb_create(p, device=0, stream=None, workspace=None, workspace_bytes=0):
    h = _vp()
    _check(load_library().epdlb_create(ctypes.byref(p), device, stream, workspace, workspace_bytes,
                                       ctypes.byref(h)), "epdlb_create")
    return h


def epdlb_seed(ctx, seed, sigma):
    _check(load_library().epdlb_seed(ctx, seed, sigma), "epdlb_seed")


def epdlb_set_fields(ctx, omega, n):
    w = _f64(omega, 3 * n)
    _check(load_library().epdlb_set_fields(ctx, _ptr(w)), "epdlb_set_fields")


def epdlb_set_state(ctx, omega, phi, fstar, u, n):
    a, b, c, d = _f64(omega, 3 * n), _f64(phi, 3 * n), _f64(fstar, 9 * n), _f64(u, 2 * n)
    _check(load_library().epdlb_set_state(ctx, _ptr(a), _ptr(b), _ptr(c), _ptr(d)), "epdlb_set_state")


def epdlb_get_state(ctx, shape):
    n = shape[0] * shape[1]
    om, ph, fs, u = np.empty(3 * n), np.empty(3 * n), np.empty(9 * n), np.empty(2 * n)
    _check(load_library().epdlb_get_state(ctx, _ptr(om), _ptr(ph), _ptr(fs), _ptr(u)), "epdlb_get_state")
    return om.reshape((3,) + tuple(shape)), ph.reshape((3,) + tuple(shape)), \
        fs.reshape((9,) + tuple(shape)), u.reshape((2,) + tuple(shape))


def epdlb_device_views(ctx):
    v = epdlb_dev_views()
    _check(load_library().epdlb_device_views(ctx, ctypes.byref(v)), "epdlb_device_views")
    return v


def epdlb_step(ctx, n):
    _check(load_library().epdlb_step(ctx, n), "epdlb_step")


def epdlb_run_stage(ctx, stage):
    _check(load_library().epdlb_run_stage(ctx, stage), "epdlb_run_stage")


def epdlb_sync(ctx):
    _check(load_library().epdlb_sync(ctx), "epdlb_sync")


def _read3(fn, ctx, shape):
    out = np.empty((3,) + shape, dtype=np.float64)
    _check(getattr(load_library(), fn)(ctx, _ptr(out[0]), _ptr(out[1]), _ptr(out[2])), fn)
    return out


def epdlb_read_densities(ctx, shape):
    return _read3("epdlb_read_densities", ctx, shape)


def epdlb_read_fields(ctx, shape):
    return _read3("epdlb_read_fields", ctx, shape)


def epdlb_read_velocity(ctx, shape):
    """Returns (rho, u) with u of shape (2, ny, nx)."""
    out = _read3("epdlb_read_velocity", ctx, shape)
    return out[0], out[1:]


def epdlb_read_populations(ctx, shape):
    out = np.empty((9,) + shape, dtype=np.float64)
    _check(load_library().epdlb_read_populations(ctx, _ptr(out)), "epdlb_read_populations")
    return out


_AUX_PLANES = {EPDLB_AUX_STILDE: 1, EPDLB_AUX_S: 1, EPDLB_AUX_FORCE: 2}


def epdlb_read_aux(ctx, which, shape):
    out = np.empty((_AUX_PLANES[which],) + shape, dtype=np.float64)
    _check(load_library().epdlb_read_aux(ctx, which, _ptr(out)), "epdlb_read_aux")
    return out


def epdlb_write_aux(ctx, which, data, shape):
    a = _f64(data, _AUX_PLANES[which] * shape[0] * shape[1])
    _check(load_library().epdlb_write_aux(ctx, which, _ptr(a)), "epdlb_write_aux")


def epdlb_read_diag(ctx):
    d = epdlb_diag()
    _check(load_library().epdlb_read_diag(ctx, ctypes.byref(d)), "epdlb_read_diag")
    return _diag_dict(d)


def epdlb_observables(ctx, threshold, max_particles, shape=None, replica=None):
    """(dict of sigma, y2p, n_particles, n_wrapping; list of particle dicts in label
    order; labels [ny, nx] int32 or None).  Labels are returned when `shape` is given.
    With `replica`, ctx is a batch and the replica's observables are measured."""
    import numpy as np
    o = epdlb_obs()
    arr = (epdlb_particle * max_particles)() if max_particles > 0 else None
    lab = None
    lab_ptr = None
    if shape is not None:
        lab = np.empty(shape, dtype=np.int32)
        lab_ptr = lab.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    if replica is None:
        _check(load_library().epdlb_observables(ctx, threshold, ctypes.byref(o), arr, max_particles, lab_ptr),
               "epdlb_observables")
    else:
        _check(load_library().epdlb_batch_observables(ctx, replica, threshold, ctypes.byref(o), arr, max_particles,
                                                      lab_ptr), "epdlb_batch_observables")
    parts = []
    for k in range(min(o.n_particles, max_particles)):
        q = arr[k]
        parts.append(_particle_dict(q))
    return dict(sigma=o.sigma, y2p=o.y2p, n_particles=o.n_particles, n_wrapping=o.n_wrapping), parts, lab


def _particle_dict(q):
    return dict(label=q.label, area=q.area, wraps=bool(q.wraps), content=q.content,
                centroid=(q.cx, q.cy), G=(q.gxx, q.gxy, q.gyy), R=q.R, c_rel=q.c_rel)


def epdlb_track_particles(ctx, threshold, max_events, replica=None):
    """(observables dict, list of new particles since the previous call in label order,
    number of new particles).  With `replica`, ctx is a batch."""
    o = epdlb_obs()
    arr = (epdlb_particle * max_events)() if max_events > 0 else None
    n = ctypes.c_int32(0)
    if replica is None:
        _check(load_library().epdlb_track_particles(ctx, threshold, ctypes.byref(o), arr, max_events,
                                                    ctypes.byref(n)), "epdlb_track_particles")
    else:
        _check(load_library().epdlb_batch_track_particles(ctx, replica, threshold, ctypes.byref(o), arr, max_events,
                                                          ctypes.byref(n)), "epdlb_batch_track_particles")
    ev = [_particle_dict(arr[k]) for k in range(min(n.value, max_events))]
    return dict(sigma=o.sigma, y2p=o.y2p, n_particles=o.n_particles, n_wrapping=o.n_wrapping), ev, n.value


def epdlb_track_reset(ctx):
    _check(load_library().epdlb_track_reset(ctx), "epdlb_track_reset")


def epdlb_sigma_delta(ctx_a, ctx_b):
    v = ctypes.c_double(0.0)
    _check(load_library().epdlb_sigma_delta(ctx_a, ctx_b, ctypes.byref(v)), "epdlb_sigma_delta")
    return v.value


def epdlb_sigma_delta_noalloc(ctx_a, ctx_b):
    v = ctypes.c_double(0.0)
    _check(load_library().epdlb_sigma_delta_noalloc(ctx_a, ctx_b, ctypes.byref(v)), "epdlb_sigma_delta_noalloc")
    return v.value


def np_shape(a):
    import numpy as np
    return tuple(np.shape(a))


def _cg_dict(r):
    return dict(iters=r.iters, evals=r.evals, restarts=r.restarts, converged=bool(r.converged),
                resid0=r.resid0, resid=r.resid)


def epdlb_invert_densities(ctx, phi_target, max_iter=1000, tol=1e-8):
    """Replace the context's omega by the potentials reproducing phi_target
    (3 x ny x nx, planes A, B, S), starting from the current omega."""
    import numpy as np
    t = np.ascontiguousarray(phi_target, dtype=np.float64)
    r = epdlb_cg_info()
    _check(load_library().epdlb_invert_densities(ctx, t.ctypes.data_as(_dp), int(max_iter), float(tol),
                                                 ctypes.byref(r)), "epdlb_invert_densities")
    return _cg_dict(r)


def epdlb_cg_stats(ctx):
    """(last inversion, totals dict of inversions, iterations, evals, unconverged)."""
    r = epdlb_cg_info()
    t = (ctypes.c_int64 * 4)()
    _check(load_library().epdlb_cg_stats(ctx, ctypes.byref(r), t), "epdlb_cg_stats")
    return _cg_dict(r), dict(inversions=t[0], iterations=t[1], evals=t[2], unconverged=t[3])


def _diag_dict(d):
    return dict(step=d.step, Q_P=d.Q_P, Q_P_bwd=d.Q_P_bwd, Q_S=d.Q_S, gauge_S=d.gauge_S,
                mean_omega=tuple(d.mean_omega), n_exact=d.n_exact, n_triggered=d.n_triggered,
                nn_err_last=d.nn_err_last, nn_err_max=d.nn_err_max, resid_nn_max=d.resid_nn_max,
                resid_exact=d.resid_exact, nn_err_in_use=d.nn_err_in_use)


def epdlb_autotune(ctx, reps=20, cache_path=None):
    cp = cache_path.encode() if cache_path else None
    _check(load_library().epdlb_autotune(ctx, reps, cp), "epdlb_autotune")


def epdlb_get_shapes(ctx):
    arr = (epdlb_shape * 8)()
    n = ctypes.c_int32(0)
    _check(load_library().epdlb_get_shapes(ctx, arr, 8, ctypes.byref(n)), "epdlb_get_shapes")
    return {arr[i].family.decode(): (arr[i].R, arr[i].nf) for i in range(n.value)}


def epdlb_set_shape(ctx, family, R, nf):
    _check(load_library().epdlb_set_shape(ctx, family.encode(), R, nf), "epdlb_set_shape")


def epdlb_profile_start(ctx, max_launches):
    _check(load_library().epdlb_profile_start(ctx, max_launches), "epdlb_profile_start")


def epdlb_profile_read(ctx):
    """{kernel family: dict(launches, total_ms, min_ms, max_ms, avg_ms)}"""
    cap = 32
    arr = (epdlb_kernel_stat * cap)()
    n = ctypes.c_int32(0)
    _check(load_library().epdlb_profile_read(ctx, arr, cap, ctypes.byref(n)), "epdlb_profile_read")
    out = {}
    for i in range(n.value):
        s = arr[i]
        out[s.name.decode()] = dict(launches=s.launches, total_ms=s.total_ms, min_ms=s.min_ms,
                                    max_ms=s.max_ms, avg_ms=s.total_ms / max(s.launches, 1))
    return out


def epdlb_destroy(ctx):
    load_library().epdlb_destroy(ctx)


def epdlb_last_error():
    return load_library().epdlb_last_error().decode()


# ---- convenience wrapper -----------------------------------------------------------------

class Simulation:
    """One replica on one GPU.  Device memory comes from torch's caching
    allocator and work is queued on `work_stream(device)`."""

    def __init__(self, params, device=0, use_torch=True):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("epdlb needs a ROCm GPU (gfx950); none is visible")
        self.p = params if isinstance(params, epdlb_params) else make_params(params)
        self.shape = (self.p.ny, self.p.nx)
        self.n = self.p.nx * self.p.ny
        self.device = device
        self._ws = None
        stream = None
        ws_ptr, ws_bytes = None, 0
        if use_torch:
            dev = torch.device("cuda", device)
            self.stream = work_stream(dev)
            stream = _vp(self.stream.cuda_stream)
            ws_bytes = epdlb_workspace_bytes(self.p)
            self._ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=dev)
            # the workspace is used on the context's stream: the caching
            # allocator must not hand it out again before that work is done
            self._ws.record_stream(self.stream)
            base = self._ws.data_ptr()
            ws_ptr = _vp((base + 255) & ~255)
        self.ctx = epdlb_create(self.p, device, stream, ws_ptr, ws_bytes)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            epdlb_destroy(self.ctx)
            self.ctx = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def seed(self, seed, sigma):
        epdlb_seed(self.ctx, seed, sigma)

    def set_fields(self, omega):
        epdlb_set_fields(self.ctx, omega, self.n)

    def set_state(self, omega, phi, fstar, u):
        epdlb_set_state(self.ctx, omega, phi, fstar, u, self.n)

    def step(self, n=1):
        epdlb_step(self.ctx, n)

    def run_stage(self, stage):
        epdlb_run_stage(self.ctx, stage)

    def sync(self):
        epdlb_sync(self.ctx)

    def densities(self):
        return epdlb_read_densities(self.ctx, self.shape)

    def fields(self):
        return epdlb_read_fields(self.ctx, self.shape)

    def velocity(self):
        return epdlb_read_velocity(self.ctx, self.shape)

    def populations(self):
        return epdlb_read_populations(self.ctx, self.shape)

    def aux(self, which):
        return epdlb_read_aux(self.ctx, which, self.shape)

    def write_aux(self, which, data):
        epdlb_write_aux(self.ctx, which, data, self.shape)

    def diag(self):
        return epdlb_read_diag(self.ctx)

    def observables(self, threshold=0.5, max_particles=4096, labels=False):
        """sigma, Y_2^P and the particles of the current densities (Sec. III, IV)."""
        return epdlb_observables(self.ctx, threshold, max_particles, self.shape if labels else None)

    def track_particles(self, threshold=0.5, max_events=4096):
        """Observables and the particles nucleated since the previous call (Sec. IV)."""
        return epdlb_track_particles(self.ctx, threshold, max_events)

    def track_reset(self):
        epdlb_track_reset(self.ctx)

    def sigma_delta(self, other):
        """sigma_Delta between this run's and another run's polymer densities (Sec. III)."""
        return epdlb_sigma_delta(self.ctx, other.ctx)

    def invert_densities(self, phi_target, max_iter=1000, tol=1e-8):
        """Potentials reproducing phi_target (App. C), from the current omega; see epdlb.h."""
        if np_shape(phi_target) != (3,) + self.shape:
            raise ValueError(f"phi_target must have shape {(3,) + self.shape}")
        return epdlb_invert_densities(self.ctx, phi_target, max_iter, tol)

    def cg_stats(self):
        return epdlb_cg_stats(self.ctx)

    def autotune(self, reps=20, cache_path=None):
        epdlb_autotune(self.ctx, reps, cache_path)
        return epdlb_get_shapes(self.ctx)

    def shapes(self):
        return epdlb_get_shapes(self.ctx)

    def set_shape(self, family, R, nf):
        epdlb_set_shape(self.ctx, family, R, nf)

    def profile_start(self, max_launches):
        epdlb_profile_start(self.ctx, max_launches)

    def profile_read(self):
        return epdlb_profile_read(self.ctx)

    def surrogate_set_weights(self, w):
        epdlb_surrogate_set_weights(self.ctx, w)

    def get_state(self):
        """(omega, phi, fstar, u) on the host, the layout set_state takes."""
        return epdlb_get_state(self.ctx, self.shape)

    def device_views(self):
        """Zero-copy torch views of the current state (valid until the next step):
        dict of omega [3, ny, nx], phi [3, ny, nx], rho [ny, nx], u [2, ny, nx]."""
        import torch
        if self._ws is None:
            raise RuntimeError("device views need the torch workspace (use_torch=True)")
        v = epdlb_device_views(self.ctx)
        dt = torch.float64 if v.precision == 0 else torch.float32
        es = 8 if v.precision == 0 else 4
        base = self._ws.data_ptr()
        out = {}
        for name, planes in (("omega", 3), ("phi", 3), ("rho", 1), ("u", 2)):
            off = getattr(v, name) - base
            t = self._ws[off:off + planes * v.plane * es].view(dt)
            out[name] = t.view((planes,) + self.shape) if planes > 1 else t.view(self.shape)
        return out


# ---- density surrogate ---------------------------------------------------------------------

def _f32(a, count):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if a.size != count:
        raise ValueError(f"expected {count} values, got {a.size}")
    return a


def epdlb_surrogate_set_weights(ctx, w):
    a = _f32(w, EPDLB_NN_PARAMS)
    _check(load_library().epdlb_surrogate_set_weights(ctx, a.ctypes.data_as(_fp), a.size),
           "epdlb_surrogate_set_weights")


def epdlb_nn_create(nx, ny, capacity, max_batch, device=0, stream=None):
    out = _vp()
    _check(load_library().epdlb_nn_create(nx, ny, capacity, max_batch, device, stream, ctypes.byref(out)),
           "epdlb_nn_create")
    return out


def epdlb_nn_set_weights(nn, w):
    a = _f32(w, EPDLB_NN_PARAMS)
    _check(load_library().epdlb_nn_set_weights(nn, a.ctypes.data_as(_fp), a.size), "epdlb_nn_set_weights")


def epdlb_nn_get_weights(nn):
    a = np.empty(EPDLB_NN_PARAMS, dtype=np.float32)
    _check(load_library().epdlb_nn_get_weights(nn, a.ctypes.data_as(_fp), a.size), "epdlb_nn_get_weights")
    return a


def epdlb_nn_set_pair(nn, slot, omega, phi, f_A, n_contour, n):
    w = _f64(omega, 3 * n)
    ph = _f64(phi, 2 * n)
    _check(load_library().epdlb_nn_set_pair(nn, slot, _ptr(w), _ptr(ph), f_A, n_contour), "epdlb_nn_set_pair")


def epdlb_nn_capture(nn, slot, ctx):
    _check(load_library().epdlb_nn_capture(nn, slot, ctx), "epdlb_nn_capture")


def _slots(slots):
    a = np.ascontiguousarray(slots, dtype=np.int32)
    return a, a.ctypes.data_as(_ip)


def epdlb_nn_evaluate(nn, slots, phi_scale, grad=False):
    a, ap = _slots(slots)
    loss, mx = ctypes.c_double(), ctypes.c_double()
    g = np.empty(EPDLB_NN_PARAMS, dtype=np.float32) if grad else None
    _check(load_library().epdlb_nn_evaluate(nn, ap, a.size, phi_scale, ctypes.byref(loss), ctypes.byref(mx),
                                            g.ctypes.data_as(_fp) if grad else None), "epdlb_nn_evaluate")
    return loss.value, mx.value, g


def epdlb_nn_train_step(nn, slots, phi_scale, lr):
    a, ap = _slots(slots)
    _check(load_library().epdlb_nn_train_step(nn, ap, a.size, phi_scale, lr), "epdlb_nn_train_step")


def epdlb_nn_last_loss(nn):
    loss, mx = ctypes.c_double(), ctypes.c_double()
    _check(load_library().epdlb_nn_last_loss(nn, ctypes.byref(loss), ctypes.byref(mx)), "epdlb_nn_last_loss")
    return loss.value, mx.value


def epdlb_nn_predict(nn, slot, shape):
    out = np.empty((2,) + tuple(shape))
    _check(load_library().epdlb_nn_predict(nn, slot, _ptr(out)), "epdlb_nn_predict")
    return out


def epdlb_nn_destroy(nn):
    load_library().epdlb_nn_destroy(nn)


class Trainer:
    """Device dataset of (potentials -> densities) pairs and the surrogate's
    training kernels; work is queued on `work_stream(device)`."""

    def __init__(self, nx, ny, capacity, max_batch, device=0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("epdlb needs a ROCm GPU (gfx950); none is visible")
        self.shape = (ny, nx)
        self.n = nx * ny
        self.capacity = capacity
        self.stream = work_stream(device)
        self.nn = epdlb_nn_create(nx, ny, capacity, max_batch, device, _vp(self.stream.cuda_stream))

    def close(self):
        if getattr(self, "nn", None) is not None:
            epdlb_nn_destroy(self.nn)
            self.nn = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_weights(self, w):
        epdlb_nn_set_weights(self.nn, w)

    def get_weights(self):
        return epdlb_nn_get_weights(self.nn)

    def set_pair(self, slot, omega, phi_ab, f_A, n_contour):
        epdlb_nn_set_pair(self.nn, slot, omega, phi_ab, f_A, n_contour, self.n)

    def capture(self, slot, sim):
        epdlb_nn_capture(self.nn, slot, sim.ctx)

    def evaluate(self, slots, phi_scale, grad=False):
        return epdlb_nn_evaluate(self.nn, slots, phi_scale, grad)

    def train_step(self, slots, phi_scale, lr):
        epdlb_nn_train_step(self.nn, slots, phi_scale, lr)

    def last_loss(self):
        return epdlb_nn_last_loss(self.nn)

    def predict(self, slot):
        return epdlb_nn_predict(self.nn, slot, self.shape)


# ---- batched replicas ----------------------------------------------------------------------

def epdlb_batch_create(params_list, device=0, stream=None):
    arr = (epdlb_params * len(params_list))(*params_list)
    h = _vp()
    _check(load_library().epdlb_batch_create(arr, len(params_list), device, stream, ctypes.byref(h)),
           "epdlb_batch_create")
    return h


def epdlb_batch_seed(b, seeds, sigma):
    arr = (ctypes.c_uint64 * len(seeds))(*seeds)
    _check(load_library().epdlb_batch_seed(b, arr, sigma), "epdlb_batch_seed")


def epdlb_batch_set_fields(b, replica, omega, n):
    w = _f64(omega, 3 * n)
    _check(load_library().epdlb_batch_set_fields(b, replica, _ptr(w)), "epdlb_batch_set_fields")


def epdlb_batch_step(b, n):
    _check(load_library().epdlb_batch_step(b, n), "epdlb_batch_step")


def epdlb_batch_sync(b):
    _check(load_library().epdlb_batch_sync(b), "epdlb_batch_sync")


def _bread3(fn, b, replica, shape):
    out = np.empty((3,) + shape, dtype=np.float64)
    _check(getattr(load_library(), fn)(b, replica, _ptr(out[0]), _ptr(out[1]), _ptr(out[2])), fn)
    return out


def epdlb_batch_read_densities(b, replica, shape):
    return _bread3("epdlb_batch_read_densities", b, replica, shape)


def epdlb_batch_read_fields(b, replica, shape):
    return _bread3("epdlb_batch_read_fields", b, replica, shape)


def epdlb_batch_read_velocity(b, replica, shape):
    out = _bread3("epdlb_batch_read_velocity", b, replica, shape)
    return out[0], out[1:]


def epdlb_batch_read_diag(b, replica):
    d = epdlb_diag()
    _check(load_library().epdlb_batch_read_diag(b, replica, ctypes.byref(d)), "epdlb_batch_read_diag")
    return _diag_dict(d)


def epdlb_batch_autotune(b, reps=20, cache_path=None):
    cp = cache_path.encode() if cache_path else None
    _check(load_library().epdlb_batch_autotune(b, reps, cp), "epdlb_batch_autotune")


def epdlb_batch_profile_start(b, max_launches):
    _check(load_library().epdlb_batch_profile_start(b, max_launches), "epdlb_batch_profile_start")


def epdlb_batch_profile_read(b):
    cap = 32
    arr = (epdlb_kernel_stat * cap)()
    n = ctypes.c_int32(0)
    _check(load_library().epdlb_batch_profile_read(b, arr, cap, ctypes.byref(n)), "epdlb_batch_profile_read")
    return {arr[i].name.decode(): dict(launches=arr[i].launches, total_ms=arr[i].total_ms,
                                       min_ms=arr[i].min_ms, max_ms=arr[i].max_ms,
                                       avg_ms=arr[i].total_ms / max(arr[i].launches, 1))
            for i in range(n.value)}


def epdlb_batch_info(b):
    g = ctypes.c_int32(0)
    s = ctypes.c_int64(0)
    _check(load_library().epdlb_batch_info(b, ctypes.byref(g), ctypes.byref(s)), "epdlb_batch_info")
    return g.value, s.value


def epdlb_batch_destroy(b):
    load_library().epdlb_batch_destroy(b)


class Batch:
    """Many replicas (uneven grids, own drive, A fraction and seed) advanced
    together on one GPU; work is queued on `work_stream(device)`."""

    def __init__(self, params_list, device=0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("epdlb needs a ROCm GPU (gfx950); none is visible")
        self.params = [p if isinstance(p, epdlb_params) else make_params(p) for p in params_list]
        self.shapes = [(p.ny, p.nx) for p in self.params]
        self.stream = work_stream(device)
        self.b = epdlb_batch_create(self.params, device, _vp(self.stream.cuda_stream))

    def close(self):
        if getattr(self, "b", None) is not None:
            epdlb_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def seed(self, seeds, sigma):
        epdlb_batch_seed(self.b, seeds, sigma)

    def observables(self, replica, threshold=0.5, max_particles=4096, labels=False):
        """sigma, Y_2^P and the particles of one replica (Sec. III, IV)."""
        return epdlb_observables(self.b, threshold, max_particles, self.shapes[replica] if labels else None,
                                 replica=replica)

    def track_particles(self, replica, threshold=0.5, max_events=4096):
        """Observables of one replica and its particles nucleated since its previous call."""
        return epdlb_track_particles(self.b, threshold, max_events, replica=replica)

    def track_reset(self, replica):
        _check(load_library().epdlb_batch_track_reset(self.b, replica), "epdlb_batch_track_reset")

    def set_fields(self, replica, omega):
        ny, nx = self.shapes[replica]
        epdlb_batch_set_fields(self.b, replica, omega, nx * ny)

    def step(self, n=1):
        epdlb_batch_step(self.b, n)

    def sync(self):
        epdlb_batch_sync(self.b)

    def densities(self, replica):
        return epdlb_batch_read_densities(self.b, replica, self.shapes[replica])

    def fields(self, replica):
        return epdlb_batch_read_fields(self.b, replica, self.shapes[replica])

    def velocity(self, replica):
        return epdlb_batch_read_velocity(self.b, replica, self.shapes[replica])

    def diag(self, replica):
        return epdlb_batch_read_diag(self.b, replica)

    def autotune(self, reps=20, cache_path=None):
        epdlb_batch_autotune(self.b, reps, cache_path)

    def info(self):
        return epdlb_batch_info(self.b)

    def profile_start(self, max_launches):
        epdlb_batch_profile_start(self.b, max_launches)

    def profile_read(self):
        return epdlb_batch_profile_read(self.b)


class Fluid3D:
    """Periodic D3Q19 fluid box (epdlb_lb3_* in include/epdlb.h): host arrays
    are FP64 with shape (planes, nz, ny, nx); work is queued on
    `work_stream(device)`."""

    def __init__(self, nx, ny, nz, tau, precision=1, device=0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("epdlb needs a ROCm GPU (gfx950); none is visible")
        self.shape = (nz, ny, nx)
        self.n = nx * ny * nz
        self.stream = work_stream(device)
        out = _vp()
        _check(load_library().epdlb_lb3_create(nx, ny, nz, tau, precision, device, _vp(self.stream.cuda_stream),
                                               ctypes.byref(out)), "epdlb_lb3_create")
        self.ctx = out

    def close(self):
        if getattr(self, "ctx", None) is not None:
            load_library().epdlb_lb3_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_populations(self, f):
        f = _f64(f, 19 * self.n)
        _check(load_library().epdlb_lb3_set_populations(self.ctx, _ptr(f)), "epdlb_lb3_set_populations")

    def set_equilibrium(self, rho=None, u=None):
        r = None if rho is None else _f64(rho, self.n)
        v = None if u is None else _f64(u, 3 * self.n)
        _check(load_library().epdlb_lb3_set_equilibrium(self.ctx, None if r is None else _ptr(r),
                                                        None if v is None else _ptr(v)),
               "epdlb_lb3_set_equilibrium")

    def set_force(self, F=None):
        a = None if F is None else _f64(F, 3 * self.n)
        _check(load_library().epdlb_lb3_set_force(self.ctx, None if a is None else _ptr(a)), "epdlb_lb3_set_force")

    def set_collision(self, mrt, gamma_s=0.0, gamma_b=0.0, gamma_g=0.0):
        """mrt = 0: BGK at tau; 1: the multi-relaxation collision with these factors."""
        _check(load_library().epdlb_lb3_set_collision(self.ctx, mrt, gamma_s, gamma_b, gamma_g),
               "epdlb_lb3_set_collision")

    def step(self, n=1):
        _check(load_library().epdlb_lb3_step(self.ctx, n), "epdlb_lb3_step")

    def profile(self, n):
        ms = np.zeros(n)
        _check(load_library().epdlb_lb3_profile(self.ctx, n, _ptr(ms)), "epdlb_lb3_profile")
        return ms

    def sync(self):
        _check(load_library().epdlb_lb3_sync(self.ctx), "epdlb_lb3_sync")

    def populations(self):
        f = np.empty((19,) + self.shape)
        _check(load_library().epdlb_lb3_read_populations(self.ctx, _ptr(f)), "epdlb_lb3_read_populations")
        return f

    def velocity(self):
        rho = np.empty(self.shape)
        u = np.empty((3,) + self.shape)
        _check(load_library().epdlb_lb3_read_velocity(self.ctx, _ptr(rho), _ptr(u)), "epdlb_lb3_read_velocity")
        return rho, u


class Densities3D:
    """Chain propagators and densities on a periodic 3D grid (epdlb_epd3_* in
    include/epdlb.h); host arrays FP64 with shape (3, nz, ny, nx)."""

    def __init__(self, nx, ny, nz, n_contour, f_A, phi_P, R_G=1.0, dx=1.0 / 3.0, precision=1, device=0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("epdlb needs a ROCm GPU (gfx950); none is visible")
        self.shape = (nz, ny, nx)
        self.n = nx * ny * nz
        self.stream = work_stream(device)
        out = _vp()
        _check(load_library().epdlb_epd3_create(nx, ny, nz, n_contour, f_A, phi_P, R_G, dx, precision, device,
                                                _vp(self.stream.cuda_stream), ctypes.byref(out)),
               "epdlb_epd3_create")
        self.ctx = out

    def close(self):
        if getattr(self, "ctx", None) is not None:
            load_library().epdlb_epd3_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def densities(self, omega):
        """(phi (3, nz, ny, nx), Q_P, Q_S) of the potentials omega."""
        w = _f64(omega, 3 * self.n)
        phi = np.empty((3,) + self.shape)
        qp = ctypes.c_double()
        qs = ctypes.c_double()
        _check(load_library().epdlb_epd3_densities(self.ctx, _ptr(w), _ptr(phi), ctypes.byref(qp), ctypes.byref(qs)),
               "epdlb_epd3_densities")
        return phi, qp.value, qs.value

    def time(self, reps):
        ms = ctypes.c_double()
        _check(load_library().epdlb_epd3_time(self.ctx, reps, ctypes.byref(ms)), "epdlb_epd3_time")
        return ms.value

    def profile(self):
        """(summed kernel ms of the FFT launches of one evaluation, their number)."""
        ms = ctypes.c_double()
        k = ctypes.c_int32()
        _check(load_library().epdlb_epd3_profile(self.ctx, ctypes.byref(ms), ctypes.byref(k)), "epdlb_epd3_profile")
        return ms.value, k.value
