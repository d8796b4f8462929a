"""Host-side checks of the C-ABI library (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1804_02883_amd import binding as B
from seeded_inputs import initial_omega, preset

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "epdlb.h")


def declared_functions():
    text = "".join(open(os.path.join(ROOT, "include", f)).read()
                   for f in sorted(os.listdir(os.path.join(ROOT, "include"))) if f.endswith(".h"))
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(epdlb_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = B.load_library()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(B.SIGNATURES), set(names) ^ set(B.SIGNATURES)


def test_params_struct_matches_header_order():
    text = open(HEADER).read()
    body = text[text.index("typedef struct {\n  int32_t abi_version"):]
    body = body[:body.index("} epdlb_params;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl or decl.startswith("typedef"):
            decl = decl.split("{")[-1].strip()
        if not decl:
            continue
        names = decl.split(None, 1)[1]
        fields += [x.strip() for x in names.split(",")]
    assert fields == [f[0] for f in B.epdlb_params._fields_]


def test_defaults_and_validation():
    p = B.make_params()
    assert p.abi_version == 1 and p.nx == 32 and p.n_contour == 16
    assert abs(p.dx - 1 / 3) < 1e-16 and p.dt == 0.002 and p.D_A == 1 / 16
    assert B.epdlb_validate(p) == 0
    assert (p.density_mode, p.fallback_every, p.check_every, p.resid_tol, p.err_tol) == (0, 50, 10, 1e-3, 1e-3)
    assert B.epdlb_validate(B.make_params(density_mode=1)) == 0
    assert (p.lb_mrt, p.lb_gamma_s, p.lb_gamma_b, p.lb_gamma_g) == (0, 0.0, 0.0, 0.0)
    gs, gb = B.mrt_gammas(1.0, 1.0)  # the paper's eta = eta_B at its dx, dt
    assert abs(gs + 0.8050541516245486) < 1e-15 and gs == gb
    assert B.epdlb_validate(B.make_params(lb_mrt=1, lb_gamma_s=gs, lb_gamma_b=gb, lb_gamma_g=0.5)) == 0
    assert (p.cg_invert, p.cg_max_iter, p.cg_tol, p.cg_precond) == (0, 1000, 1e-8, 0)
    assert p.mach_max == 0.5 and B.epdlb_validate(B.make_params(mach_max=0.0)) == 0
    assert B.epdlb_validate(B.make_params(cg_invert=1)) == 0
    assert B.epdlb_validate(B.make_params(cg_invert=1, precision=1, cg_tol=1e-6)) == 0
    for bad in [dict(nx=48), dict(nx=16), dict(ny=8), dict(n_contour=1), dict(f_A=1.0),
                dict(phi_P=0.0), dict(lb_tau=0.5), dict(precision=2), dict(abi_version=7),
                dict(g=float("nan")), dict(density_mode=2), dict(density_mode=1, fallback_every=0),
                dict(density_mode=1, check_every=0), dict(density_mode=1, resid_tol=0.0),
                dict(density_mode=1, err_tol=-1.0), dict(lb_mrt=2), dict(lb_mrt=1, lb_gamma_s=1.0),
                dict(lb_mrt=1, lb_gamma_b=-1.0), dict(lb_mrt=1, lb_gamma_g=float("nan")),
                dict(cg_invert=2), dict(cg_invert=1, density_mode=1), dict(cg_invert=1, cg_tol=0.0),
                dict(cg_invert=1, cg_max_iter=-1), dict(cg_invert=1, cg_tol=float("inf")),
                dict(cg_invert=1, precision=1), dict(cg_precond=2), dict(mach_max=-0.1),
                dict(mach_max=float("nan"))]:
        q = B.make_params(**bad)
        assert B.epdlb_validate(q) == B.EPDLB_EINVAL, bad
        assert B.epdlb_last_error() != ""


def test_mrt_gammas_from_the_library_match_the_oracle():
    """The viscosity relations of Sec. II are computed in the library
    (epdlb_mrt_gammas); they agree with the pinned oracle relation in two and
    three dimensions, and bad arguments are refused."""
    from oracle import epdlb_oracle as O
    for d in (2, 3):
        for eta, eta_B, rho, dx, dt in ((1.0, 1.0, 1.0, 1 / 3, 0.002), (0.7, 2.5, 1.3, 0.25, 0.004)):
            got = B.epdlb_mrt_gammas(eta, eta_B, rho, dx, dt, d)
            ref = O.mrt_gammas(eta, eta_B, rho, dx, dt, d=d)
            assert max(abs(got[0] - ref[0]), abs(got[1] - ref[1])) < 1e-15, (d, eta, eta_B)
    for bad in [(0.0, 1.0, 1.0, 0.3, 0.002, 2), (1.0, -1.0, 1.0, 0.3, 0.002, 2), (1.0, 1.0, 1.0, 0.3, 0.0, 2),
                (1.0, 1.0, float("nan"), 0.3, 0.002, 2), (1.0, 1.0, 1.0, 0.3, 0.002, 4)]:
        with pytest.raises(B.EpdlbError) as e:
            B.epdlb_mrt_gammas(*bad)
        assert e.value.code == B.EPDLB_EINVAL


def test_workspace_bytes_scale():
    p32 = B.make_params(preset("cfg3"))
    p64 = B.make_params(preset("cfg3"), precision=0)
    b32, b64 = B.epdlb_workspace_bytes(p32), B.epdlb_workspace_bytes(p64)
    n = 1024 * 512
    N = 64
    planes = 2 * N + 40  # omega 6, phi 3, S~ 1, S 1, q 2N, tmp 2, spec 2, F 2, f* 18, rho 1, u 2, E 2
    assert planes * n * 4 <= b32 < planes * n * 4 + (1 << 22)
    assert abs(b64 - 2 * b32) < (1 << 22)
    # surrogate mode adds two 64-channel bf16 activations, the network's
    # densities (2 planes), the S correction (1 plane), 18 FP32 output-tap
    # planes, weights
    bs = B.epdlb_workspace_bytes(B.make_params(preset("cfg3"), density_mode=1))
    extra = n * (2 * 64 * 2 + 3 * 4 + 18 * 4)
    assert extra <= bs - b32 < extra + (1 << 20)


def test_noise_matches_seeded_inputs():
    out = B.epdlb_noise_fill(1001, 1e-3, 32, 16)
    ref = initial_omega(32, 16, 1001, 1e-3)
    assert np.max(np.abs(out - ref)) <= 1e-18
    assert out.shape == (3, 16, 32)


def test_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    p = B.make_params()
    with pytest.raises(B.EpdlbError) as e:
        B.epdlb_create(p)
    assert e.value.code in (B.EPDLB_ENODEV, B.EPDLB_EHIP)


def test_trainer_create_rejects_bad_sizes_before_device_calls():
    # argument checks come before any HIP call, so they hold without a GPU
    for nx, ny, cap, mb in [(48, 32, 8, 4), (32, 8, 8, 4), (32, 32, 8, 9), (32, 32, 100, 65), (32, 32, 8, 0)]:
        with pytest.raises(B.EpdlbError) as e:
            B.epdlb_nn_create(nx, ny, cap, mb)
        assert e.value.code == B.EPDLB_EINVAL, (nx, ny, cap, mb)


def test_batch_rejects_mixed_collision_models_before_device_calls():
    # replicas of one batch share the model: a BGK and a multi-relaxation replica
    # (or two different gamma sets) are refused before any HIP call
    a = B.make_params(nx=64, ny=64)
    m = B.make_params(nx=64, ny=64, lb_mrt=1, lb_gamma_s=-0.5, lb_gamma_b=-0.5)
    m2 = B.make_params(nx=64, ny=64, lb_mrt=1, lb_gamma_s=-0.5, lb_gamma_b=0.1)
    for pair in ([a, m], [m, m2]):
        with pytest.raises(B.EpdlbError) as e:
            B.epdlb_batch_create(pair)
        assert e.value.code == B.EPDLB_EINVAL


def test_inversion_arguments_checked_before_device_calls():
    # a batch cannot run the host-driven inversion; a NULL context is refused
    with pytest.raises(B.EpdlbError) as e:
        B.epdlb_batch_create([B.make_params(nx=64, ny=64, cg_invert=1)] * 2)
    assert e.value.code == B.EPDLB_EINVAL
    import numpy as np
    with pytest.raises(B.EpdlbError) as e:
        B.epdlb_invert_densities(None, np.ones((3, 32, 32)))
    assert e.value.code == B.EPDLB_EINVAL
    with pytest.raises(B.EpdlbError) as e:
        B.epdlb_cg_stats(None)
    assert e.value.code == B.EPDLB_EINVAL
