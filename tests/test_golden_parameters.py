"""The paper's printed model parameters (tests/golden/paper_parameters.json, each
value with its citation) against the presets, the study's parameter sets, the
library defaults and the viscosity relation."""
import json
import os

from paper_1804_02883_amd import binding as B
from paper_1804_02883_amd.nucleation_study import paper_system
from seeded_inputs.presets import base_params

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.json")))["values"]


def v(key):
    return GOLD[key]["value"]


def test_study_parameter_sets():
    for system, chi_bs in (("droplet", v("chi_BS_droplet")), ("vesicle", v("chi_BS_vesicle"))):
        p = paper_system(system)
        assert p["n_contour"] == v("N") and p["f_A"] == v("q_A") and p["phi_P"] == v("phi_P")
        assert (p["kappa_H"], p["chi_AB"], p["chi_AS"], p["chi_BS"]) == (v("kappa_H"), v("chi_AB"), v("chi_AS"), chi_bs)
        assert p["D_A"] * p["n_contour"] == v("D_AB_times_N_over_D_S") == p["D_B"] * p["n_contour"]


def test_presets_follow_the_paper_units_and_scalings():
    """Grid spacing, time step and D_A,B = D_S/N as printed; kappa_H = 20/N and the
    fixed-chi*N reading give the printed values at the paper's N."""
    p = base_params(64, 64, v("N"), v("q_A"), v("phi_P"), "Q")
    assert p["dx"] == v("dx_over_R_G") and p["dt"] == v("dt_over_tau")
    assert p["D_A"] * v("N") / p["D_S"] == v("D_AB_times_N_over_D_S")
    assert abs(p["kappa_H"] - v("kappa_H")) < 5e-4
    assert abs(p["chi_AB"] - v("chi_AB")) < 1e-12 and abs(p["chi_AS"] - v("chi_AS")) < 1e-12


def test_library_defaults_and_viscosity_relation():
    q = B.make_params()
    assert q.cg_tol == v("N_tr") and abs(q.dx - v("dx_over_R_G")) < 1e-16 and q.dt == v("dt_over_tau")
    gs, gb = B.mrt_gammas(v("eta"), v("eta_B"), 1.0, v("dx_over_R_G"), v("dt_over_tau"))
    # Sec. II: eta = (dt rho cs^2 / 2)(1 + gs)/(1 - gs), eta_B = (dt rho cs^2 / d)(1 + gb)/(1 - gb),
    # cs^2 = dx^2 / (3 dt^2), d = 2
    cs2 = v("dx_over_R_G") ** 2 / (3 * v("dt_over_tau") ** 2)
    assert abs(v("dt_over_tau") * cs2 / 2 * (1 + gs) / (1 - gs) - v("eta")) < 1e-12
    assert abs(v("dt_over_tau") * cs2 / 2 * (1 + gb) / (1 - gb) - v("eta_B")) < 1e-12
