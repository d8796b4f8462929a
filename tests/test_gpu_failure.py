"""Failure detection through the C ABI: a non-finite value injected with
epdlb_set_state surfaces as EPDLB_ENONFINITE at the next synchronisation, the
flow guard of the LB step (epdlb_params.mach_max; the lattice speed of sound
of Sec. II) as EPDLB_EUNSTABLE, and replacing the state clears both.  The
conditions are set from the host: every kernel runs to its normal end."""
import numpy as np
import pytest

from oracle import epdlb_oracle as O
from seeded_inputs import initial_omega, preset

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def _state(p, ux=0.0):
    ny, nx = p["ny"], p["nx"]
    w = initial_omega(nx, ny, 1001, 1e-3)
    phi = O.densities(w, p)["phi"]
    u = np.zeros((2, ny, nx))
    u[0] = ux
    f = O.lb_equilibrium(np.ones((ny, nx)), u)
    return w, phi, f, u


def _expect(sim, code):
    from paper_1804_02883_amd import EpdlbError
    with pytest.raises(EpdlbError) as e:
        sim.sync()
    assert e.value.code == code, str(e.value)
    return str(e.value)


@pytest.mark.parametrize("prec", [0, 1])
def test_nan_in_the_potentials_is_reported(prec):
    from paper_1804_02883_amd import Simulation, binding as B
    say(f"[failure] NaN in omega_A, 32x32 prec={prec}")
    p = preset("cfg1", precision=prec)
    w, phi, f, u = _state(p)
    w[0, 5, 7] = np.nan
    sim = Simulation(p)
    sim.set_state(w, phi, f, u)
    sim.step(1)
    _expect(sim, B.EPDLB_ENONFINITE)
    sim.seed(1001, 1e-3)  # a new state clears the report
    sim.step(2)
    sim.sync()
    sim.close()


@pytest.mark.parametrize("mrt", [0, 1])
def test_nan_in_the_populations_is_reported(mrt):
    from paper_1804_02883_amd import Simulation, mrt_gammas, binding as B
    say(f"[failure] NaN population, mrt={mrt}")
    extra = {}
    if mrt:
        gs, gb = mrt_gammas(1.0, 1.0)
        extra = dict(lb_mrt=1, lb_gamma_s=gs, lb_gamma_b=gb)
    p = preset("cfg1", **extra)
    w, phi, f, u = _state(p)
    f[3, 10, 20] = np.inf
    sim = Simulation(p)
    sim.set_state(w, phi, f, u)
    sim.step(1)
    msg = _expect(sim, B.EPDLB_ENONFINITE)
    assert "LB" in msg
    sim.close()


def test_flow_speed_guard():
    """A uniform flow of 0.4 lattice units is Mach 0.69: above the default
    guard of 0.5, below a guard of 0.8."""
    from paper_1804_02883_amd import Simulation, binding as B
    say("[failure] Mach guard")
    p = preset("cfg1", couple_lb=0, init_flow=0)
    state = _state(p, ux=0.4)
    sim = Simulation(p)
    sim.set_state(*state)
    sim.step(1)
    msg = _expect(sim, B.EPDLB_EUNSTABLE)
    assert "speed" in msg
    sim.close()
    sim = Simulation(dict(p, mach_max=0.8))
    sim.set_state(*state)
    sim.step(1)
    sim.sync()
    sim.close()


def test_negative_population_guard():
    """At |u| = 0.9 the rest population of the equilibrium, (4/9)(1 - 1.5 u^2),
    is negative; with the speed test off (mach_max = 0) that is what trips."""
    from paper_1804_02883_amd import Simulation, binding as B
    say("[failure] negative population")
    p = preset("cfg1", couple_lb=0, init_flow=0, mach_max=0.0)
    sim = Simulation(p)
    sim.set_state(*_state(p, ux=0.9))
    sim.step(1)
    msg = _expect(sim, B.EPDLB_EUNSTABLE)
    assert "negative" in msg
    sim.set_state(*_state(p, ux=0.0))  # a new state clears the flags
    sim.step(1)
    sim.sync()
    sim.close()


def test_batch_reports_the_replica():
    """A NaN in one replica's potentials is refused when it is set (the field
    means turn non-finite), naming the replica's group position."""
    from paper_1804_02883_amd import Batch, binding as B, EpdlbError
    say("[failure] batch replica NaN")
    p = preset("cfg1")
    b = Batch([p, p])
    b.seed([1, 2], 1e-3)
    w = initial_omega(32, 32, 3, 1e-3)
    w[2, 0, 0] = np.nan
    with pytest.raises(EpdlbError) as e:
        b.set_fields(1, w)
        b.step(1)
        b.sync()
    assert e.value.code == B.EPDLB_ENONFINITE and "replica 1" in str(e.value)
    b.close()
