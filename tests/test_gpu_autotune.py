"""The autotuner times its candidates on the live context, and the force-row
candidates include the LB step (fused with the row inverse where the shape
allows, as the step runs it).  Tuning in the middle of a run must leave the
state as it found it: fields, densities, populations and velocity bit for bit,
and no guard word set."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [1, 0])
def test_autotune_keeps_the_state(tmp_path, precision):
    from paper_1804_02883_amd import Simulation
    from seeded_inputs import preset
    p = preset("cfg1", nx=256, ny=128, n_contour=16, precision=precision)
    sim = Simulation(p)
    sim.seed(1234, 0.05)
    sim.step(3)
    sim.sync()
    before = sim.get_state()
    u0 = np.abs(before[3]).max()
    sim.autotune(5, str(tmp_path / "tune.txt"))  # empty cache: every candidate is timed
    after = sim.get_state()
    sim.sync()  # raises if a guard word was left set
    for name, a, b in zip(("omega", "phi", "populations", "u"), before, after):
        assert np.array_equal(a, b), name
    assert u0 > 0.0  # the flow is on, so the LB candidates had a velocity to overwrite
    lines = (tmp_path / "tune.txt").read_text().splitlines()
    assert any(" force_row " in l for l in lines)
    # and the run goes on from the kept state
    sim.step(2)
    sim.sync()
    sim.close()
