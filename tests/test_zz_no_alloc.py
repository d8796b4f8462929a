"""The allocation-free entry point (epdlb_sigma_delta_noalloc) through the C
ABI against the allocating one (epdlb_sigma_delta), on two calls in a row, the
second on a smaller grid, and again on the first grid."""
import pytest

from seeded_inputs import preset

pytestmark = pytest.mark.gpu


def _pair(nx, ny, prec):
    from paper_1804_02883_amd import Simulation
    p = preset("cfg1", nx=nx, ny=ny, n_contour=8, precision=prec)
    a, b = Simulation(p), Simulation(p)
    a.seed(11, 0.05)
    b.seed(12, 0.05)
    a.step(3)
    b.step(3)
    return a, b


def test_sigma_delta_noalloc_matches_the_allocating_call():
    from paper_1804_02883_amd import binding as B
    big = _pair(512, 256, 1)
    small = _pair(64, 32, 0)
    for a, b in (big, small, big):
        ref = B.epdlb_sigma_delta(a.ctx, b.ctx)
        got = B.epdlb_sigma_delta_noalloc(a.ctx, b.ctx)
        print(f"sigma_Delta {a.p.nx}x{a.p.ny}: {ref!r} vs {got!r}", flush=True)
        assert ref > 0 and got == ref
    for s in big + small:
        s.close()


def test_sigma_delta_noalloc_checks_its_arguments():
    from paper_1804_02883_amd import Simulation, binding as B
    a, b = _pair(64, 32, 0)
    c = Simulation(preset("cfg1", nx=32, ny=32, n_contour=8, precision=0))
    c.seed(1, 1e-3)
    with pytest.raises(B.EpdlbError) as e:
        B.epdlb_sigma_delta_noalloc(a.ctx, c.ctx)
    assert e.value.code == B.EPDLB_EINVAL
    for s in (a, b, c):
        s.close()
