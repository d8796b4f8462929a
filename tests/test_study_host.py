"""Host arithmetic of the study drivers (no GPU)."""
from paper_1804_02883_amd.nucleation_study import channel_offset


def test_channel_offset():
    ny, dx = 64, 1 / 3
    # cell-centre coordinate y + 1/2; channel centres at ny/4 and 3 ny/4
    assert channel_offset(15.5, ny, dx) == 0.0
    assert channel_offset(47.5, ny, dx) == 0.0
    assert abs(channel_offset(0.0 - 0.5, ny, dx) + 16 * dx) < 1e-15
    assert abs(channel_offset(31.0, ny, dx) - 15.5 * dx) < 1e-15
    assert abs(channel_offset(32.0, ny, dx) + 15.5 * dx) < 1e-15
