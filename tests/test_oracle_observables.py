"""Pins of the observables oracle (sigma, sigma_Delta, Y_2^P, particles and their
gyration tensors; readings R18-R20 in oracle/observables_oracle.py)."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import observables_oracle as B


def test_sigma_two_valued_field():
    """Half the sites at phibar + a, half at phibar - a: sigma = a; uniform: 0."""
    ny, nx, pb, a = 8, 16, 0.1, 0.03
    phiP = np.full((ny, nx), pb)
    phiP[:, : nx // 2] += a
    phiP[:, nx // 2:] -= a
    phi = np.stack([0.4 * phiP, 0.6 * phiP, 1 - phiP])
    assert abs(B.sigma(phi, pb) - a) < 1e-15
    assert B.sigma(np.stack([np.full((4, 4), 0.05)] * 2 + [np.full((4, 4), 0.9)]), 0.1) < 1e-16
    # a quarter at +3a, the rest at -a (mean phibar): mean |dev| = 1.5 a (the RMS would be sqrt(3) a)
    phiP = np.full((ny, nx), pb - a)
    phiP[:, : nx // 4] = pb + 3 * a
    phi = np.stack([phiP, np.zeros_like(phiP), 1 - phiP])
    assert abs(B.sigma(phi, pb) - 1.5 * a) < 1e-15


def test_sigma_delta():
    rng = np.random.default_rng(2)
    a = rng.random((8, 8))
    assert B.sigma_delta(a, a) == 0.0
    assert abs(B.sigma_delta(a, a + 0.25) - 0.25) < 1e-15
    assert abs(B.sigma_delta(a, -a) - 2 * np.mean(np.abs(a))) < 1e-15


def test_y2p_closed_forms():
    """Uniform: 1.  All polymer on the two rows at +-y0 (same mean): sqrt(ny y0^2 / sum y^2),
    with sum over cell centres y^2 = (ny^3 - ny)/12."""
    ny, nx, pb = 16, 8, 0.1
    assert abs(B.y2p(np.full((ny, nx), pb), pb) - 1.0) < 1e-15
    for j in (0, 3, 7):
        y0 = j + 0.5 - ny / 2
        phiP = np.zeros((ny, nx))
        phiP[j] = phiP[ny - 1 - j] = pb * ny / 2
        expect = np.sqrt(ny * y0 * y0 / ((ny ** 3 - ny) / 12.0))
        assert abs(B.y2p(phiP, pb) - expect) < 1e-14
    # away from the centre -> above one, at the centre -> below one
    edge = np.zeros((ny, nx)); edge[0] = edge[-1] = pb * ny / 2
    mid = np.zeros((ny, nx)); mid[ny // 2 - 1] = mid[ny // 2] = pb * ny / 2
    assert B.y2p(edge, pb) > 1 > B.y2p(mid, pb)


def test_labels_match_scipy_away_from_the_boundary():
    """On fields whose foreground stays off the border the periodic labelling is
    plain 4-connected labelling: the same partition as scipy.ndimage.label."""
    rng = np.random.default_rng(5)
    for trial in range(6):
        ny, nx = 24, 40
        phiP = ndimage.gaussian_filter(rng.random((ny, nx)), 1.2)
        phiP = (phiP - phiP.min()) / (phiP.max() - phiP.min())
        phiP[0, :] = phiP[-1, :] = phiP[:, 0] = phiP[:, -1] = 0.0
        lab = B.label_particles(phiP, 0.5)
        ref, n = ndimage.label(phiP >= 0.5)
        assert n >= 2
        ref_c = np.full(ref.shape, -1, dtype=np.int64)
        for k in range(1, n + 1):
            idx = np.nonzero(ref.ravel() == k)[0]
            ref_c.ravel()[idx] = idx.min()
        assert np.array_equal(lab, ref_c)


def test_periodic_wrap_and_translation():
    """A disk across the corner is one particle; translated to the middle it has the
    same area, content, tensor, R and c_rel."""
    ny, nx, r = 32, 32, 5.3
    yy, xx = np.mgrid[0:ny, 0:nx]
    def disk(cy, cx):
        d2 = ((yy - cy + ny / 2) % ny - ny / 2) ** 2 + ((xx - cx + nx / 2) % nx - nx / 2) ** 2
        return np.where(d2 <= r * r, 0.7 + 0.001 * d2, 0.1)
    a = B.particle_table(disk(0, 0))
    b = B.particle_table(disk(16, 16))
    assert len(a) == len(b) == 1
    for k in ("area", "content", "R", "c_rel"):
        assert abs(a[0][k] - b[0][k]) < 1e-12, k
    assert np.allclose(a[0]["G"], b[0]["G"], atol=1e-12)
    assert not a[0]["wraps"]


def test_checkerboard_band_and_threshold():
    ny, nx = 8, 8
    cb = np.where((np.add.outer(np.arange(ny), np.arange(nx)) % 2) == 0, 0.9, 0.1)
    t = B.particle_table(cb)
    assert len(t) == ny * nx // 2 and all(p["area"] == 1 and p["R"] == 0 and p["c_rel"] == 0 for p in t)
    band = np.full((ny, nx), 0.2)
    band[3:5, :] = 0.8
    t = B.particle_table(band)
    assert len(t) == 1 and t[0]["area"] == 2 * nx and t[0]["wraps"]
    edge = np.full((4, 4), 0.2)
    edge[1, 1] = 0.5  # >= threshold counts
    edge[2, 2] = np.nextafter(0.5, 0)
    assert [p["area"] for p in B.particle_table(edge)] == [1]


@pytest.mark.parametrize("a,b", [(3, 3), (5, 2), (7, 4), (1, 6)])
def test_rectangle_gyration_tensor_exact(a, b):
    """A uniform a x b block: G = diag((a^2 - 1)/12, (b^2 - 1)/12), the variance of
    a uniform discrete distribution; R^2 = trace; c_rel = ((a^2 - b^2)/(a^2 + b^2 - 2))^2."""
    phiP = np.full((16, 16), 0.05)
    phiP[5:5 + b, 4:4 + a] = 0.8
    (p,) = B.particle_table(phiP)
    assert p["area"] == a * b and abs(p["content"] - 0.8 * a * b) < 1e-13
    assert abs(p["G"][0] - (a * a - 1) / 12) < 1e-13 and abs(p["G"][2] - (b * b - 1) / 12) < 1e-13
    assert abs(p["G"][1]) < 1e-13
    assert abs(p["R"] ** 2 - (a * a + b * b - 2) / 12) < 1e-13
    s = a * a + b * b - 2
    expect = ((a * a - b * b) / s) ** 2 if s > 0 else 0.0
    assert abs(p["c_rel"] - expect) < 1e-12


def test_rotation_and_covariance_form():
    """A 90-degree rotation keeps R and c_rel and maps (Gxx, Gxy, Gyy) to (Gyy, -Gxy, Gxx);
    the double sum equals the weighted covariance about the weighted centroid."""
    rng = np.random.default_rng(9)
    n = 20
    blob = ndimage.gaussian_filter(rng.random((n, n)), 1.5)
    blob = (blob - blob.min()) / (blob.max() - blob.min())
    phiP = np.full((32, 32), 0.1)
    phiP[6:6 + n, 6:6 + n] = np.where(blob > 0.55, 0.5 + 0.5 * blob, 0.1)
    t = B.particle_table(phiP)
    big = max(t, key=lambda p: p["area"])
    rot = np.rot90(phiP).copy()
    t2 = B.particle_table(rot)
    big2 = max(t2, key=lambda p: p["area"])
    assert big["area"] == big2["area"]
    assert abs(big["R"] - big2["R"]) < 1e-12 and abs(big["c_rel"] - big2["c_rel"]) < 1e-12
    gxx, gxy, gyy = big["G"]
    hxx, hxy, hyy = big2["G"]
    assert abs(gxx - hyy) < 1e-12 and abs(gyy - hxx) < 1e-12 and abs(gxy + hxy) < 1e-12
    # covariance form on the same sites
    lab = B.label_particles(phiP)
    ys, xs = np.nonzero(lab == big["label"])
    w = phiP[ys, xs]
    mx, my = np.average(xs, weights=w), np.average(ys, weights=w)
    cxx = np.average((xs - mx) ** 2, weights=w)
    cxy = np.average((xs - mx) * (ys - my), weights=w)
    cyy = np.average((ys - my) ** 2, weights=w)
    assert np.allclose(big["G"], (cxx, cxy, cyy), atol=1e-12)


def _disk(ny, nx, cy, cx, r, inside=0.8, outside=0.1):
    yy, xx = np.mgrid[0:ny, 0:nx]
    d2 = ((yy - cy + ny / 2) % ny - ny / 2) ** 2 + ((xx - cx + nx / 2) % nx - nx / 2) ** 2
    return np.where(d2 <= r * r, inside, outside)


def test_nucleation_events_cases():
    """New, persisting, moved, merged and vanished particles between two samples."""
    ny, nx = 32, 48
    a = np.maximum(_disk(ny, nx, 8, 8, 3), _disk(ny, nx, 20, 30, 3))
    # the first sample: every particle is new
    assert [t["label"] for t in B.nucleation_events(None, a)] == [t["label"] for t in B.particle_table(a)]
    assert len(B.nucleation_events(None, a)) == 2
    # unchanged, or shifted by one site (overlapping): nothing new
    assert B.nucleation_events(a, a) == []
    shifted = np.maximum(_disk(ny, nx, 9, 8, 3), _disk(ny, nx, 20, 31, 3))
    assert B.nucleation_events(a, shifted) == []
    # one old particle stays, one vanishes, two appear: the two new ones, with their tables
    b = np.maximum.reduce([_disk(ny, nx, 8, 8, 3), _disk(ny, nx, 26, 4, 2), _disk(ny, nx, 4, 40, 2.5)])
    ev = B.nucleation_events(a, b)
    assert len(ev) == 2
    new = [t for t in B.particle_table(b) if abs(t["centroid"][0] - 8) > 1e-9 or abs(t["centroid"][1] - 8) > 1e-9]
    assert ev == new
    assert {(round(t["centroid"][1]), round(t["centroid"][0])) for t in ev} == {(26, 4), (4, 40)}
    # two old particles merging into one: not new
    c = np.maximum(_disk(ny, nx, 8, 8, 3), _disk(ny, nx, 8, 13, 3))
    pre = np.maximum(_disk(ny, nx, 8, 8, 2), _disk(ny, nx, 8, 14, 2))
    assert len(B.particle_table(pre)) == 2 and len(B.particle_table(c)) == 1
    assert B.nucleation_events(pre, c) == []
    # a particle that jumps by more than its size counts again (the sampling caveat)
    far = np.maximum(_disk(ny, nx, 8, 20, 3), _disk(ny, nx, 20, 30, 3))
    assert len(B.nucleation_events(a, far)) == 1


def test_particle_density():
    assert B.particle_density(10, 64, 32, 1 / 3) == 10 / (64 * 32 / 9)
