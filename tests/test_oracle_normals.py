"""Pins of the oracle's normal estimation (Sec. IV-A: plane fit over the unprojected neighbours in
a radius inversely proportional to the range, oriented towards the observer)."""
import numpy as np
import pytest

import oracle
import synth


@pytest.mark.parametrize("model", ["pinhole", "spherical"])
def test_plane_normals_exact(model):
    """Noise-free one-plane scene: every fitted normal is the plane's (from the ray-caster) and
    faces the sensor.  Coplanar points fit exactly; what is left is the FP32 storage of the depth
    image: a relative rounding of 2^-24 at range d over the smallest window (2 px, a baseline of
    2 d / |fx|) tilts the fit by at most ~2^-24 |fx| / 2, so the bar is 1e-7 |fx| rad."""
    p = synth.make("plane_pair", model=model, noise=False)
    sen = p.sensors[0]
    N, ok, _, _ = oracle.estimate_normals(sen, p.depth[1], tau=0.5 if model == "pinhole" else 1.0)
    ex = p.normals[1].astype(np.float64)
    has = np.linalg.norm(ex, axis=-1) > 0.5
    assert ok[has].mean() > 0.9 and not ok[~has].any()
    chord = np.linalg.norm(N[ok].astype(np.float64) - ex[ok], axis=-1)
    ang = 2.0 * np.arcsin(np.minimum(chord / 2.0, 1.0))
    assert ang.max() < 1e-7 * abs(sen["fx"]), ang.max()
    q = oracle.unproject_image(sen, p.depth[1])
    assert np.all(np.sum(N[ok] * q[ok], -1) < 0)


def test_neighbourhood_radius_scales_with_range():
    """Fronto-parallel constant-depth plane: the neighbour count is the number of integer offsets
    strictly inside the disc of radius clamp(r |fx| / d, 2, 5) px (lattice-point count)."""
    sen = dict(model=0, H=40, W=40, fx=100.0, fy=100.0, cx=19.5, cy=19.5, min_depth=0.1, max_depth=100.0)
    for d, rad in ((10.0, 2.0), (3.0, 100 * 0.1 / 3.0), (1.0, 5.0)):
        D = np.full((40, 40), d, np.float32)
        _, ok, _, n = oracle.estimate_normals(sen, D, radius_m=0.1)
        want = sum(1 for dy in range(-5, 6) for dx in range(-5, 6) if np.hypot(dx, dy) < rad)
        assert n[20, 20] == want, (d, n[20, 20], want)
        assert ok[20, 20]


def _pinhole(H=41, W=41, c=20.0):
    return dict(model=0, H=H, W=W, fx=100.0, fy=100.0, cx=c, cy=c, min_depth=0.1, max_depth=100.0)


def test_sphere_seen_from_its_centre():
    """Camera at the centre of a sphere of radius 5 m: the principal-axis pixel's neighbourhood is
    symmetric under x -> -x, y -> -y and x <-> y, so the optical axis is an eigenvector of its
    covariance, and the curvature makes it the smallest one: the normal is exactly (0, 0, -1).
    Every other normal points back to the centre up to the curvature bias of a 5 px disc."""
    sen = _pinhole()
    v, u = np.mgrid[0:41, 0:41].astype(np.float64)
    ray = np.stack([(u - 20.0) / 100.0, (v - 20.0) / 100.0, np.ones_like(u)], -1)
    D = (5.0 / np.linalg.norm(ray, axis=-1)).astype(np.float32)
    N, ok, w, _ = oracle.estimate_normals(sen, D, radius_m=0.5, tau=0.5)
    assert ok[20, 20] and w[20, 20, 0] < 1e-3 * w[20, 20, 1]
    np.testing.assert_allclose(N[20, 20], [0.0, 0.0, -1.0], atol=1e-7)
    q = oracle.unproject_image(sen, D)
    radial = -q / np.linalg.norm(q, axis=-1, keepdims=True)
    inner = ok.copy()
    inner[:6], inner[-6:], inner[:, :6], inner[:, -6:] = False, False, False, False
    ang = np.arccos(np.clip(np.sum(N[inner].astype(np.float64) * radial[inner], -1), -1, 1))
    assert ang.max() < 0.02, ang.max()


def test_degenerate_windows_have_no_normal():
    """Too few points (an isolated 2 x 2 patch: 4 < 5 neighbours) and collinear points (one valid
    image row: rank-1 covariance, second eigenvalue at rounding level) give no normal."""
    sen = _pinhole()
    D = np.zeros((41, 41), np.float32)
    D[10:12, 10:12] = 3.0
    D[30, :] = 3.0
    N, ok, w, n = oracle.estimate_normals(sen, D)
    assert not ok.any() and not N.any()
    assert n[10, 10] == 4 and n[30, 20] >= 5
    assert w[30, 20, 1] <= 1e-12 * w[30, 20].sum()


def test_depth_edge_splits_the_neighbourhood():
    """Two fronto-parallel planes at 2 m and 4 m meeting at column 20: neighbours across the
    2 m step fail the depth test, so the pixels beside the edge still get exactly (0, 0, -1); with
    the depth test removed (tau = 10 m) the windows that straddle the edge tilt."""
    sen = _pinhole()
    D = np.full((41, 41), 2.0, np.float32)
    D[:, 20:] = 4.0
    N, ok, _, n = oracle.estimate_normals(sen, D, radius_m=0.1)
    assert ok[10:31, 5:36].all()
    np.testing.assert_allclose(N[10:31, 5:36], np.broadcast_to([0, 0, -1.0], (21, 31, 3)), atol=1e-6)
    assert n[20, 19] < n[20, 10]
    N2, ok2, _, _ = oracle.estimate_normals(sen, D, radius_m=0.1, tau=10.0)
    assert ok2[20, 19] and abs(N2[20, 19, 2]) < 0.99
