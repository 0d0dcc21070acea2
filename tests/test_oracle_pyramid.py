"""Pins of the oracle's image pyramid (Sec. IV-A: multi-resolution copies of every keyframe, each
level half the resolution of the one below; Sec. IV-C: coarse-to-fine optimisation).

The level intrinsics are pinned against the ray-caster rendering the same scene directly at the
coarse resolution; the 2x2 reduction against closed forms; the schedule against the single-level
optimiser from the same start."""
import copy

import numpy as np
import pytest

import oracle
import synth


def _direct_render(p, sensor, k):
    q = copy.copy(p)
    q.sensors = [sensor]
    q.intensity, q.depth, q.normals = [], [], []
    synth.render(q, kfs=[k], noise=False)
    return q.intensity[k], q.depth[k], q.normals[k]


@pytest.mark.parametrize("cfg,kw,k,tol", [("rgbd_small", {}, 0, 1e-4),
                                          ("plane_pair", {"model": "spherical"}, 1, 2e-4)])
def test_level_intrinsics_match_a_direct_render(cfg, kw, k, tol):
    """Downsampled depth of a noise-free render equals the scene rendered directly with the level
    intrinsics (median relative difference; an intrinsics offset of a quarter texel gives ~1e-3)."""
    p = synth.make(cfg, noise=False, **kw)
    sen = p.sensors[0]
    tau = 0.5 if sen["model"] == 0 else 1.0
    I2, D2, N2 = oracle.downsample_keyframe(p.intensity[k], p.depth[k], p.normals[k], sen, tau)
    ls = oracle.level_sensor(sen)
    assert (ls["H"], ls["W"]) == D2.shape
    Id, Dd, Nd = _direct_render(p, ls, k)
    m = (D2 > 0) & (Dd > 0)
    assert m.mean() > 0.05
    rel = np.abs(D2[m] - Dd[m]) / Dd[m]
    assert np.median(rel) < tol, np.median(rel)
    # the wrong centre convention (cx / 2) is visibly off on the same data
    bad = dict(ls, cx=sen["cx"] / 2, cy=sen["cy"] / 2)
    _, Db, _ = _direct_render(p, bad, k)
    mb = (D2 > 0) & (Db > 0)
    assert np.median(np.abs(D2[mb] - Db[mb]) / Db[mb]) > 10 * tol


def test_downsample_closed_forms():
    """Dyadic ramps stay exact: the block mean of a*col + b*row + c is the ramp at the block
    centre (2j + 1/2, 2i + 1/2); normals come out unit length; the odd last row/column is dropped."""
    H, W = 9, 12
    r, c = np.mgrid[0:H, 0:W].astype(np.float64)
    I = (0.25 * c + 0.125 * r + 0.5).astype(np.float32)
    D = (2.0 + 0.0625 * c - 0.03125 * r).astype(np.float32)
    N = np.zeros((H, W, 3), np.float32)
    N[..., 0], N[..., 2] = 0.6, 0.8
    N[1::2, :, 0] = 0.0
    N[1::2, :, 2] = 1.0
    sen = dict(model=0, H=H, W=W, fx=10.0, fy=10.0, cx=6.0, cy=4.0, min_depth=0.1, max_depth=10.0)
    I2, D2, N2 = oracle.downsample_keyframe(I, D, N, sen, tau=0.5)
    assert I2.shape == (4, 6)
    i, j = np.mgrid[0:4, 0:6].astype(np.float64)
    np.testing.assert_array_equal(I2, (0.25 * (2 * j + 0.5) + 0.125 * (2 * i + 0.5) + 0.5).astype(np.float32))
    np.testing.assert_array_equal(D2, (2.0 + 0.0625 * (2 * j + 0.5) - 0.03125 * (2 * i + 0.5)).astype(np.float32))
    np.testing.assert_allclose(np.linalg.norm(N2.astype(np.float64), axis=-1), 1.0, atol=1e-7)
    mean = np.array([0.3, 0.0, 0.9])
    np.testing.assert_allclose(N2[0, 0], mean / np.linalg.norm(mean), atol=1e-7)


def test_downsample_validity_rules():
    """A block is valid only if all four depths are valid and within tau of each other; invalid
    texels carry no intensity or normal."""
    D = np.full((4, 4), 3.0, np.float32)
    D[0, 0] = 0.0                   # block (0,0): one missing depth
    D[0, 2] = 3.5                   # block (0,1): spread exactly tau
    D[2, 0] = 3.6                   # block (1,0): spread above tau
    D[3, 3] = 50.0                  # block (1,1): outside the depth interval
    I = np.ones((4, 4), np.float32)
    N = np.zeros((4, 4, 3), np.float32)
    N[..., 2] = 1.0
    sen = dict(model=0, H=4, W=4, fx=10.0, fy=10.0, cx=2.0, cy=2.0, min_depth=0.1, max_depth=20.0)
    I2, D2, N2 = oracle.downsample_keyframe(I, D, N, sen, tau=0.5)
    assert D2[0, 0] == 0 and I2[0, 0] == 0 and not N2[0, 0].any()
    assert D2[0, 1] == np.float32(3.125) and I2[0, 1] == 1 and N2[0, 1, 2] == 1
    assert D2[1, 0] == 0 and D2[1, 1] == 0


def test_coarse_to_fine_widens_the_basin():
    """From 0.1 m / 4 deg on the 160x120 set, 17 single-level LM iterations stall while the
    three-level schedule (10 / 5 / 2 iterations, coarse first) reaches the noise floor."""
    p = synth.make("rgbd_small")
    init = synth._perturb(p.gt_poses, np.random.default_rng(7), 0.1, 4.0)
    X1, _ = oracle.optimize(p, init, iters=17, lm=True)
    X2, log = oracle.optimize_coarse_to_fine(p, init, 3, iters=(2, 5, 10), rel_tol=1e-3)
    assert [r["level"] for r in log] == sorted((r["level"] for r in log), reverse=True)
    assert oracle.ate_rmse(X1, p.gt_poses) > 0.02
    assert oracle.ate_rmse(X2, p.gt_poses) < 2e-3
