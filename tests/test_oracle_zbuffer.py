"""Pins of the oracle's z-buffer occlusion variant (occlusion suppression, Sec. IV-C; the z-buffer
mechanism is a reading): a point is dropped when it lies more than tau behind the nearest of the
pair's own warped source points that land in the same target cell.

The pinned scene is closed-form: a pinhole camera sees a plane at 5 m with a square at 2 m in
front of it; the target camera is translated (no rotation), so every source pixel moves along
its row by fx t_x / z and down by -fy t_y / z, and the target depth image holds the plane only
(the square has left).  The plain depth-consistency gate then keeps the background points that
land where the square's points land; the z-buffer drops exactly those."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.filterwarnings("ignore")

SQ_R, SQ_C = (40, 80), (50, 90)          # square rows / columns (half-open)
TX, TY = 0.51, -0.625 * 2.0 / 120.0       # target offset: shifts 12.24 / 30.6 px, 0.25 / 0.625 px


def _scene(zbuffer, tau=0.5):
    base = synth.make("rgbd_small")
    sen = base.sensors[0]
    H, W = sen["H"], sen["W"]
    I = (0.5 + 0.1 * np.sin(np.arange(W) / 7.0)[None, :] + 0.1 * np.cos(np.arange(H) / 5.0)[:, None]).astype(np.float32)
    Ds = np.full((H, W), 5.0, np.float32)
    Ds[SQ_R[0]:SQ_R[1], SQ_C[0]:SQ_C[1]] = 2.0
    Dt = np.full((H, W), 5.0, np.float32)
    N = np.zeros((H, W, 3), np.float32)
    N[..., 2] = -1.0
    eye = np.array([1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0], np.float64)
    Xt = eye.copy()
    Xt[9:] = [TX, TY, 0.0]
    poses = np.stack([eye, Xt])
    prm = dict(base.params, channels=2, occ_tau_pinhole=tau, occlusion_zbuffer=zbuffer)
    prob = synth.Problem("zbuffer_scene", [sen], np.zeros(2, np.int32), poses, poses,
                         np.array([[0, 1]], np.int32), prm)
    prob.intensity, prob.depth, prob.normals = [I, I], [Ds, Dt], [N, N]
    return prob, poses


def _expected_zoccluded(H, W):
    """Background pixels whose cell floor(u - fx t_x / 5) is also the cell of a square pixel
    (floor(u - fx t_x / 2)) on the same row: the rows stay put (fractions 0.25 and 0.625)."""
    fx = 120.0
    m = np.zeros((H, W), bool)
    sq_cells = set(int(np.floor(c - fx * TX / 2.0)) for c in range(*SQ_C))
    for r in range(*SQ_R):
        for c in range(W):
            if SQ_C[0] <= c < SQ_C[1]:
                continue
            x0 = int(np.floor(c - fx * TX / 5.0))
            if 1 <= x0 <= W - 3 and x0 in sq_cells:
                m[r, c] = True
    return m


def test_zbuffer_values_closed_form():
    prob, poses = _scene(1)
    Z = oracle.zbuffer(prob, poses, 0, 1)
    H, W = Z.shape
    sq_cells = [int(np.floor(c - 120.0 * TX / 2.0)) for c in range(*SQ_C)]
    assert np.all(Z[SQ_R[0]:SQ_R[1], sq_cells[0]:sq_cells[-1] + 1] == 2.0)
    # rows without the square: every cell reached by a background pixel holds 5, the others +inf
    reached = sorted(set(int(np.floor(c - 120.0 * TX / 5.0)) for c in range(W)) & set(range(1, W - 2)))
    assert np.all(Z[10, reached] == 5.0)
    assert np.all(np.isinf(np.delete(Z[10], reached)))
    assert np.all(np.isinf(Z[0])) and np.all(np.isinf(Z[H - 2:]))   # outside the evaluated rows


def test_zbuffer_drops_exactly_the_points_behind_the_square():
    prob, poses = _scene(0)
    plain = oracle.eval_pair(prob, poses, 0, 1, pixels=True)
    prob_z, _ = _scene(1)
    zb = oracle.eval_pair(prob_z, poses, 0, 1, pixels=True)
    H, W = plain["status"].shape
    exp = _expected_zoccluded(H, W)
    assert exp.sum() == 40 * 18
    assert np.array_equal(zb["status"] == oracle.ST_ZOCCLUDED, exp)
    # those points pass the plain gate (the target depth shows the plane), nothing else changes
    assert np.all(plain["status"][exp] == oracle.ST_VALID)
    assert np.array_equal(zb["status"][~exp], plain["status"][~exp])
    # the square itself is dropped by the plain gate in both (target depth 5 m, zeta 2 m)
    sq = np.zeros((H, W), bool)
    sq[SQ_R[0]:SQ_R[1], SQ_C[0]:SQ_C[1]] = True
    inside = sq & (plain["status"] != oracle.ST_OUTSIDE)
    assert inside.any() and np.all(zb["status"][inside] == oracle.ST_OCCLUDED)
    assert zb["n_valid"] == plain["n_valid"] - exp.sum()
    assert zb["n_eval"] == plain["n_eval"]


def test_zbuffer_with_unbounded_tau_changes_nothing():
    prob, poses = _scene(1, tau=1e9)
    a = oracle.eval_pair(prob, poses, 0, 1, pixels=True)
    prob0, _ = _scene(0, tau=1e9)
    b = oracle.eval_pair(prob0, poses, 0, 1, pixels=True)
    assert np.array_equal(a["status"], b["status"])
    assert np.array_equal(a["H12"], b["H12"]) and a["F"] == b["F"]


def _generated(name):
    if name == "rgbd_small":
        return synth.make("rgbd_small")
    return synth.make("lidar128", kfs=[0, 1, 2], H=48, W=768).subset([0, 1, 2])


@pytest.mark.parametrize("name", ["rgbd_small", "lidar_mini"])
def test_zbuffer_masks_are_subsets(name):
    """On the generated scenes (perturbed poses), the variant keeps a subset of the plain gate's
    points, and every point it drops has a nearer point of the pair in its cell."""
    p = _generated(name)
    q = synth.Problem(p.name, p.sensors, p.kf_sensor, p.gt_poses, p.init_poses, p.pairs,
                      dict(p.params, occlusion_zbuffer=1))
    q.intensity, q.depth, q.normals = p.intensity, p.depth, p.normals
    for s, t in p.pairs[:6]:
        a = oracle.eval_pair(p, p.init_poses, s, t, pixels=True)
        b = oracle.eval_pair(q, p.init_poses, s, t, pixels=True)
        vb = b["status"] == oracle.ST_VALID
        assert np.all(a["status"][vb] == oracle.ST_VALID)
        dropped = b["status"] == oracle.ST_ZOCCLUDED
        assert np.all(a["status"][dropped] == oracle.ST_VALID)
        if dropped.any():
            Z = oracle.zbuffer(p, p.init_poses, s, t)
            uv = b["uv"][dropped]
            cells = Z[np.floor(uv[:, 1]).astype(int), np.floor(uv[:, 0]).astype(int)]
            assert np.all(np.isfinite(cells))
    print(name, "pairs checked:", min(6, len(p.pairs)))
