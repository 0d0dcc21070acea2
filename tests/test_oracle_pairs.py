"""Pins of the oracle's pair-graph construction (Sec. IV-B: matching pairs from close, similarly
oriented poses with enough validly reprojected points, plus sequential links)."""
import numpy as np

import oracle
import synth


def _posed(p, poses):
    """len(poses) keyframes that all carry keyframe 0's images, at the given poses."""
    n = len(poses)
    q = synth.Problem(p.name, p.sensors, np.zeros(n, np.int32), poses, poses, np.zeros((0, 2), np.int32),
                      dict(p.params))
    q.intensity, q.depth, q.normals = [p.intensity[0]] * n, [p.depth[0]] * n, [p.normals[0]] * n
    return q


def test_pose_thresholds_are_sharp(rgbd_small):
    """Keyframe 0 and copies of its pose rotated by 29 / 31 deg and shifted by 0.99 / 1.01 m: with
    the ratio test off, exactly the pairs inside both thresholds are kept (both directions)."""
    p = rgbd_small
    X0 = p.gt_poses[0]
    R0 = X0[:9].reshape(3, 3)
    axis = np.array([0.3, -0.5, 0.8])
    poses = [X0]
    for deg, shift in ((29.0, 0.0), (31.0, 0.0), (0.0, 0.99), (0.0, 1.01)):
        R = R0 @ synth.rot_axis_angle(axis, np.radians(deg))
        t = X0[9:] + shift * np.array([0.6, 0.8, 0.0])
        poses.append(np.concatenate([R.reshape(-1), t]))
    poses = np.array(poses)
    q = _posed(p, poses)
    pairs, _ = oracle.build_pairs(q, poses, min_ratio=0.0, sequential=False)
    got = set(map(tuple, pairs.tolist()))
    # pose 1 (29 deg) and 3 (0.99 m) are close to 0, 2 (31 deg) and 4 (1.01 m) are not; 1-2 differ by
    # 2 deg, 1-3 by 29 deg and 0.99 m, 3-4 by 0.02 m: kept; every other pair exceeds a threshold
    want = {(0, 1), (1, 0), (0, 3), (3, 0), (1, 2), (2, 1), (1, 3), (3, 1), (3, 4), (4, 3)}
    assert got == want, got


def test_ratio_threshold_and_sequential_links(rgbd_small):
    """Same pose: every pixel reprojects onto itself, valid except at the image border and next to
    depth edges (ratio 0.83 here, kept at 1/3); a keyframe turned away by 180 deg sees none of it
    (ratio 0, dropped) unless the pair is sequential."""
    p = rgbd_small
    X0 = p.gt_poses[0]
    R0 = X0[:9].reshape(3, 3)
    away = np.concatenate([(R0 @ synth.rot_axis_angle(np.array([0.0, 1.0, 0.0]), np.pi)).reshape(-1), X0[9:]])
    poses = np.array([X0, X0, away])
    q = _posed(p, poses)
    pairs, ratios = oracle.build_pairs(q, poses, max_angle=np.pi + 0.1, max_dist=10.0, sequential=False)
    assert ratios[(0, 1)] > 0.75 and ratios[(0, 2)] == 0.0
    assert set(map(tuple, pairs.tolist())) == {(0, 1), (1, 0)}
    pairs, _ = oracle.build_pairs(q, poses, max_angle=np.pi + 0.1, max_dist=10.0, sequential=True)
    assert set(map(tuple, pairs.tolist())) == {(0, 1), (1, 0), (1, 2), (2, 1)}
    pairs, _ = oracle.build_pairs(q, poses, max_angle=0.0, max_dist=0.0, sequential=True)
    assert set(map(tuple, pairs.tolist())) == {(0, 1), (1, 0), (1, 2), (2, 1)}
