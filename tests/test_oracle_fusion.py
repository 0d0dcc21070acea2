"""Pins of the oracle's shared rig poses and of the fusion schedules (coupled / consecutive
LiDAR + RGB-D refinement of one rig frame aligned to a copy of itself)."""
import copy

import numpy as np
import pytest

import oracle
import synth

LIDAR = np.array([(0, 2), (2, 0)], np.int32)
CAMERA = np.array([(1, 3), (3, 1)], np.int32)


@pytest.fixture(scope="module")
def rig():
    return synth.make("rig_pair")


def _ungrouped(p):
    q = copy.copy(p)
    q.pose_of = None
    return q


def _G(p):
    """Keyframe tangents from pose-variable tangents: 6N x 6V, identity blocks at (k, pose_of[k])."""
    M = np.zeros((p.n, p.n_poses))
    M[np.arange(p.n), p.pose_of] = 1.0
    return np.kron(M, np.eye(6))


def _err(X):
    dt = np.linalg.norm(X[1, 9:] - X[0, 9:])
    c = (np.trace(X[0, :9].reshape(3, 3).T @ X[1, :9].reshape(3, 3)) - 1.0) / 2.0
    return dt, float(np.arccos(np.clip(c, -1.0, 1.0)))


def test_shared_poses_follow_the_chain_rule(rig):
    """Keyframes of one rig frame share its pose, X_kf = X_var: the grouped system is G^T H G,
    G^T b of the per-keyframe system at the expanded poses (checked by matrix algebra, not by the
    assembly's own block additions)."""
    G = _G(rig)
    ev = oracle.evaluate(rig, rig.init_poses)
    evf = oracle.evaluate(_ungrouped(rig), rig.kf_poses(rig.init_poses))
    assert ev["F"] == evf["F"]
    scale = np.abs(evf["H"]).max()
    assert np.abs(ev["H"] - G.T @ evf["H"] @ G).max() <= 1e-13 * scale
    assert np.abs(ev["b"] - G.T @ evf["b"]).max() <= 1e-13 * np.abs(evf["b"]).max()


def test_pair_inside_one_frame_has_no_gradient(rig):
    """LiDAR -> camera of the same frame: the residuals do not depend on the frame's pose, so the
    source and target Jacobians cancel exactly (J_s + J_t = 0): the grouped blocks vanish to
    rounding while each keyframe's blocks are large."""
    pr = np.array([(0, 1)], np.int32)
    ev = oracle.evaluate(rig, rig.init_poses, pairs=pr)
    evf = oracle.evaluate(_ungrouped(rig), rig.kf_poses(rig.init_poses), pairs=pr)
    assert ev["n_valid"] > 1000
    assert np.abs(ev["H"]).max() <= 1e-12 * np.abs(evf["H"]).max()
    assert np.abs(ev["b"]).max() <= 1e-12 * np.abs(evf["b"]).max()


def test_loss_gradient_with_shared_poses(rig):
    """F of the grouped problem at delta equals F of the per-keyframe problem at G delta, so its
    gradient is G^T times the per-keyframe gradient."""
    rng = np.random.default_rng(3)
    d = 1e-3 * rng.normal(size=(rig.n_poses, 6))
    d[0] = 0.0
    a = oracle.loss_and_grad(rig, rig.init_poses, d)
    q = _ungrouped(rig)
    b = oracle.loss_and_grad(q, rig.kf_poses(rig.init_poses), (_G(rig) @ d.reshape(-1)).reshape(q.n, 6))
    assert a["F"] == b["F"]
    ga, gb = a["g_delta"].reshape(-1), _G(rig).T @ b["g_delta"].reshape(-1)
    assert np.abs(ga - gb).max() <= 1e-12 * np.abs(gb).max()


def test_self_alignment_schedules(rig):
    """Aligning a frame to a copy of itself has its optimum at the identity (every residual is
    exactly zero there).  From 0.1 m / 3 deg, LiDAR alone and the consecutive schedule (LiDAR,
    then RGB-D from its result) reach it."""
    assert _err(rig.init_poses)[0] > 0.09
    X, _ = oracle.optimize(rig, rig.init_poses, iters=30, lm=True, pairs=LIDAR)
    assert max(_err(X)) < 1e-6, _err(X)
    X, _ = oracle.optimize(rig, X, iters=10, lm=True, pairs=CAMERA)
    assert max(_err(X)) < 1e-6, _err(X)
