"""Shared rig poses on the GPU (pba_set_pose_groups) against the oracle, and the fusion
schedules on the self-aligned rig frame."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pba():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2303_16878_amd as pba
    pba.load_library()
    return pba


@pytest.fixture(scope="module")
def rig():
    return synth.make("rig_pair")


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _G(n, pose_of):
    M = np.zeros((n, int(np.max(pose_of)) + 1))
    M[np.arange(n), pose_of] = 1.0
    return np.kron(M, np.eye(6))


@pytest.mark.parametrize("precision", ["F32", "F64"])
def test_grouped_system(rig, pba, precision):
    """Two rig frames (four keyframes; LiDAR and camera pairs plus within-frame cross-sensor pairs,
    whose Jacobians cancel): the grouped system equals G^T H G, G^T b of the same context's
    per-keyframe system at the expanded poses (same kernels and masks: only the assembly onto
    pose variables differs), and F and the valid count agree with the oracle's grouped evaluation."""
    pairs = np.array([(0, 2), (2, 0), (1, 3), (3, 1), (0, 1), (3, 2)], np.int32)
    prob = synth.Problem(rig.name, rig.sensors, rig.kf_sensor, rig.gt_poses, rig.init_poses, pairs, dict(rig.params),
                         rig.intensity, rig.depth, rig.normals, rig.scene, rig.pose_of)
    ref = oracle.evaluate(prob, prob.init_poses)
    prec = pba.PBA_F32 if precision == "F32" else pba.PBA_F64
    with pba.context_for_problem(prob, precision=prec) as ctx:
        assert ctx.n_poses == 2
        evg = ctx.evaluate(want_system=True)
        ctx.set_pose_groups(None)
        ctx.set_poses(prob.kf_poses(prob.init_poses))
        evf = ctx.evaluate(want_system=True)
    G = _G(prob.n, prob.pose_of)
    Hx, bx = G.T @ evf["H"] @ G, G.T @ evf["b"]
    dH = np.abs(evg["H"] - Hx).max() / np.abs(Hx).max()
    db = np.abs(evg["b"] - bx).max() / np.abs(bx).max()
    _log("%s grouped: valid %d (oracle %d), H vs G^T H G %.2e, b %.2e" % (precision, evg["n_valid"], ref["n_valid"],
                                                                         dH, db))
    assert evg["F"] == evf["F"] and evg["n_valid"] == evf["n_valid"]
    assert dH <= 1e-12 and db <= 1e-12
    assert abs(evg["n_valid"] - ref["n_valid"]) <= 1e-4 * ref["n_valid"]
    assert abs(evg["F"] - ref["F"]) <= 1e-4 * ref["F"]


def test_grouped_lm_matches_oracle(rig, pba):
    """LM on the frame's pose variable (LiDAR pairs), FP64 path: same accept pattern and poses
    within 1e-6 of the oracle's."""
    lid = np.array([(0, 2), (2, 0)], np.int32)
    X_or, log_or = oracle.optimize(rig, rig.init_poses, iters=6, lm=True, lam0=1e-4, pairs=lid)
    with pba.context_for_problem(rig, precision=pba.PBA_F64) as ctx:
        ctx.set_pairs(lid)
        logs = ctx.iterate(6, use_lm=True, lambda0=1e-4)
        X = ctx.get_poses()
    assert X.shape == (2, 12)
    assert [l["accepted"] for l in logs] == [l["accepted"] for l in log_or]
    d = np.abs(X - X_or).max()
    _log("grouped LM pose diff vs oracle %.3g" % d)
    assert d < 1e-6


def test_fusion_schedules_self_alignment(rig, pba):
    """From 0.1 m / 3 deg, LiDAR alone and the consecutive schedule bring the frame back onto its
    copy (the identity), on both paths; every schedule runs."""
    from paper_2303_16878_amd import fusion
    kf_model = np.array([rig.sensors[s]["model"] for s in rig.kf_sensor])
    lid, cam = fusion.split_pairs(rig.pairs, kf_model)
    assert len(lid) == 2 and len(cam) == 2
    for prec in (pba.PBA_F32, pba.PBA_F64):
        errs = {}
        for sched in fusion.SCHEDULES:
            with pba.context_for_problem(rig, precision=prec) as ctx:
                X, logs = fusion.run_schedule(ctx, sched, lid, cam, iters=30)
            errs[sched] = fusion.frame_error(X)
        _log("precision %d:" % prec, {k: "%.1e m %.1e rad" % v for k, v in errs.items()})
        for sched in ("lidar", "consecutive"):
            assert max(errs[sched]) < 1e-5, (sched, errs[sched])


def test_pose_group_errors(rig, pba):
    with pba.context_for_problem(rig) as ctx:
        for bad in ([0, 0, 2, 2], [0, 0, -1, 1]):
            g = np.array(bad, np.int32)
            with pytest.raises(pba.PbaError):
                ctx._check(ctx.lib.pba_set_pose_groups(ctx.h, g.ctypes.data, 2))
        four = np.ascontiguousarray(np.tile(rig.gt_poses[:1], (4, 1)))
        with pytest.raises(pba.PbaError):   # still two pose variables
            ctx._check(ctx.lib.pba_set_poses(ctx.h, 4, four.ctypes.data, 0))
        ctx.set_pose_groups(None)
        assert ctx.n_poses == 4
        ctx.set_poses(rig.kf_poses(rig.init_poses))
        ev = ctx.evaluate(want_system=True)
        assert ev["H"].shape == (24, 24)


def test_loss_gradients_with_pose_groups(rig, pba):
    """Loss adjoint with shared rig poses (two pose variables, four keyframes): the gradient per
    pose variable and the image gradients of every keyframe -- including those whose index is
    past the number of pose variables -- match the oracle's.  The outputs start as NaN, so a
    keyframe the backward skips fails."""
    pairs = np.array([(0, 2), (2, 0), (1, 3), (3, 1), (0, 1), (3, 2)], np.int32)
    prob = synth.Problem(rig.name, rig.sensors, rig.kf_sensor, rig.gt_poses, rig.init_poses, pairs, dict(rig.params),
                         rig.intensity, rig.depth, rig.normals, rig.scene, rig.pose_of)
    nv = prob.n_poses
    delta = (np.random.default_rng(11).normal(size=(nv, 6)) * 1e-3).astype(np.float32)
    ref = oracle.loss_and_grad(prob, prob.init_poses, delta.astype(np.float64))
    with pba.context_for_problem(prob) as ctx:
        assert ctx.n_poses == nv == 2 and ctx.n == 4
        F = ctx.loss_forward(delta)
        gd = np.full((nv, 6), np.nan, np.float32)
        gI = [np.full(prob.depth[k].shape, np.nan, np.float32) for k in range(prob.n)]
        gD = [np.full(prob.depth[k].shape, np.nan, np.float32) for k in range(prob.n)]
        gN = [np.full(prob.depth[k].shape + (3,), np.nan, np.float32) for k in range(prob.n)]
        ctx.loss_backward(1.0, gd, (gI, gD, gN))
    _log("grouped loss: F gpu %.9g oracle %.9g" % (F, ref["F"]))
    assert abs(F - ref["F"]) <= 1e-5 * ref["F"]
    assert np.abs(gd - ref["g_delta"]).max() <= 1e-4 * np.abs(ref["g_delta"]).max()
    for name, g_gpu, g_orc in (("intensity", gI, ref["gI"]), ("depth", gD, ref["gD"]), ("normals", gN, ref["gN"])):
        for k in range(prob.n):
            assert np.all(np.isfinite(g_gpu[k])), (name, k)
        a = np.concatenate([np.ravel(x) for x in g_gpu])
        b = np.concatenate([np.ravel(x) for x in g_orc])
        rel_l2 = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)
        frac_bad = np.mean(np.abs(a - b) > 1e-3 * np.abs(b).max())
        _log("  %s: rel L2 %.2e, texels beyond 1e-3: %.2e" % (name, rel_l2, frac_bad))
        assert rel_l2 < 1e-3 and frac_bad < 1e-3, name
