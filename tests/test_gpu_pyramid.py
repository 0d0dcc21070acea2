"""GPU image pyramid and coarse-to-fine optimisation (Sec. IV-A, IV-C) against the oracle.

Level images: bit-exact (depth validity, depth, intensity; normals within 1 FP32 ulp).  Level
evaluation: the pair protocol of the single-level parity tests (masks, then H/b on the GPU's own
correspondences) at levels 1 and 2.  Coarse-to-fine LM in FP64: same accept pattern and levels,
poses within 1e-6 m / 1e-6 rad.  FP32: the widened basin (the oracle's own pin) is reproduced."""
import sys

import numpy as np
import pytest

import oracle
import synth
from parity import compare_pair_masks, compare_pair_sums, forced_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pba():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2303_16878_amd as pba
    pba.load_library()
    return pba


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _p5(p):
    q = synth.Problem(p.name, p.sensors, p.kf_sensor, p.gt_poses, p.init_poses, p.pairs, dict(p.params, channels=5))
    q.intensity, q.depth, q.normals = list(p.intensity), list(p.depth), list(p.normals)
    return q


@pytest.mark.parametrize("fixture,ch", [("rgbd_small", 5), ("rgbd_small", 2), ("lidar_mini", 5)])
def test_level_images_match_oracle(fixture, ch, request, pba):
    p = request.getfixturevalue(fixture)
    p = _p5(p) if ch == 5 else p
    levels = oracle.pyramid(p, 3)
    with pba.context_for_problem(p, channels=ch) as ctx:
        ctx.build_pyramid(3)
        for lev in range(3):
            for k in range(p.n):
                I, D, N = ctx.get_level_image(lev, k)
                lo = levels[lev]
                assert D.shape == lo.depth[k].shape
                ok_g, ok_o = D > 0, lo.depth[k] > 0
                if lev == 0:   # level 0: the loaded images, invalid depth reported as 0
                    sen = p.sensors[p.kf_sensor[k]]
                    d = lo.depth[k]
                    ok_o = np.isfinite(d) & (d >= sen["min_depth"]) & (d <= sen["max_depth"]) & (d > 0)
                assert np.array_equal(ok_g, ok_o), (lev, k, int((ok_g != ok_o).sum()))
                assert np.array_equal(D[ok_g], lo.depth[k][ok_g]), (lev, k)
                assert np.array_equal(I[ok_g], lo.intensity[k][ok_g]), (lev, k)
                if ch == 5:
                    dn = np.abs(N[ok_g].astype(np.float64) - lo.normals[k][ok_g])
                    assert dn.max(initial=0.0) <= 1.2e-7, (lev, k, dn.max())
        _log(fixture, ch, "levels", [lv.depth[0].shape for lv in levels])


@pytest.mark.parametrize("fixture,prec", [("rgbd_small", "F32"), ("lidar_mini", "F32"), ("lidar_mini", "F64")])
def test_level_evaluation_matches_oracle(fixture, prec, request, pba):
    p = _p5(request.getfixturevalue(fixture))
    levels = oracle.pyramid(p, 3)
    precision = pba.PBA_F64 if prec == "F64" else pba.PBA_F32
    tol = 1e-9 if prec == "F64" else 1e-5
    with pba.context_for_problem(p, precision=precision) as ctx:
        ctx.build_pyramid(3)
        for lev in (2, 1):
            ctx.set_level(lev)
            lp = levels[lev]
            ev = ctx.evaluate(want_system=True, want_pairs=True)
            band = 0
            for k in range(len(p.pairs)):
                m = compare_pair_masks(ctx, lp, p.init_poses, k)
                assert m["n_bad"] == 0, (lev, k, m["n_mismatch"], m["bad_idx"])
                band += m["n_band"]
                fo = forced_oracle(lp, p.init_poses, k, m["gpu"])
                c = compare_pair_sums(ev["pairs"][k], fo, tol)
                assert c["ok"], (lev, k, c)
            o = oracle.evaluate(lp, p.init_poses)
            assert ev["n_evaluated"] == o["n_eval"]
            _log(fixture, prec, "level", lev, "valid", ev["n_valid"], "oracle", o["n_valid"], "band", band)
        ctx.set_level(0)
        ev0 = ctx.evaluate()
        assert ev0["n_evaluated"] == oracle.evaluate(p, p.init_poses)["n_eval"]


def _pose_err(X, Y):
    dt = np.abs(X[:, 9:] - Y[:, 9:]).max()
    dr = 0.0
    for a, b in zip(X, Y):
        R = a[:9].reshape(3, 3).T @ b[:9].reshape(3, 3)
        dr = max(dr, np.arccos(np.clip((np.trace(R) - 1) / 2, -1, 1)))
    return dt, dr


def test_coarse_to_fine_lm_matches_oracle(rgbd_small, pba):
    p = rgbd_small
    init = synth._perturb(p.gt_poses, np.random.default_rng(7), 0.1, 4.0)
    iters = (2, 5, 10)
    X_or, log_or = oracle.optimize_coarse_to_fine(p, init, 3, iters=iters, rel_tol=1e-3)
    with pba.context_for_problem(p, precision=pba.PBA_F64, poses=init) as ctx:
        ctx.build_pyramid(3)
        logs = ctx.optimize_pyramid(iters, rel_tol=1e-3)
        X = ctx.get_poses()
    assert [(l["level"], l["accepted"]) for l in logs] == [(l["level"], l["accepted"]) for l in log_or]
    for lg, lo in zip(logs, log_or):
        assert abs(lg["F"] - lo["F"]) <= 1e-8 * lo["F"]
    dt, dr = _pose_err(X, X_or)
    _log("coarse-to-fine pose diff vs oracle: %.3g m %.3g rad over %d iterations" % (dt, dr, len(logs)))
    assert dt < 1e-6 and dr < 1e-6


def test_coarse_to_fine_widens_the_basin_fp32(rgbd_small, pba):
    p = rgbd_small
    init = synth._perturb(p.gt_poses, np.random.default_rng(7), 0.1, 4.0)
    with pba.context_for_problem(p, poses=init) as ctx:
        single = ctx.iterate(17, use_lm=True, lambda0=1e-4)
        X1 = ctx.get_poses()
        ctx.set_poses(init)
        ctx.build_pyramid(3)
        logs = ctx.optimize_pyramid((2, 5, 10), rel_tol=1e-3)
        X2 = ctx.get_poses()
    a1, a2 = oracle.ate_rmse(X1, p.gt_poses), oracle.ate_rmse(X2, p.gt_poses)
    _log("ATE single level %.4f (F %.4g), pyramid %.4f (F %.4g)" % (a1, single[-1]["F"], a2, logs[-1]["F"]))
    assert a1 > 0.02 and a2 < 2e-3


def test_pyramid_errors_and_reload(rgbd_small, pba):
    p = rgbd_small
    with pba.context_for_problem(p) as ctx:
        with pytest.raises(pba.PbaError):
            ctx.set_level(1)
        with pytest.raises(pba.PbaError):
            ctx.build_pyramid(0)
        with pytest.raises(pba.PbaError):
            ctx.build_pyramid(6)            # 120 >> 5 < 4
        ctx.build_pyramid(2)
        ctx.set_level(1)
        e1 = ctx.evaluate()
        ctx.load_keyframes(p.kf_sensor, p.intensity, p.depth, None)   # drops the pyramid, level 0 active
        with pytest.raises(pba.PbaError):
            ctx.set_level(1)
        e0 = ctx.evaluate()
        assert e0["n_evaluated"] > 3 * e1["n_evaluated"]
