"""GPU parity of the z-buffer occlusion variant (occlusion suppression, Sec. IV-C, z-buffer reading:
a point more than tau behind the nearest of the pair's own warped source points in its target cell
is dropped) against the oracle: masks point by point, the pair sums, and LM iterations."""
import math

import numpy as np
import pytest

import oracle
import synth
from parity import compare_pair_masks, compare_pair_sums, forced_oracle
from test_oracle_zbuffer import _scene, _expected_zoccluded

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pba():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2303_16878_amd as pba
    pba.load_library()
    return pba


def _with_zbuffer(p):
    q = synth.Problem(p.name, p.sensors, p.kf_sensor, p.gt_poses, p.init_poses, p.pairs,
                      dict(p.params, occlusion_zbuffer=1))
    q.intensity, q.depth, q.normals = p.intensity, p.depth, p.normals
    return q


@pytest.mark.parametrize("prec", ["F32", "F64"])
def test_closed_form_scene(pba, prec):
    """The scene whose dropped points are known in closed form: exactly the 720 background
    pixels that land in the square's cells are dropped, on the GPU as in the oracle."""
    prob, poses = _scene(1)
    precision = pba.PBA_F64 if prec == "F64" else pba.PBA_F32
    with pba.context_for_problem(prob, precision=precision) as ctx:
        ev = ctx.evaluate(want_pairs=True)
        m = compare_pair_masks(ctx, prob, poses, 0)
    H, W = prob.depth[0].shape
    exp = _expected_zoccluded(H, W)
    gv = m["gpu"]["status"] == 0
    plain = oracle.eval_pair(_scene(0)[0], poses, 0, 1, pixels=True)
    assert np.array_equal(gv, (plain["status"] == 0) & ~exp)
    assert m["n_mismatch"] == 0
    assert int(ev["pairs"][0, 158]) == m["n_valid"]


@pytest.mark.parametrize("name,prec", [("rgbd_small", "F32"), ("rgbd_small", "F64"), ("lidar_mini", "F32")])
def test_generated_scenes_match_oracle(pba, name, prec, request):
    """Masks pair by pair (ties at cell boundaries and at the gates excused and counted), the
    pair sums on the GPU's own correspondences, and the dropped points are not a vacuous set."""
    prob = _with_zbuffer(request.getfixturevalue(name))
    precision = pba.PBA_F64 if prec == "F64" else pba.PBA_F32
    tol = 1e-9 if prec == "F64" else 1e-5
    dropped = ties = 0
    with pba.context_for_problem(prob, precision=precision) as ctx:
        ev = ctx.evaluate(want_pairs=True)
        for k in range(len(prob.pairs)):
            m = compare_pair_masks(ctx, prob, prob.init_poses, k)
            assert m["n_bad"] == 0, (k, m["n_mismatch"], m["bad_idx"])
            ties += m["n_band"] + m["n_gate"]
            dropped += int((m["orc"]["status"] == oracle.ST_ZOCCLUDED).sum())
            orc = forced_oracle(prob, prob.init_poses, k, m["gpu"])
            c = compare_pair_sums(ev["pairs"][k], orc, tol)
            assert c["ok"], (k, c)
    print(name, prec, "z-dropped points", dropped, "ties", ties)
    assert dropped > 0


def test_lm_with_zbuffer_matches_oracle(pba, rgbd_small):
    """Five LM iterations with the variant (the z-buffer pass inside each captured iteration):
    same accept/reject sequence and poses within 1e-6 as the oracle's."""
    prob = _with_zbuffer(rgbd_small)
    X_or, log_or = oracle.optimize(prob, prob.init_poses, iters=5, lm=True, lam0=1e-4)
    with pba.context_for_problem(prob, precision=pba.PBA_F64) as ctx:
        logs = ctx.iterate(5, use_lm=True, lambda0=1e-4)
        X = ctx.get_poses()
    assert [l["accepted"] for l in logs] == [l["accepted"] for l in log_or]
    dt = np.abs(X[:, 9:] - X_or[:, 9:]).max()
    dr = max(math.acos(np.clip((np.trace(a[:9].reshape(3, 3).T @ b[:9].reshape(3, 3)) - 1) / 2, -1, 1))
             for a, b in zip(X, X_or))
    assert dt < 1e-6 and dr < 1e-6, (dt, dr)
    for lg, lo in zip(logs, log_or):
        assert abs(lg["F"] - lo["F"]) <= 1e-8 * lo["F"]


def test_graph_replays_match_eager_with_zbuffer(pba, lidar_mini):
    prob = _with_zbuffer(lidar_mini)
    with pba.context_for_problem(prob, use_graph=True) as cg, pba.context_for_problem(prob, use_graph=False) as ce:
        for it in range(3):
            lg = cg.iterate(1, use_lm=True, lambda0=1e-4 if it == 0 else 0.0)
            le = ce.iterate(1, use_lm=True, lambda0=1e-4 if it == 0 else 0.0)
            assert np.array_equal(cg.get_poses(), ce.get_poses()), it
            # every field but the measured device time
            assert [dict(l, ms=0) for l in lg] == [dict(l, ms=0) for l in le], it


def test_zbuffer_config_errors(pba):
    cfg = pba.config_default()
    cfg.occlusion_zbuffer = 2
    import ctypes
    h = ctypes.c_void_p()
    assert pba.load_library().pba_create(ctypes.byref(cfg), ctypes.byref(h)) == pba.PBA_EINVAL
    cfg.occlusion_zbuffer = 1
    cfg.storage_bf16 = 1          # the z-buffer variant has no BF16 instantiation
    assert pba.load_library().pba_create(ctypes.byref(cfg), ctypes.byref(h)) == pba.PBA_EINVAL
