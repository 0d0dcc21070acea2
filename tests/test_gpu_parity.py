"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the same seeded inputs.

Sizes: the 160x120 RGB-D set (19200 px per keyframe: 2 work items, the second one ragged) and
3-keyframe 48x768 LiDAR sets (36864 px: 3 items, ragged tail), both through every pair; then the
full 640x480 RGB-D and 128x2048 LiDAR configurations in the launch configuration bench.py uses,
on sampled pairs.  Tolerances: masks exact outside the 1e-4 px band (counted); H/b within 1e-5
relative (FP32 path), 1e-9 (FP64 path); poses after iterating within 1e-6 m / 1e-6 rad.
"""
import math
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


CASES = [
    ("rgbd_small", "F64", 2, 0),
    ("rgbd_small", "F32", 2, 0),
    ("rgbd_small", "F32", 5, 0),
    ("rgbd_small", "F32", 5, 1),
    ("lidar_mini", "F32", 5, 0),
    ("lidar_mini", "F64", 5, 0),
    ("lidar_mini", "F32", 5, 1),
    ("lidar_mini", "F32", 2, 0),
    ("joint_mini", "F32", 5, 0),     # two sensors with offsets, all four model combinations
    ("joint_mini", "F64", 5, 0),
]


@pytest.mark.parametrize("fixture,prec,ch,gm", CASES)
def test_pairs_match_oracle(fixture, prec, ch, gm, request, pba):
    prob = request.getfixturevalue(fixture)
    params = dict(prob.params, channels=ch)
    precision = pba.PBA_F64 if prec == "F64" else pba.PBA_F32
    _log("case", fixture, prec, ch, gm)
    with pba.context_for_problem(prob, precision=precision, channels=ch, grad_mode=gm) as ctx:
        ev = ctx.evaluate(want_system=True, want_pairs=True)
        tol = 1e-9 if prec == "F64" else 1e-5
        tot_band = 0
        for k in range(len(prob.pairs)):
            m = compare_pair_masks(ctx, prob, prob.init_poses, k, params=params, grad_mode=gm)
            assert m["n_bad"] == 0, (k, m["n_mismatch"], m["bad_idx"])
            assert m["n_code"] == 0, k
            tot_band += m["n_band"]
            if prec == "F64":
                assert m["n_mismatch"] == 0
            fo = forced_oracle(prob, prob.init_poses, k, m["gpu"], params=params, grad_mode=gm)
            c = compare_pair_sums(ev["pairs"][k], fo, tol)
            assert c["ok"], (k, c)
        _log("  band mismatches", tot_band, "valid", ev["n_valid"])
        # the assembled system against the oracle's own assembly (unforced)
        o = oracle.evaluate(prob, prob.init_poses, params, grad_mode=gm)
        assert ev["n_evaluated"] == o["n_eval"]
        if prec == "F64":
            assert ev["n_valid"] == o["n_valid"]
            sc = np.abs(o["H"]).max()
            assert np.abs(ev["H"] - o["H"]).max() <= 1e-9 * sc
            np.testing.assert_allclose(ev["F"], o["F"], rtol=1e-10)
        assert np.array_equal(ev["H"], ev["H"].T)


def _lidar_variant(H, W, up=8.0, down=-25.0):
    """Three keyframes of the LiDAR loop seen by an H x W spherical sensor with elevations up..down."""
    full = synth.make("lidar128", render_images=False, H=H, W=W)
    full.sensors = [synth.spherical_sensor(H, W, el_up_deg=up, el_down_deg=down)]
    synth.render(full, kfs=[0, 1, 2])
    synth._mask_source(full)
    return full.subset([0, 1, 2])


@pytest.mark.parametrize("variant,prec", [("wide", "F32"), ("wide", "F64"), ("fine", "F32")])
def test_spherical_sensor_variants_match_oracle(variant, prec, pba):
    """The first projection's other branches: elevations beyond 45 degrees inside the image (the
    coarse elevation by the general atan2), and 8192 columns, where the coarse estimate can be more
    than half a pixel off (no depth-interval rejection, only the exact path).  Masks, codes and pair
    sums against the oracle, as for the other fixtures."""
    if variant == "wide":
        prob = _lidar_variant(48, 768, up=50.0, down=-50.0)
    else:
        prob = _lidar_variant(16, 8192)
    precision = pba.PBA_F64 if prec == "F64" else pba.PBA_F32
    tol = 1e-9 if prec == "F64" else 1e-5
    with pba.context_for_problem(prob, precision=precision) as ctx:
        ev = ctx.evaluate(want_pairs=True)
        for k in range(len(prob.pairs)):
            m = compare_pair_masks(ctx, prob, prob.init_poses, k)
            assert m["n_bad"] == 0 and m["n_code"] == 0, (k, m["n_mismatch"], m["bad_idx"])
            fo = forced_oracle(prob, prob.init_poses, k, m["gpu"])
            c = compare_pair_sums(ev["pairs"][k], fo, tol)
            assert c["ok"], (k, c)
        o = oracle.evaluate(prob, prob.init_poses)
        assert ev["n_evaluated"] == o["n_eval"]
        assert abs(ev["n_valid"] - o["n_valid"]) <= 20
        assert ev["n_valid"] > 1000
    _log(variant, prec, "valid", ev["n_valid"], "oracle", o["n_valid"])


def test_evaluation_is_deterministic(lidar_mini, pba):
    with pba.context_for_problem(lidar_mini) as ctx:
        a = ctx.evaluate(want_system=True, want_pairs=True)
        b = ctx.evaluate(want_system=True, want_pairs=True)
        assert np.array_equal(a["pairs"], b["pairs"]) and np.array_equal(a["H"], b["H"])
        assert a["F"] == b["F"]


@pytest.mark.parametrize("prec", ["F64", "F32"])
def test_solve_step_matches_dense_solve(rgbd_small, prec, pba):
    precision = pba.PBA_F64 if prec == "F64" else pba.PBA_F32
    with pba.context_for_problem(rgbd_small, precision=precision) as ctx:
        ev = ctx.evaluate(want_system=True)
        for lam in (0.0, 1e-3):
            dx = ctx.solve_step(lam)
            ref, ok = oracle.solve_step(ev["H"], ev["b"], lam, anchor=0)
            assert ok
            assert np.abs(dx - ref).max() <= 1e-8 * np.abs(ref).max()
        # apply it and compare with the oracle's boxplus
        X0 = ctx.get_poses()
        ctx.apply_step()
        np.testing.assert_allclose(ctx.get_poses(), oracle.boxplus(X0, dx), atol=1e-14)


def _pose_err(A, B):
    dt = np.abs(A[:, 9:] - B[:, 9:]).max()
    dr = 0.0
    for a, b in zip(A, B):
        Ra, Rb = a[:9].reshape(3, 3), b[:9].reshape(3, 3)
        c = np.clip((np.trace(Ra.T @ Rb) - 1) / 2, -1, 1)
        dr = max(dr, math.acos(c) if c < 1 else 0.0)
    return dt, dr


def test_gauss_newton_iterations_match_oracle(rgbd_small, pba):
    prob = rgbd_small
    X_or, log_or = oracle.optimize(prob, prob.init_poses, iters=10, lm=False)
    finals = {}
    for prec in ("F64", "F32"):
        precision = pba.PBA_F64 if prec == "F64" else pba.PBA_F32
        with pba.context_for_problem(prob, precision=precision) as ctx:
            logs = ctx.iterate(10, use_lm=False)
            X = ctx.get_poses()
        dt, dr = _pose_err(X, X_or)
        _log(prec, "GN pose diff vs oracle: %.3g m %.3g rad" % (dt, dr), "F", logs[-1]["F"], log_or[-1]["F"])
        if prec == "F64":
            assert dt < 1e-6 and dr < 1e-6
            for lg, lo in zip(logs, log_or):
                assert abs(lg["F"] - lo["F"]) <= 1e-8 * lo["F"]
        finals[prec] = oracle.ate_rmse(X, prob.gt_poses)
    assert abs(finals["F32"] - finals["F64"]) < 1e-6
    assert finals["F64"] < oracle.ate_rmse(prob.init_poses, prob.gt_poses) / 20


def test_levenberg_marquardt_matches_oracle(lidar_mini, pba):
    prob = lidar_mini
    X_or, log_or = oracle.optimize(prob, prob.init_poses, iters=6, lm=True, lam0=1e-4)
    with pba.context_for_problem(prob, precision=pba.PBA_F64) as ctx:
        logs = ctx.iterate(6, use_lm=True, lambda0=1e-4)
        X = ctx.get_poses()
    assert [l["accepted"] for l in logs] == [l["accepted"] for l in log_or]
    dt, dr = _pose_err(X, X_or)
    _log("LM pose diff vs oracle: %.3g m %.3g rad" % (dt, dr))
    assert dt < 1e-6 and dr < 1e-6
    for lg, lo in zip(logs, log_or):
        assert abs(lg["F"] - lo["F"]) <= 1e-8 * lo["F"]
        assert abs(lg["lam"] - lo["lam"]) <= 1e-12 * max(lo["lam"], 1e-300)


def test_levenberg_marquardt_joint_rig_matches_oracle(joint_mini, pba):
    """LiDAR + camera rig (sensor offsets, cross-sensor pairs, four model groups in one launch)."""
    prob = joint_mini
    X_or, log_or = oracle.optimize(prob, prob.init_poses, iters=5, lm=True, lam0=1e-4)
    with pba.context_for_problem(prob, precision=pba.PBA_F64) as ctx:
        logs = ctx.iterate(5, use_lm=True, lambda0=1e-4)
        X = ctx.get_poses()
    assert [l["accepted"] for l in logs] == [l["accepted"] for l in log_or]
    dt, dr = _pose_err(X, X_or)
    _log("joint LM pose diff vs oracle: %.3g m %.3g rad" % (dt, dr))
    assert dt < 1e-6 and dr < 1e-6
    for lg, lo in zip(logs, log_or):
        assert abs(lg["F"] - lo["F"]) <= 1e-8 * lo["F"]


# ---------------------------------------------------------------- edge cases

def test_identity_pair_and_invalid_keyframe(rgbd_small, pba):
    prob = synth.Problem(rgbd_small.name, rgbd_small.sensors, np.zeros(3, np.int32), rgbd_small.gt_poses[:3].copy(),
                         rgbd_small.init_poses[:3].copy(), np.array([[0, 0], [1, 2], [2, 1], [0, 1]], np.int32),
                         dict(rgbd_small.params))
    prob.intensity = list(rgbd_small.intensity[:3])
    prob.depth = [rgbd_small.depth[0], np.zeros_like(rgbd_small.depth[1]), rgbd_small.depth[2]]
    prob.normals = list(rgbd_small.normals[:3])
    for precision in (pba.PBA_F32, pba.PBA_F64):
        with pba.context_for_problem(prob, precision=precision) as ctx:
            ev = ctx.evaluate(want_pairs=True)
            po = ev["pairs"]
            assert po[0, 158] > 0 and abs(po[0, 156]) < 1e-6 * po[0, 158]     # identity pair: e == 0
            assert po[1, 157] == 0 and po[1, 158] == 0                         # source without depth
            assert po[2, 158] == 0 and po[2, 157] > 0                          # target without depth
            for k in range(len(prob.pairs)):
                m = compare_pair_masks(ctx, prob, prob.init_poses, k)
                assert m["n_bad"] == 0, (precision, k, m["n_mismatch"], m["bad_idx"])


def test_error_paths(rgbd_small, pba):
    prob = rgbd_small
    ctx = pba.Context(channels=2)
    s = prob.sensors[0]
    with pytest.raises(pba.PbaError) as e:
        ctx.add_sensor(7, s["H"], s["W"], s["fx"], s["fy"], s["cx"], s["cy"], 0.1, 10.0)
    assert e.value.status == pba.PBA_EINVAL
    # a spherical sensor finer than 1550 px/rad (the first projection must land within a pixel)
    fine = synth.spherical_sensor(4, 16384)
    with pytest.raises(pba.PbaError) as e:
        ctx.add_sensor(fine["model"], 4, 16384, fine["fx"], fine["fy"], fine["cx"], fine["cy"], 0.5, 80.0)
    assert e.value.status == pba.PBA_EINVAL
    ctx.add_sensor(s["model"], s["H"], s["W"], s["fx"], s["fy"], s["cx"], s["cy"], s["min_depth"], s["max_depth"])
    with pytest.raises(pba.PbaError) as e:
        ctx.evaluate()
    assert e.value.status == pba.PBA_ESTATE
    ctx.load_keyframes(prob.kf_sensor, prob.intensity, prob.depth)
    with pytest.raises(pba.PbaError) as e:
        ctx.evaluate()
    assert e.value.status == pba.PBA_ESTATE
    bad = prob.init_poses.copy()
    bad[2, 0] = np.nan
    with pytest.raises(pba.PbaError) as e:
        ctx.set_poses(bad)
    assert e.value.status == pba.PBA_EINVAL
    bad = prob.init_poses.copy()
    bad[1, :9] *= 1.01
    with pytest.raises(pba.PbaError):
        ctx.set_poses(bad)
    ctx.set_poses(prob.init_poses)
    with pytest.raises(pba.PbaError) as e:
        ctx.set_pairs(np.array([[0, 5]]))
    assert e.value.status == pba.PBA_EINVAL
    with pytest.raises(pba.PbaError) as e:
        ctx.evaluate()
    assert e.value.status == pba.PBA_ESTATE
    ctx.set_pairs(prob.pairs)
    ev = ctx.evaluate()
    assert ev["n_valid"] > 0
    with pytest.raises(pba.PbaError) as e:
        ctx.solve_step(-1.0)
    assert e.value.status == pba.PBA_EINVAL
    with pytest.raises(pba.PbaError) as e:
        ctx.debug_pair(len(prob.pairs), (s["H"], s["W"]))
    assert e.value.status == pba.PBA_EINVAL
    ctx.close()


# ---------------------------------------------------------------- full-size configurations, sampled pairs

@pytest.mark.parametrize("name,sample", [("rgbd_room", [0, 17, 333, 640, 999]),
                                         ("lidar128", [0, 401, 1202, 1800, 2405]),
                                         # loop closures: 0 -> 296 .. 299 and back, 3 -> 299
                                         ("lidar128", [4, 7, 31, 2374, 2382])])
def test_full_size_sampled_pairs(name, sample, pba):
    prob = synth.make(name)
    _log("generated", name, prob.n, "keyframes", len(prob.pairs), "pairs")
    with pba.context_for_problem(prob) as ctx:
        ev = ctx.evaluate(want_pairs=True)
        _log("  valid", ev["n_valid"], "of", ev["n_evaluated"])
        for k in sample:
            m = compare_pair_masks(ctx, prob, prob.init_poses, k)
            assert m["n_bad"] == 0, (k, m["n_mismatch"], m["bad_idx"])
            fo = forced_oracle(prob, prob.init_poses, k, m["gpu"])
            c = compare_pair_sums(ev["pairs"][k], fo, 1e-5)
            _log("  pair", k, "band", m["n_band"], "H err %.2e b err %.2e" % (c["H"], c["b"]))
            assert c["ok"], (k, c)


def test_multiblock_solve_and_lm(pba):
    """A 40-keyframe LiDAR segment at 32x512: n = 240 spans four 64-wide Cholesky blocks (ragged
    last block); the solve matches a dense solve of the same system and LM matches the oracle."""
    full = synth.make("lidar128", kfs=range(40), H=32, W=512)
    prob = full.subset(range(40))
    with pba.context_for_problem(prob, precision=pba.PBA_F64) as ctx:
        ev = ctx.evaluate(want_system=True)
        for lam in (0.0, 1e-4):
            dx = ctx.solve_step(lam)
            ref, ok = oracle.solve_step(ev["H"], ev["b"], lam, anchor=0)
            assert ok
            assert np.abs(dx - ref).max() <= 1e-8 * np.abs(ref).max(), lam
        logs = ctx.iterate(3, use_lm=True, lambda0=1e-4)
        X = ctx.get_poses()
    X_or, log_or = oracle.optimize(prob, prob.init_poses, iters=3, lm=True, lam0=1e-4)
    dt, dr = _pose_err(X, X_or)
    _log("multiblock LM pose diff vs oracle: %.3g m %.3g rad" % (dt, dr))
    assert [l["accepted"] for l in logs] == [l["accepted"] for l in log_or]
    assert dt < 1e-6 and dr < 1e-6


@pytest.mark.parametrize("lds_max", [None, "0"])
@pytest.mark.parametrize("lpr", ["4", "8", "16"])
def test_scattered_pattern_solve(pba, lds_max, lpr, monkeypatch):
    """Keyframes mapped to pose variables by a random permutation: the chain of pairs then couples
    each 64-wide block to most others and the factorisation fills in, so block columns carry more
    tiles than the triangular solve prefetches.  The solve matches a dense solve of the same
    system, with the vector of the triangular solves in LDS and (PBA_TRSV_LDS_MAX=0) in global
    memory, for each supported number of lanes per row of their products (PBA_TRSV_LPR), in the
    natural order (whose single-workgroup triangular solve these settings tune)."""
    if lds_max is not None:
        monkeypatch.setenv("PBA_TRSV_LDS_MAX", lds_max)
    monkeypatch.setenv("PBA_TRSV_LPR", lpr)
    n_kf = 72
    prob = synth.make("lidar128", kfs=range(n_kf), H=16, W=256).subset(range(n_kf))
    perm = np.random.default_rng(7).permutation(n_kf).astype(np.int32)
    X_var = np.empty_like(prob.init_poses)
    X_var[perm] = prob.init_poses
    with pba.context_for_problem(prob, precision=pba.PBA_F64, solve_order=pba.PBA_ORDER_NATURAL) as ctx:
        ctx.set_pose_groups(perm)
        ctx.set_poses(X_var)
        ev = ctx.evaluate(want_system=True)
        H = ev["H"]
        nt = (H.shape[0] + 63) // 64
        coupled = [sum(np.abs(H[64 * i:64 * i + 64, 64 * k:64 * k + 64]).max() > 0 for i in range(k + 1, nt))
                   for k in range(nt)]
        assert max(coupled) > 4, coupled
        for lam in (0.0, 1e-4):
            dx = ctx.solve_step(lam)
            ref, ok = oracle.solve_step(H, ev["b"], lam, anchor=0)
            assert ok
            assert np.abs(dx - ref).max() <= 1e-8 * np.abs(ref).max(), lam


def test_not_positive_definite_then_recovers(lidar_mini, pba):
    """A keyframe left out of every pair has an all-zero 6x6 block, so the damped system is singular:
    solve_step reports PBA_ENOTPD and the step it writes is zero.  With the pairs restored, the next
    solve matches the dense solve again (the failure flag does not stick)."""
    prob = lidar_mini
    pairs = np.asarray(prob.pairs, np.int32)
    lone = prob.n - 1   # not the gauge anchor (keyframe 0)
    keep = pairs[(pairs[:, 0] != lone) & (pairs[:, 1] != lone)]
    assert 0 < len(keep) < len(pairs)
    with pba.context_for_problem(prob, precision=pba.PBA_F64) as ctx:
        ctx.set_pairs(keep)
        dx = np.full(6 * ctx.n_poses, np.nan)
        st = ctx.lib.pba_solve_step(ctx.h, 1e-3, dx.ctypes.data, 0)
        assert st == pba.PBA_ENOTPD
        assert np.all(dx == 0.0)
        with pytest.raises(pba.PbaError):
            ctx.solve_step(1e-3)
        ctx.set_pairs(pairs)
        ev = ctx.evaluate(want_system=True)
        dx = ctx.solve_step(1e-3)
        ref, ok = oracle.solve_step(ev["H"], ev["b"], 1e-3, anchor=0)
        assert ok
        assert np.abs(dx - ref).max() <= 1e-8 * np.abs(ref).max()


def test_graph_replays_match_eager_iterations(lidar_mini, pba):
    """Each replay of the captured iteration graph gives bitwise the same poses and log as the
    same kernels launched one by one; the host reads results between replays."""
    prob = lidar_mini
    with pba.context_for_problem(prob, use_graph=True) as cg, pba.context_for_problem(prob, use_graph=False) as ce:
        for it in range(4):
            lg = cg.iterate(1, use_lm=True, lambda0=1e-4 if it == 0 else 0.0)
            le = ce.iterate(1, use_lm=True, lambda0=1e-4 if it == 0 else 0.0)
            Xg, Xe = cg.get_poses(), ce.get_poses()
            assert np.array_equal(Xg, Xe), it
            # every field but the measured device time
            assert [dict(l, ms=0) for l in lg] == [dict(l, ms=0) for l in le], it
        eg, ee = cg.evaluate(want_system=True), ce.evaluate(want_system=True)
        assert np.array_equal(eg["H"], ee["H"])


def test_iteration_eval_stamps(lidar_mini, pba):
    """The wall-clock stamps around the evaluation inside each iteration (graph replays included)
    give one positive duration per iteration, shorter than the whole iteration."""
    for use_graph in (True, False):
        with pba.context_for_problem(lidar_mini, use_graph=use_graph) as ctx:
            ctx.evaluate()
            ctx.timings(reset=True)
            ctx.iterate(3, use_lm=True)
            t = ctx.timings(reset=True)
            assert t["iter_evals"] == 3 and t["iterations"] == 3, t
            assert 0.0 < t["iter_eval_ms"] < t["iterate_ms"], t


def test_autotune_keeps_results(lidar_mini, pba):
    """The autotuner only changes the work decomposition: the evaluation after it equals the one
    before up to summation order (which pixels share a wave's FP32 tree sum, and the order of the
    FP64 item partials): 1e-6 of max|H|, far inside the 1e-5 parity tolerance."""
    with pba.context_for_problem(lidar_mini) as ctx:
        a = ctx.evaluate(want_system=True)
        pts = ctx.autotune()
        assert len(pts) == 18 and all(ms > 0 for _, _, ms in pts)
        t = ctx.timings()
        assert (t["items_px"], t["grid"]) in [(p, g) for p, g, _ in pts]
        b = ctx.evaluate(want_system=True)
        assert a["n_valid"] == b["n_valid"] and a["n_evaluated"] == b["n_evaluated"]
        assert abs(a["F"] - b["F"]) <= 1e-12 * abs(a["F"])
        assert np.abs(a["H"] - b["H"]).max() <= 1e-6 * np.abs(a["H"]).max()
        logs = ctx.iterate(2, use_lm=True)
        assert all(np.isfinite(l["F"]) for l in logs)


def test_build_pairs_matches_oracle(pba):
    """Sec. IV-B pair graph on a 12-keyframe stretch of the 640x480 room trajectory (at 160x120):
    the FP64 path's counts equal the oracle's, so the kept pair sets are identical; the FP32 path
    may differ only for pairs whose valid ratio is within 1e-3 of the threshold."""
    kfs = list(range(12))
    p = synth.make("rgbd_room", kfs=kfs, H=120, W=160).subset(kfs)
    want, ratios = oracle.build_pairs(p, p.init_poses, max_dist=1.0)
    for precision in (pba.PBA_F64, pba.PBA_F32):
        with pba.context_for_problem(p, precision=precision) as ctx:
            got = ctx.build_pairs(max_dist=1.0)
            ev = ctx.evaluate()
        g, w = set(map(tuple, got.tolist())), set(map(tuple, want.tolist()))
        _log("build_pairs: %d kept (oracle %d) of %d candidates" % (len(g), len(w), len(ratios)))
        if precision == pba.PBA_F64:
            assert g == w
        else:
            for pr in g ^ w:
                assert abs(ratios[pr] - 1.0 / 3.0) < 1e-3, (pr, ratios[pr])
        assert ev["n_evaluated"] > 0


def _predicted_depth(prob, poses, s, t):
    """zeta of every source pixel of pair (s, t): range (spherical target) or depth (pinhole) of the
    source point in the target sensor frame, FP64 (Sec. III, the sensor offsets of the Supplementary)."""
    ss, st = prob.sensors[prob.kf_sensor[s]], prob.sensors[prob.kf_sensor[t]]
    q = oracle.unproject_image(ss, prob.depth[s].astype(np.float64))
    frame = lambda X: (np.asarray(X[:9], np.float64).reshape(3, 3), np.asarray(X[9:12], np.float64))
    Xk = prob.kf_poses(poses)
    (Ros, tos), (Rot, tot) = frame(ss["offset"]), frame(st["offset"])
    (Rs, ts), (Rt, tt) = frame(Xk[s]), frame(Xk[t])
    p = (((q @ Ros.T + tos) @ Rs.T + ts - tt) @ Rt - tot) @ Rot
    return np.linalg.norm(p, axis=-1) if st["model"] == 1 else p[..., 2]


def _gate_dev(Dt, x0, y0, zeta):
    """max |D - zeta| over the 12-tap stencil of cells (x0, y0) (invalid depths: a -1e30 sentinel)."""
    taps = [(0, -1), (0, 0), (0, 1), (0, 2), (1, -1), (1, 0), (1, 1), (1, 2), (-1, 0), (-1, 1), (2, 0), (2, 1)]
    return np.stack([np.abs(Dt[y0 + dy, x0 + dx] - zeta) for dy, dx in taps], -1).max(-1)


@pytest.mark.parametrize("fixture,prec", [("rgbd_small", "F32"), ("lidar_mini", "F32"), ("lidar_mini", "F64"),
                                          ("joint_mini", "F32")])
def test_boundary_band_counts(fixture, prec, request, pba):
    """The evaluation counts, per pair and in total, the points whose stencil lies inside the target
    image, whose projected coordinate is within 1e-4 px of a cell boundary, and which pass the
    occlusion gate in their cell or in a cell across that boundary (the cells a rounding of u' could
    pick; a point failing in all of them keeps its outcome under any rounding).  The same count from
    the oracle's FP64 projections (cells from its u', taps from the target depth image, zeta
    recomputed here in FP64), with no point at 1e-4 +- 1e-11 px or at tau +- 1e-9 m aside, where
    rounding could tip a side."""
    prob = request.getfixturevalue(fixture)
    precision = pba.PBA_F64 if prec == "F64" else pba.PBA_F32
    with pba.context_for_problem(prob, precision=precision) as ctx:
        ev = ctx.evaluate(want_pairs=True)
    total = 0
    for k, (s, t) in enumerate(prob.pairs):
        s, t = int(s), int(t)
        o = oracle.eval_pair(prob, prob.init_poses, s, t, pixels=True)
        reached = (o["status"] == 0) | (o["status"] == 4) | (o["status"] == 5)   # passed the stencil test
        uv = o["uv"][reached]
        frac = uv - np.floor(uv)
        dist = np.minimum(frac, 1.0 - frac)
        assert not np.any(np.abs(dist - 1e-4) < 1e-11)
        inb = dist < 1e-4                      # per axis: within the band of a boundary
        band = inb.any(-1)
        st = prob.sensors[prob.kf_sensor[t]]
        Ht, Wt = st["H"], st["W"]
        Dt = prob.depth[t].astype(np.float64)
        Dt = np.where(np.isfinite(Dt) & (Dt > 0) & (Dt >= st["min_depth"]) & (Dt <= st["max_depth"]), Dt, -1e30)
        zeta = _predicted_depth(prob, prob.init_poses, s, t)[reached][band]
        tau = prob.params["occ_tau_spherical" if st["model"] == 1 else "occ_tau_pinhole"]
        x0, y0 = np.floor(uv[band, 0]).astype(int), np.floor(uv[band, 1]).astype(int)
        su = np.where(frac[band, 0] < 0.5, -1, 1)
        sv = np.where(frac[band, 1] < 0.5, -1, 1)
        reach = np.zeros(len(x0), bool)
        for cu in (0, 1):
            for cv in (0, 1):
                cx, cy = x0 + cu * su, y0 + cv * sv
                use = ((cu == 0) | inb[band, 0]) & ((cv == 0) | inb[band, 1])
                use &= (cx >= 1) & (cx <= Wt - 3) & (cy >= 1) & (cy <= Ht - 3)
                dev = np.full(len(x0), np.inf)
                dev[use] = _gate_dev(Dt, cx[use], cy[use], zeta[use])
                assert not np.any(np.abs(dev - tau) < 1e-9)
                reach |= dev <= tau
        n = int(reach.sum())
        assert int(ev["pairs"][k][159]) == n, (k, ev["pairs"][k][159], n)
        total += n
    _log(fixture, prec, "boundary band", total, "of", ev["n_valid"], "valid")
    assert ev["n_boundary_band"] == total
    assert total > 0


def test_full_size_lidar_lm_matches_oracle(pba):
    """The full 128x2048 LiDAR loop (300 keyframes, 2406 pairs, n = 1800) on the FP64 path: two LM
    iterations accept and reject as the oracle's do and end within 1e-6 m / 1e-6 rad of its poses
    (the oracle needs three full evaluations of 6.2e8 px-pairs: about 100 s on 16 host cores)."""
    prob = synth.make("lidar128")
    iters = 2
    with pba.context_for_problem(prob, precision=pba.PBA_F64) as ctx:
        logs = ctx.iterate(iters, use_lm=True, lambda0=1e-4)
        X = ctx.get_poses()
    _log("GPU FP64 LM:", [(round(l["F"], 3), l["accepted"]) for l in logs])
    X_or, log_or = oracle.optimize(prob, prob.init_poses, iters=iters, lm=True, lam0=1e-4)
    _log("oracle LM:  ", [(round(l["F"], 3), l["accepted"]) for l in log_or])
    dt, dr = _pose_err(X, X_or)
    _log("full-size LM pose diff vs oracle: %.3g m %.3g rad" % (dt, dr))
    assert [l["accepted"] for l in logs] == [l["accepted"] for l in log_or]
    for a, b in zip(logs, log_or):
        assert abs(a["F"] - b["F"]) <= 1e-7 * abs(b["F"])   # summation order; band points
    assert dt < 1e-6 and dr < 1e-6


def test_fp32_and_fp64_paths_reach_the_same_accuracy(pba):
    """A 30-keyframe stretch of the 128x2048 LiDAR loop: after 25 LM iterations the FP32 evaluation
    path's ATE RMSE equals the FP64 path's within 1e-6 m (both start from the same perturbed poses)."""
    from paper_2303_16878_amd.metrics import ate_rmse
    kfs = list(range(30))
    prob = synth.make("lidar128", kfs=kfs).subset(kfs)
    ate = {}
    for name, prec in (("f32", pba.PBA_F32), ("f64", pba.PBA_F64)):
        with pba.context_for_problem(prob, precision=prec) as ctx:
            ctx.iterate(25, use_lm=True, lambda0=1e-4)
            ate[name] = ate_rmse(ctx.get_poses(), prob.gt_poses)
    a0 = ate_rmse(prob.init_poses, prob.gt_poses)
    _log("30-keyframe segment ATE: start %.6f m, FP32 %.9f m, FP64 %.9f m, |diff| %.3g m" % (
        a0, ate["f32"], ate["f64"], abs(ate["f32"] - ate["f64"])))
    assert ate["f64"] < a0
    assert abs(ate["f32"] - ate["f64"]) < 1e-6
