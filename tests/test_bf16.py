"""BF16 storage of the intensity and normal images (pba_config.storage_bf16), FP32 evaluation.

The library rounds the images to BF16 (nearest even) when it loads them; the oracle is given the
same images rounded the same way (done here, on the inputs), so the evaluation must match it as
the FP32 path matches the oracle on FP32 images: masks exact outside the 1e-4 px band (depth stays
FP32, so the masks are those of FP32 storage), per-pair H/b within 1e-5."""
import sys

import numpy as np
import pytest

import oracle
import synth
from parity import compare_pair_masks, compare_pair_sums, forced_oracle

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


def bf16_round(x):
    """float32 -> nearest-even BF16, returned as float32 (exactly representable)."""
    b = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).reshape(np.shape(x))


def _rounded(prob):
    import copy
    q = copy.copy(prob)
    q.intensity = [bf16_round(I) for I in prob.intensity]
    q.normals = [bf16_round(N) for N in prob.normals]
    return q


def test_bf16_rounding_pin():
    """The rounding applied to the oracle's inputs: 8 significant bits, halfway cases to the even
    mantissa (the unit in the last place at 1 is 2^-7)."""
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9, 1.0 + 3 * 2.0 ** -8, 0.3, -0.7], np.float32)
    r = bf16_round(x)
    assert r[0] == 1.0
    assert r[1] == 1.0                      # halfway between 1 and 1 + 2^-7: the even one
    assert r[2] == 1.0 + 2.0 ** -7          # beyond halfway: up
    assert r[3] == 1.0 + 2.0 ** -6          # halfway between 1 + 2^-7 and 1 + 2^-6: the even one
    assert abs(r[4] - 0.3) <= 2.0 ** -10 and abs(r[5] + 0.7) <= 2.0 ** -9
    assert np.array_equal(bf16_round(r), r)


@pytest.mark.gpu
@pytest.mark.parametrize("fixture", ["lidar_mini", "joint_mini", "rgbd_small"])
def test_bf16_pairs_match_oracle_on_rounded_images(fixture, request, pba):
    prob = request.getfixturevalue(fixture)
    ref = _rounded(prob)
    ch = prob.params["channels"]
    with pba.context_for_problem(prob, storage_bf16=True) as ctx:
        ev = ctx.evaluate(want_system=True, want_pairs=True)
        worst = (0.0, 0.0)
        for k in range(len(prob.pairs)):
            m = compare_pair_masks(ctx, ref, ref.init_poses, k)
            assert m["n_bad"] == 0, (k, m["n_mismatch"], m["bad_idx"])
            fo = forced_oracle(ref, ref.init_poses, k, m["gpu"])
            c = compare_pair_sums(ev["pairs"][k], fo, 1e-5)
            worst = (max(worst[0], c["H"]), max(worst[1], c["b"]))
            assert c["ok"], (k, c)
    _log(fixture, "BF16 storage, %d channels: worst H %.2e b %.2e" % (ch, worst[0], worst[1]))
    # the images really are held in BF16: the level-0 image read back is the rounded one
    with pba.context_for_problem(prob, storage_bf16=True) as ctx:
        I, D, N = ctx.get_level_image(0, 1)
    assert np.array_equal(I, ref.intensity[1])
    if ch == 5:
        assert np.array_equal(N, ref.normals[1])


@pytest.mark.gpu
def test_bf16_lm_and_pyramid(lidar_mini, pba):
    """LM on BF16 storage reaches the poses LM reaches on the BF16-rounded images held in FP32 (the
    same values, the same FP32 arithmetic); the pyramid built from BF16 storage holds BF16 values
    (means rounded once to BF16) and the coarse-to-fine schedule lowers F on it."""
    ref = _rounded(lidar_mini)
    res = []
    for prob, bf in ((lidar_mini, True), (ref, False)):
        with pba.context_for_problem(prob, storage_bf16=bf) as ctx:
            ctx.iterate(4, use_lm=True, lambda0=1e-4)
            res.append(ctx.get_poses())
    dt = np.abs(res[0][:, 9:] - res[1][:, 9:]).max()
    dr = np.abs(res[0][:, :9] - res[1][:, :9]).max()
    _log("BF16 storage vs rounded FP32 images after 4 LM iterations: %.3g m, %.3g" % (dt, dr))
    assert dt < 1e-6 and dr < 1e-6
    with pba.context_for_problem(lidar_mini, storage_bf16=True) as ctx:
        F0 = ctx.evaluate()["F"]
        ctx.build_pyramid(2)
        I1, D1, N1 = ctx.get_level_image(1, 0)
        assert np.array_equal(bf16_round(I1), I1) and np.array_equal(bf16_round(N1), N1)
        log = ctx.optimize_pyramid([3, 3], rel_tol=1e-3, use_lm=True, lambda0=1e-4)
        ctx.set_level(0)
        assert ctx.evaluate()["F"] < F0
    assert len(log) > 0


@pytest.mark.gpu
def test_bf16_config_errors(pba):
    import ctypes
    lib = pba.load_library()
    h = ctypes.c_void_p()
    cfg = pba.config_default()
    cfg.storage_bf16 = 1
    cfg.precision = pba.PBA_F64
    assert lib.pba_create(ctypes.byref(cfg), ctypes.byref(h)) == pba.PBA_EINVAL
    cfg.precision = pba.PBA_F32
    cfg.storage_bf16 = 2
    assert lib.pba_create(ctypes.byref(cfg), ctypes.byref(h)) == pba.PBA_EINVAL


@pytest.mark.gpu
def test_bf16_full_size_joint_sampled_pairs(pba):
    """The full joint configuration (200 spherical 128x1024 + 400 pinhole 640x480 keyframes, 7200
    pairs) on BF16 storage, in the launch bench.py times: sampled pairs of all four source/target
    sensor combinations against the oracle given the BF16-rounded images."""
    prob = synth.make("joint")
    ref = _rounded(prob)
    sample = [0, 1200, 4, 1204, 2400, 4800, 2404, 7199]   # LiDAR->LiDAR, LiDAR->cam, cam->LiDAR, cam->cam
    with pba.context_for_problem(prob, storage_bf16=True) as ctx:
        ctx.autotune()
        ev = ctx.evaluate(want_pairs=True)
        for k in sample:
            m = compare_pair_masks(ctx, ref, ref.init_poses, k)
            assert m["n_bad"] == 0, (k, m["n_mismatch"], m["bad_idx"])
            fo = forced_oracle(ref, ref.init_poses, k, m["gpu"])
            c = compare_pair_sums(ev["pairs"][k], fo, 1e-5)
            _log("joint pair", k, "valid", m["n_valid"], "band", m["n_band"], "H err %.2e b err %.2e" % (c["H"], c["b"]))
            assert c["ok"], (k, c)
