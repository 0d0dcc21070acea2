"""Planted mistakes in copies of the oracle (CPU only): each must fail at least one pin.

The pins in test_oracle_pins.py are only worth something if a plausible slip in
the oracle trips them.  Each mutant below is one such slip (a sign, a factor,
a transpose, the printed source-normal Jacobian, a dropped half in the central
difference, the wrong depth cue, two slips in the loss adjoint, two in the sensor offsets); the checks are
condensed versions of the pins: FD gradient, ground-truth residuals, the
linear-ramp identity, FD of the image gradients, the closed-form image Jacobian on
quadratic textures, the exact valid set of the border rule and the brute-force pair
evaluation on tiny images.  The last three mutants (a central difference from the wrong
rows, two blend weights exchanged, the border one column too permissive) pass the FD,
ground-truth, ramp and adjoint checks; the quadratic-texture and valid-set pins and the
brute force catch them (the first two mutants: quadratic and brute force; the third: all three).
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth
from test_oracle_bruteforce import compare_with_oracle, tiny_rig
from test_oracle_pins import fd_grad_F
from test_oracle_stencil import expected_valid, quadratic_G_error, valid_set

SRC = os.path.join(os.path.dirname(oracle.__file__), "pba_oracle.c")

MUTANTS = {
    "skew_sign": ("S[0] = 0;     S[1] = v[2];  S[2] = -v[1];", "S[0] = 0;     S[1] = -v[2];  S[2] = v[1];"),
    "rot_factor": ("Ms[6*i+3+j] = 2.0 * L[3*i+j];", "Ms[6*i+3+j] = 1.0 * L[3*i+j];"),
    "target_factor": ("Mt[6*i+3+j] = -2.0 * L[3*i+j];", "Mt[6*i+3+j] = 2.0 * L[3*i+j];"),
    "warp_transpose": ("matvec3(RjT, w3, y);", "matvec3(Rj, w3, y);"),
    "printed_normal_jacobian": ("matmul3(M_RotRjRi, Sn, A);",
                                "{ double Sn0[9], RR[9]; const double nu[3] = {Ns[3*pix], Ns[3*pix+1], Ns[3*pix+2]};"
                                " skewp(nu, Sn0); matmul3(RotT, Rj, RR); matmul3(RR, Ri, RR); matmul3(RR, ss->Ro, RR);"
                                " matmul3(RR, Sn0, A); }"),
    "central_diff_half": ("double gc00 = 0.5 * (T(y0, x0+1) - T(y0, x0-1));",
                          "double gc00 = 1.0 * (T(y0, x0+1) - T(y0, x0-1));"),
    "pinhole_jac_sign": ("-v[0] * iz2, 0, v[2] * iz2", "v[0] * iz2, 0, v[2] * iz2"),
    "range_cue_as_depth": ("zeta[1] = st->model == 0 ? pbar[2] : range;", "zeta[1] = pbar[2];"),
    "adjoint_depth_sign": ("g += k[ch] * (ac[0] * dp[0] + ac[1] * dp[1] + ac[2] * dp[2]);",
                           "g -= k[ch] * (ac[0] * dp[0] + ac[1] * dp[1] + ac[2] * dp[2]);"),
    "adjoint_normal_transpose": ("k[2] * RR[j] + k[3] * RR[3+j] + k[4] * RR[6+j];",
                                 "k[2] * RR[3*j] + k[3] * RR[3*j+1] + k[4] * RR[3*j+2];"),
    "source_offset_sign": ("for (int k = 0; k < 3; ++k) pu[k] += ss->to[k];",
                           "for (int k = 0; k < 3; ++k) pu[k] -= ss->to[k];"),
    "target_offset_untransposed": ("matvec3(RotT, ym, pbar);", "matvec3(st->Ro, ym, pbar);"),
    # the image-Jacobian stencil: a central difference read from the wrong rows, the bilinear
    # weights of two taps exchanged, the border rule one column too permissive
    "gr10_wrong_row": ("double gr10 = 0.5 * (T(y0+2, x0) - T(y0, x0));",
                       "double gr10 = 0.5 * (T(y0+1, x0) - T(y0-1, x0));"),
    "blend_weights_swapped": ("G[ch][0] = (1-bb) * ((1-a) * gc00 + a * gc01) + bb * ((1-a) * gc10 + a * gc11);",
                              "G[ch][0] = (1-bb) * ((1-a) * gc00 + a * gc10) + bb * ((1-a) * gc01 + a * gc11);"),
    "stencil_bound_off_by_one": ("fx0 <= Wt - 3.0 && fy0 >= 1.0 && fy0 <= Ht - 3.0)) { status",
                                 "fx0 <= Wt - 2.0 && fy0 >= 1.0 && fy0 <= Ht - 3.0)) { status"),
}


def _fd_ok(p, prm):
    X = p.init_poses
    r = oracle.eval_pair(p, X, 1, 0, prm, grad_mode=1)
    g = 2 * r["b12"]
    fd, _ = fd_grad_F(p, X, 1, 0, prm)
    return np.abs(g - fd).max() < 2e-5 * np.abs(fd).max()


def _gt_ok(p, prm, s=1, t=0):
    r = oracle.eval_pair(p, p.gt_poses, s, t, prm, pixels=True)
    v = r["status"] == 0
    if v.sum() < 0.3 * r["n_eval"]:
        return False
    med = np.median(np.abs(r["res"][v]), 0)
    return med[1] < 1e-3 and np.all(med[2:] < 1e-6)


def _ramp_ok(p, prm):
    H, W = p.depth[0].shape
    rr, cc = np.mgrid[0:H, 0:W].astype(np.float64)
    q = synth.Problem(p.name, p.sensors, p.kf_sensor, p.gt_poses, p.init_poses, p.pairs, p.params)
    q.intensity = [(0.25 + cc / 512 - rr / 1024).astype(np.float32)] + list(p.intensity[1:])
    q.depth = [(3.0 + cc / 128 + rr / 256).astype(np.float32)] + list(p.depth[1:])
    q.normals = [np.stack([0.125 + cc / 1024, -0.25 + rr / 512, -0.875 + (cc + rr) / 2048], -1).astype(np.float32)] \
        + list(p.normals[1:])
    prm = dict(prm, occ_tau_pinhole=1e9, huber_delta=1e9)
    a = oracle.eval_pair(q, q.init_poses, 1, 0, prm, grad_mode=0)
    b = oracle.eval_pair(q, q.init_poses, 1, 0, prm, grad_mode=1)
    return np.abs(a["H12"] - b["H12"]).max() <= 1e-9 * np.abs(b["H12"]).max()


def _adj_ok(p, prm):
    q = synth.Problem(p.name, p.sensors, p.kf_sensor, p.gt_poses, p.init_poses, p.pairs, prm)
    q.intensity, q.depth, q.normals = list(p.intensity), list(p.depth), list(p.normals)
    delta = np.zeros((q.n, 6))
    r = oracle.loss_and_grad(q, q.init_poses, delta)
    for arr, garr in (("depth", "gD"), ("normals", "gN")):
        g = r[garr][1]
        for i in np.argsort(-np.abs(g).ravel())[:2]:
            imgs = getattr(q, arr)
            orig = imgs[1]
            vals = []
            for sgn in (1, -1):
                a = orig.copy()
                a.ravel()[i] += sgn * 1e-4
                imgs[1] = a
                vals.append(oracle.evaluate(q, q.init_poses)["F"])
            imgs[1] = orig
            hp = float(np.float32(orig.ravel()[i] + 1e-4) - np.float32(orig.ravel()[i] - 1e-4))
            if abs((vals[0] - vals[1]) / hp - g.ravel()[i]) > 1e-2 * abs(g.ravel()[i]):
                return False
    return True


def _quadratic_ok(rg, li):
    for p in (rg, li):
        for gm in (0, 1):
            err, n, verr, _ = quadratic_G_error(p, 1, 0, gm)
            if not (n > 2000 and err < 1e-12 and verr < 1e-12):
                return False
    return True


def _valid_set_ok():
    for kx, ky in ((2.5, 0.5), (-2.5, -0.5)):
        r, H, W = valid_set(kx, ky)
        if not np.array_equal(r["status"] == oracle.ST_VALID, expected_valid(kx, ky, H, W)):
            return False
    return True


def _brute_ok(rig):
    try:
        for s, t in ((0, 1), (2, 3), (0, 2), (2, 0)):
            for X in (rig.gt_poses, rig.init_poses):
                compare_with_oracle(rig, X, s, t, rig.params, 0)
    except AssertionError:
        return False
    return True


@pytest.fixture(scope="module")
def problems():
    rg = synth.make("rgbd_small")
    rgc = synth.make("rgbd_small", noise=False)
    li = synth.make("lidar128", kfs=[0, 1], H=32, W=512).subset([0, 1])
    lic = synth.make("lidar128", kfs=[0, 1], H=32, W=512, noise=False).subset([0, 1])
    kfs = [0, 1, 200, 201]   # two LiDAR and two camera keyframes of the joint rig
    jc = synth.make("joint", H_l=32, W_l=256, H_c=60, W_c=80, kfs=kfs, noise=False).subset(kfs)
    return rg, rgc, li, lic, jc, tiny_rig()


def _joint_gt_ok(jc):
    # camera -> LiDAR and LiDAR -> camera through both sensor offsets (looser valid fraction: the
    # camera sees part of the LiDAR panorama only)
    for s, t in ((2, 1), (1, 2)):
        r = oracle.eval_pair(jc, jc.gt_poses, s, t, jc.params, pixels=True)
        v = r["status"] == 0
        if v.sum() < 100:
            return False
        med = np.median(np.abs(r["res"][v]), 0)
        if not (med[1] < 2e-3 and np.all(med[2:] < 1e-5)):
            return False
    return True


def _checks(problems):
    rg, rgc, li, lic, jc, rig = problems
    p5 = dict(rg.params, channels=5)
    l5 = dict(li.params, channels=5)
    return {"fd_rgbd": _fd_ok(rg, p5), "fd_lidar": _fd_ok(li, l5), "gt_rgbd": _gt_ok(rgc, p5),
            "gt_lidar": _gt_ok(lic, l5), "ramp": _ramp_ok(rg, p5), "adjoint": _adj_ok(rg, p5),
            "gt_joint": _joint_gt_ok(jc), "quadratic": _quadratic_ok(rg, li), "valid_set": _valid_set_ok(),
            "brute": _brute_ok(rig)}


def test_unmutated_oracle_passes_condensed_checks(problems):
    oracle.use_library(oracle.build_lib())
    assert all(_checks(problems).values())


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, problems, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, name
    mpath = tmp_path / ("oracle_%s.c" % name)
    mpath.write_text(src.replace(old, new))
    so = str(tmp_path / ("liboracle_%s.so" % name))
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-o", so,
                           str(mpath), "-lm"])
    try:
        oracle.use_library(so)
        res = _checks(problems)
    finally:
        oracle.use_library(os.path.join(os.path.dirname(SRC), "liboracle.so"))
    assert not all(res.values()), (name, res)
    if name in DESIGNED:
        assert not res[DESIGNED[name]], (name, res)


# the pin each stencil mutant was designed against (it must be among those that fail)
DESIGNED = {"gr10_wrong_row": "quadratic", "blend_weights_swapped": "quadratic",
            "stencil_bound_off_by_one": "valid_set"}
