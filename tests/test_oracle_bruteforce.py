"""Brute-force single-pair evaluation on tiny images, pixel by pixel in plain Python (CPU only).

An independent route to what the oracle computes for one ordered pair, written from the
paper's definitions and not from the oracle's formulas:

  * pi^-1 and pi (Sec. III): pinhole K^-1 [u, v, 1] d and phi(K p); spherical ray from the
    azimuth/elevation of the pixel, and K_12 psi(p) with psi = [atan2(y, x), atan2(z, rho)];
  * the warp through both platform poses and both sensor offsets as 4x4 rigid motions
    (Sec. IV-C Eq. (uprime); Supplementary, multi-sensor point transform);
  * X boxplus dx = X [R(dq), dt] with R(dq) the rotation of the unit quaternion
    (sqrt(1 - |dq|^2), dq) (Supplementary);
  * bilinear sampling, and the image Jacobian as the bilinear blend of the central differences
    1/2 (I[x+1] - I[x-1]) taken at the four bilinear taps (Supplementary, image Jacobians);
    the stencil is formed here as the union of those taps and their four neighbours;
  * cues zeta (intensity of the source pixel, depth or range of the warped point, the source
    normal rotated into the target sensor frame) and e = zeta - I_t(u');
  * the Huber weight on chi^2 = sum_c Omega^c |e^c|^2 (Eq. total-error-multicue).

Every derivative with respect to the 12 pose components (source and target right
perturbations) is taken by complex-step differentiation of the warp itself: f'(x) =
Im f(x + i h) / h with h = 1e-30 carries no cancellation, so it matches an analytic Jacobian to
rounding.  It therefore checks the supplementary point, projective and cue Jacobians (skew
convention, factor 2, transposes, offset composition) without retyping any of them.  The image
term enters as J = d zeta / dx - g^T d u' / dx (chain rule through u' = pi(p_bar)).
"""
import math

import numpy as np
import pytest

import oracle
import synth

H_IMG, W_IMG = 6, 8          # pinhole keyframes
H_SPH, W_SPH = 8, 32         # spherical keyframes: 11.25 deg per column
CS_H = 1e-30


# ---------------------------------------------------------------- rigid motions (complex-safe)

def quat_R(dq):
    """Rotation of the unit quaternion (sqrt(1 - |dq|^2), dq), written for complex arguments."""
    x, y, z = dq
    w = np.sqrt(1.0 - (x * x + y * y + z * z) + 0j)
    return np.array([[w * w + x * x - y * y - z * z, 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), w * w - x * x + y * y - z * z, 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), w * w - x * x - y * y + z * z]])


def mat4(R, t):
    M = np.eye(4, dtype=complex)
    M[:3, :3] = R
    M[:3, 3] = t
    return M


def rigid_inv(M):
    Rt = M[:3, :3].T
    return mat4(Rt, -Rt @ M[:3, 3])


def pose_mat(x12):
    return mat4(np.asarray(x12[:9]).reshape(3, 3), np.asarray(x12[9:]))


def boxplus_mat(X, dx6):
    return X @ mat4(quat_R(dx6[3:]), dx6[:3])


def atan2c(y, x):
    """atan2 for complex-step arguments: the branch is chosen from the real parts, the value and
    its derivative come from the analytic arctan."""
    if abs(x.real) >= abs(y.real):
        a = np.arctan(y / x)
        if x.real < 0:
            a = a + (math.pi if y.real >= 0 else -math.pi)
    else:
        a = math.pi / 2 - np.arctan(x / y)
        if y.real < 0:
            a = a - math.pi
    return a


# ---------------------------------------------------------------- projections (Sec. III)

def ray(sen, c, r):
    """pi^-1(u, 1): the point at unit depth (pinhole) or unit range (spherical) of pixel (col, row)."""
    if sen["model"] == 0:
        return np.array([(c - sen["cx"]) / sen["fx"], (r - sen["cy"]) / sen["fy"], 1.0])
    az = (c - sen["cx"]) / sen["fx"]
    el = (r - sen["cy"]) / sen["fy"]
    return np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])


def project(sen, p):
    """u' = pi(p) (complex-safe) and whether p projects at all."""
    x, y, z = p
    if sen["model"] == 0:
        ok = z.real >= sen["min_depth"]
        return np.array([sen["fx"] * x / z + sen["cx"], sen["fy"] * y / z + sen["cy"]]), ok
    rho = np.sqrt(x * x + y * y)
    rng = np.sqrt(x * x + y * y + z * z)
    ok = rho.real > 0 and rng.real >= sen["min_depth"]
    return np.array([sen["fx"] * atan2c(y, x) + sen["cx"], sen["fy"] * atan2c(z, rho) + sen["cy"]]), ok


def project_real(sen, p):
    """The same projection on real values with the C library's atan2 (the cell decision)."""
    x, y, z = (float(v) for v in p)
    if sen["model"] == 0:
        return (sen["fx"] * x + sen["cx"] * z) / z, (sen["fy"] * y + sen["cy"] * z) / z
    rho = math.sqrt(x * x + y * y)
    return sen["fx"] * math.atan2(y, x) + sen["cx"], sen["fy"] * math.atan2(z, rho) + sen["cy"]


def depth_ok(sen, d):
    return math.isfinite(d) and d > 0 and sen["min_depth"] <= d <= sen["max_depth"]


# ---------------------------------------------------------------- one pair, pixel by pixel

def brute_force_pair(prob, X, s, t, prm, grad_mode=0):
    ss, st = prob.sensors[prob.kf_sensor[s]], prob.sensors[prob.kf_sensor[t]]
    Is, Ds, Ns = (np.asarray(a, np.float64) for a in (prob.intensity[s], prob.depth[s], prob.normals[s]))
    It, Dt, Nt = (np.asarray(a, np.float64) for a in (prob.intensity[t], prob.depth[t], prob.normals[t]))
    chans = [It, Dt] + ([Nt[..., k] for k in range(3)] if prm["channels"] == 5 else [])
    C = len(chans)
    om = [prm["omega_intensity"], prm["omega_depth"]] + [prm["omega_normal"]] * 3
    tau = prm["occ_tau_pinhole"] if st["model"] == 0 else prm["occ_tau_spherical"]
    delta = prm["huber_delta"]
    Xs, Xt = pose_mat(X[s]), pose_mat(X[t])
    Tos, Tot = pose_mat(ss["offset"]), pose_mat(st["offset"])
    Hs, Ws = Ds.shape
    Ht, Wt = Dt.shape
    H12 = np.zeros((12, 12))
    b12 = np.zeros(12)
    F = 0.0
    mask = np.zeros((Hs, Ws), bool)

    def warp(r, c, d, eps):
        """(p_bar, zeta^d, source normal in the target sensor frame) at pose perturbation eps."""
        Ms = boxplus_mat(Xs, eps[:6]) @ Tos
        Mt = rigid_inv(boxplus_mat(Xt, eps[6:]) @ Tot)
        M = Mt @ Ms
        q = d * ray(ss, c, r)
        pbar = M[:3, :3] @ q + M[:3, 3]
        zeta_d = pbar[2] if st["model"] == 0 else np.sqrt(pbar @ pbar)
        n_t = M[:3, :3] @ Ns[r, c]
        return pbar, zeta_d, n_t

    for r in range(Hs):
        for c in range(Ws):
            d = Ds[r, c]
            if not depth_ok(ss, d):
                continue
            pbar0, zd0, n0 = warp(r, c, d, np.zeros(12, complex))
            _, ok = project(st, pbar0)
            if not ok:
                continue
            u, v = project_real(st, pbar0.real)
            x0, y0 = math.floor(u), math.floor(v)
            if not (1 <= x0 <= Wt - 3 and 1 <= y0 <= Ht - 3):
                continue
            # the four bilinear taps and the neighbours their central differences read
            taps4 = [(x0 + i, y0 + j) for j in (0, 1) for i in (0, 1)]
            stencil = set()
            for (x, y) in taps4:
                stencil |= {(x, y), (x - 1, y), (x + 1, y), (x, y - 1), (x, y + 1)}
            assert len(stencil) == 12
            zd = zd0.real
            if not all(depth_ok(st, Dt[y, x]) and abs(Dt[y, x] - zd) <= tau for (x, y) in stencil):
                continue
            a, bb = u - x0, v - y0
            wts = {(x0, y0): (1 - a) * (1 - bb), (x0 + 1, y0): a * (1 - bb),
                   (x0, y0 + 1): (1 - a) * bb, (x0 + 1, y0 + 1): a * bb}
            V = np.zeros(C)
            G = np.zeros((C, 2))
            for ch, img in enumerate(chans):
                for (x, y), w in wts.items():
                    V[ch] += w * img[y, x]
                    if grad_mode == 0:
                        G[ch, 0] += w * 0.5 * (img[y, x + 1] - img[y, x - 1])
                        G[ch, 1] += w * 0.5 * (img[y + 1, x] - img[y - 1, x])
                if grad_mode == 1:   # slope of the bilinear interpolant
                    G[ch, 0] = (1 - bb) * (img[y0, x0 + 1] - img[y0, x0]) + bb * (img[y0 + 1, x0 + 1] - img[y0 + 1, x0])
                    G[ch, 1] = (1 - a) * (img[y0 + 1, x0] - img[y0, x0]) + a * (img[y0 + 1, x0 + 1] - img[y0, x0 + 1])
            zeta = np.array([Is[r, c], zd] + list(n0.real))[:C]
            e = zeta - V
            chi2 = sum(om[ch] * e[ch] ** 2 for ch in range(C))
            if delta > 0 and math.sqrt(chi2) > delta:
                w = delta / math.sqrt(chi2)
                rho = 2 * delta * math.sqrt(chi2) - delta * delta
            else:
                w, rho = 1.0, chi2
            # Jacobians by complex steps through boxplus, the warp and pi
            J = np.zeros((C, 12))
            for k in range(12):
                eps = np.zeros(12, complex)
                eps[k] = CS_H * 1j
                pb, zdk, nk = warp(r, c, d, eps)
                uvk, _ = project(st, pb)
                du = uvk.imag / CS_H
                dz = np.array([0.0, zdk.imag / CS_H] + list(nk.imag / CS_H))[:C]
                for ch in range(C):
                    J[ch, k] = dz[ch] - (G[ch, 0] * du[0] + G[ch, 1] * du[1])
            for ch in range(C):
                H12 += w * om[ch] * np.outer(J[ch], J[ch])
                b12 += w * om[ch] * J[ch] * e[ch]
            F += rho
            mask[r, c] = True
    return dict(H12=H12, b12=b12, F=F, mask=mask)


# ---------------------------------------------------------------- a tiny seeded rig in a box room

def _ray_box_depth(o, dirs, lo, hi):
    """Parameter along each ray from o (inside the box) to the first wall, and the wall's normal."""
    tmin = np.full(len(dirs), np.inf)
    nrm = np.zeros((len(dirs), 3))
    for ax in range(3):
        for bound, sgn in ((lo[ax], 1.0), (hi[ax], -1.0)):
            with np.errstate(divide="ignore", invalid="ignore"):
                tt = (bound - o[ax]) / dirs[:, ax]
            hit = (tt > 0) & (tt < tmin)
            tmin[hit] = tt[hit]
            n = np.zeros(3)
            n[ax] = sgn
            nrm[hit] = n
    return tmin, nrm


def _rot(axis, deg):
    return synth.rot_axis_angle(np.asarray(axis, float), math.radians(deg))


def tiny_rig(seed=0, noise=True):
    """Two pinhole 8 x 6 and two spherical 32 x 8 keyframes (sensor offsets on both) in a box
    room; per-pixel random intensities, rendered depth/range with small noise, wall normals."""
    rng = np.random.default_rng(seed)
    pin_off = np.concatenate([(np.array([[0, 0, 1], [-1, 0, 0], [0, -1, 0]], float) @ _rot([0.3, 1, 0.2], 4)).ravel(),
                              [0.1, 0.05, -0.2]])
    sph_off = np.concatenate([_rot([1, -0.5, 2], 3).ravel(), [0.0, 0.02, 0.3]])
    el_up, el_dn = math.radians(15.0), math.radians(-15.0)
    sensors = [
        dict(model=0, H=H_IMG, W=W_IMG, fx=8.0, fy=8.0, cx=3.5, cy=2.5, min_depth=0.1, max_depth=50.0,
             offset=pin_off),
        dict(model=1, H=H_SPH, W=W_SPH, fx=-W_SPH / (2 * math.pi), fy=-(H_SPH - 1) / (el_up - el_dn),
             cx=W_SPH / 2.0, cy=(H_SPH - 1) * el_up / (el_up - el_dn), min_depth=0.1, max_depth=50.0,
             offset=sph_off),
    ]
    kf_sensor = np.array([0, 0, 1, 1], np.int32)
    gt = []
    for k in range(4):
        R = _rot(rng.normal(size=3), rng.uniform(1.0, 3.0))
        tvec = rng.normal(size=3) * 0.06
        gt.append(np.concatenate([R.ravel(), tvec]))
    gt = np.array(gt)
    lo, hi = np.array([-7.0, -6.0, -4.0]), np.array([9.0, 6.0, 4.0])
    I, D, N = [], [], []
    for k in range(4):
        sen = sensors[kf_sensor[k]]
        Rp, tp = gt[k, :9].reshape(3, 3), gt[k, 9:]
        Ro, to = sen["offset"][:9].reshape(3, 3), sen["offset"][9:]
        Rw, o = Rp @ Ro, Rp @ to + tp
        Hk, Wk = sen["H"], sen["W"]
        rays = np.array([ray(sen, c, r) for r in range(Hk) for c in range(Wk)])
        tpar, nw = _ray_box_depth(o, rays @ Rw.T, lo, hi)
        dep = tpar.reshape(Hk, Wk)
        if noise:
            dep = dep + rng.normal(size=dep.shape) * 0.01
        nrm = (nw @ Rw).reshape(Hk, Wk, 3)   # wall normal in the sensor frame (faces the sensor)
        I.append(rng.uniform(0, 1, (Hk, Wk)).astype(np.float32))
        D.append(dep.astype(np.float32))
        N.append(nrm.astype(np.float32))
    pairs = np.array([(s, t) for s in range(4) for t in range(4) if s != t], np.int32)
    params = dict(channels=5, omega_intensity=1.0, omega_depth=1.0, omega_normal=1.0, huber_delta=0.1,
                  occ_tau_pinhole=0.5, occ_tau_spherical=1.0, anchor=0)
    p = synth.Problem("tiny_rig", sensors, kf_sensor, gt, gt.copy(), pairs, params)
    p.intensity, p.depth, p.normals = I, D, N
    # a perturbed second set of poses (0.05 m / 2 deg)
    init = gt.copy()
    for k in range(1, 4):
        R = gt[k, :9].reshape(3, 3) @ _rot(rng.normal(size=3), 2.0)
        init[k, :9] = R.ravel()
        init[k, 9:] = gt[k, 9:] + rng.normal(size=3) / math.sqrt(3) * 0.05
    p.init_poses = init
    return p


def compare_with_oracle(p, X, s, t, prm, grad_mode=0):
    """(brute force, oracle) for one pair; raises AssertionError on any mismatch."""
    bf = brute_force_pair(p, X, s, t, prm, grad_mode)
    orc = oracle.eval_pair(p, X, s, t, prm, pixels=True, grad_mode=grad_mode)
    np.testing.assert_array_equal(orc["status"] == oracle.ST_VALID, bf["mask"])
    sc = max(np.abs(bf["H12"]).max(), 1e-300)
    assert np.abs(orc["H12"] - bf["H12"]).max() <= 1e-12 * sc, np.abs(orc["H12"] - bf["H12"]).max() / sc
    bsc = max(np.abs(orc["babs12"]).max(), 1e-300)
    assert np.abs(orc["b12"] - bf["b12"]).max() <= 1e-12 * bsc
    assert abs(orc["F"] - bf["F"]) <= 1e-12 * max(bf["F"], 1e-300)
    return bf, orc


@pytest.fixture(scope="module")
def rig():
    return tiny_rig()


@pytest.mark.parametrize("poses", ["gt", "init"])
@pytest.mark.parametrize("grad_mode", [0, 1])
def test_bruteforce_matches_oracle_every_pair(rig, poses, grad_mode):
    """Every ordered pair of the rig (pinhole/spherical in all four combinations, offsets on both
    sensors): identical valid masks, H, b and F within 1e-12."""
    X = rig.gt_poses if poses == "gt" else rig.init_poses
    n_valid = 0
    models = set()
    for s, t in rig.pairs:
        bf, _ = compare_with_oracle(rig, X, int(s), int(t), rig.params, grad_mode)
        n_valid += int(bf["mask"].sum())
        if bf["mask"].any():
            models.add((rig.sensors[rig.kf_sensor[s]]["model"], rig.sensors[rig.kf_sensor[t]]["model"]))
    assert n_valid >= 200
    assert models == {(0, 0), (0, 1), (1, 0), (1, 1)}


def test_bruteforce_exercises_every_decision(rig):
    """The fixture is not degenerate: among its source pixels some fall outside the stencil
    region, some are occluded by the depth gate, some are down-weighted by the Huber kernel."""
    X = rig.init_poses
    codes = set()
    huber = 0
    for s, t in rig.pairs:
        r = oracle.eval_pair(rig, X, int(s), int(t), rig.params, pixels=True)
        codes |= set(np.unique(r["status"]).tolist())
        v = r["status"] == oracle.ST_VALID
        chi2 = (r["res"][v] ** 2).sum(-1)
        huber += int((np.sqrt(chi2) > rig.params["huber_delta"]).sum())
    assert {oracle.ST_VALID, oracle.ST_OUTSIDE, oracle.ST_OCCLUDED} <= codes
    assert huber > 10
