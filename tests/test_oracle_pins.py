"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test names the passage of the paper it checks and the independent fact
it uses: finite differences, a closed form, an invariant, an exact special
case, a different algorithm from a library, or convergence to ground truth.
"""
import math

import numpy as np
import pytest

import oracle
import synth

from conftest import rot_angle_deg

CH5 = dict(channels=5)


def _params(p, **kw):
    d = dict(p.params)
    d.update(kw)
    return d


# ---------------------------------------------------------------- warp / projection (Sec. III, Eq. uprime)

@pytest.mark.parametrize("fixture", ["rgbd_small", "lidar_mini"])
def test_identity_pair_roundtrip_and_zero_residual(fixture, request):
    """s = t at the same pose: u' = u exactly (pi(pi^-1(u, d)) = u) and every residual is 0."""
    p = request.getfixturevalue(fixture)
    r = oracle.eval_pair(p, p.gt_poses, 0, 0, _params(p, **CH5), pixels=True)
    H, W = p.depth[0].shape
    has_depth = r["status"] != oracle.ST_NODEPTH
    rows, cols = np.nonzero(has_depth)
    uv = r["uv"][rows, cols]
    ok = np.isfinite(uv[:, 0])
    assert ok.mean() > 0.99
    np.testing.assert_allclose(uv[ok, 0], cols[ok], atol=1e-9)
    np.testing.assert_allclose(uv[ok, 1], rows[ok], atol=1e-9)
    valid = r["status"] == oracle.ST_VALID
    assert valid.sum() > 0.5 * has_depth.sum()
    assert np.abs(r["res"][valid]).max() < 1e-9
    assert abs(r["F"]) < 1e-12 * max(1, r["n_valid"])
    np.testing.assert_allclose(r["b12"], 0, atol=1e-7)


@pytest.mark.parametrize("fixture", ["rgbd_small_clean", "lidar_mini_clean"])
def test_ground_truth_residuals_near_zero(fixture, request):
    """Noise-free rendering at ground-truth poses: the warp predicts the target's depth/range and
    normals (geometry is exact up to interpolation), intensities match up to interpolation error;
    at the perturbed poses depth/range residuals are >10x and intensity residuals >2x larger."""
    p = request.getfixturevalue(fixture)
    prm = _params(p, **CH5)
    gt = oracle.eval_pair(p, p.gt_poses, 1, 0, prm, pixels=True)
    bad = oracle.eval_pair(p, p.init_poses, 1, 0, prm, pixels=True)
    eg = np.abs(gt["res"][gt["status"] == 0])
    eb = np.abs(bad["res"][bad["status"] == 0])
    med_g, med_b = np.median(eg, 0), np.median(eb, 0)
    assert gt["n_valid"] > 0.3 * gt["n_eval"]
    assert med_g[1] < 1e-3                       # depth / range [m]
    assert np.all(med_g[2:] < 1e-6)              # normals
    assert med_g[0] < 0.05                       # intensity (interpolation error)
    assert med_g[1] * 10 < med_b[1] and med_g[0] * 2 < med_b[0]


def test_pinhole_exact_integer_shift():
    """Fronto-parallel plane, target camera translated laterally by k*Z/fx: every source pixel lands
    exactly k pixels over, so the (noise-free) residuals vanish and u' - u = k."""
    Z, fx, k = 3.0, 120.0, 2
    prob = synth.make("rgbd_small", render_images=False)
    sen = prob.sensors[0]
    H, W = sen["H"], sen["W"]
    cols = np.arange(W, dtype=np.float64)
    rows = np.arange(H, dtype=np.float64)
    X = (cols[None, :] - sen["cx"]) / fx * Z
    Y = (rows[:, None] - sen["cy"]) / fx * Z
    tex = lambda x, y: 0.5 + 0.2 * np.sin(2.1 * x + 0.3) * np.cos(1.7 * y)
    I0 = tex(X, Y + 0 * X).astype(np.float32)
    # target at x-offset dx sees world point (x) at column c with x = (c - cx) Z / fx + dx
    dx = k * Z / fx
    I1 = tex(X + dx, Y + 0 * X).astype(np.float32)
    D = np.full((H, W), Z, np.float32)
    Nn = np.zeros((H, W, 3), np.float32)
    Nn[..., 2] = -1.0
    prob.intensity, prob.depth, prob.normals = [I0, I1], [D, D], [Nn, Nn]
    prob.kf_sensor = np.zeros(2, np.int32)
    eye = np.array([1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0], np.float64)
    X1 = eye.copy()
    X1[9] = dx
    poses = np.stack([eye, X1])
    r = oracle.eval_pair(prob, poses, 0, 1, _params(prob, **CH5), pixels=True)
    v = r["status"] == 0
    rr, cc = np.nonzero(v)
    assert v.sum() > 0.8 * (H - 4) * (W - 4 - k)
    np.testing.assert_allclose(r["uv"][rr, cc, 0] - cc, -k, atol=1e-9)
    np.testing.assert_allclose(r["uv"][rr, cc, 1] - rr, 0, atol=1e-9)
    assert np.abs(r["res"][v]).max() < 1e-6


# ---------------------------------------------------------------- Jacobians (Supplementary)

def fd_grad_F(p, X, s, t, prm, h_t=1e-8, h_r=1e-9):
    """Central differences of F over the 12 pose components of (s, t).  Translation steps use the
    step actually realised in the pose (t + R dt rounds at world scale), rotation steps are small
    so that few pixels cross a bilinear cell boundary (a kink of the interpolant)."""
    g = np.zeros(12)
    flips = 0
    for k in range(12):
        pose, comp = (s, k) if k < 6 else (t, k - 6)
        h = h_t if comp < 3 else h_r
        vals, steps = [], []
        for sgn in (1, -1):
            dx = np.zeros(6 * p.n)
            dx[6 * pose + comp] = sgn * h
            Xp = oracle.boxplus(X, dx)
            if comp < 3:
                R = X[pose, :9].reshape(3, 3)
                steps.append((R.T @ (Xp[pose, 9:] - X[pose, 9:]))[comp])
            else:
                steps.append(sgn * h)
            vals.append(oracle.eval_pair(p, Xp, s, t, prm, grad_mode=1))
        flips += vals[0]["n_valid"] != vals[1]["n_valid"]
        g[k] = (vals[0]["F"] - vals[1]["F"]) / (steps[0] - steps[1])
    return g, flips


@pytest.mark.parametrize("fixture,channels", [("rgbd_small", 2), ("rgbd_small", 5), ("lidar_mini", 5)])
def test_gradient_matches_finite_differences(fixture, channels, request):
    """b = sum w J^T Omega e with the exact-slope image Jacobian equals (1/2) dF/dx by central FD,
    for both poses: pins dp_bar/dx_i, dp_bar/dx_j (skew convention, factor 2), the projective
    Jacobians, the cue maps, the normal Jacobians and the Huber weight w = d rho / d chi^2."""
    p = request.getfixturevalue(fixture)
    prm = _params(p, channels=channels)
    X = p.init_poses
    s, t = 1, 0
    r = oracle.eval_pair(p, X, s, t, prm, grad_mode=1)
    g_fd, flips = fd_grad_F(p, X, s, t, prm)
    assert flips == 0
    g = 2 * r["b12"]
    assert np.abs(g - g_fd).max() < 2e-5 * np.abs(g_fd).max()


def _huber_rho(chi2, delta):
    e = np.sqrt(chi2)
    return np.where(e <= delta, chi2, 2 * delta * e - delta * delta)


# pairs of the joint rig (keyframes 0-2 LiDAR, 3-7 camera): camera -> LiDAR, LiDAR -> camera,
# camera -> camera, each through both sensor offsets
JOINT_PAIRS = [(4, 1), (1, 4), (4, 3)]


@pytest.mark.parametrize("s,t", JOINT_PAIRS)
def test_joint_rig_ground_truth_residuals(joint_mini_clean, s, t):
    """Noise-free rig at ground truth: points of one sensor, moved through its offset, both
    platform poses and the other sensor's offset, land on the other sensor's depth/range and
    normals; at the perturbed poses the depth/range residuals are >10x larger.  Pins the offset
    composition of the warp (Supplementary: multi-sensor point transform)."""
    p = joint_mini_clean
    prm = _params(p, **CH5)
    gt = oracle.eval_pair(p, p.gt_poses, s, t, prm, pixels=True)
    bad = oracle.eval_pair(p, p.init_poses, s, t, prm, pixels=True)
    assert gt["n_valid"] > 100
    eg = np.abs(gt["res"][gt["status"] == 0])
    eb = np.abs(bad["res"][bad["status"] == 0])
    med_g, med_b = np.median(eg, 0), np.median(eb, 0)
    assert med_g[1] < 2e-3, med_g
    assert np.all(med_g[2:] < 1e-5), med_g
    assert med_g[1] * 10 < med_b[1]


@pytest.mark.parametrize("s,t", JOINT_PAIRS)
def test_joint_rig_gradient_matches_finite_differences(joint_mini, s, t):
    """2b = dF/dx by central differences for both platform poses of a pair whose sensors carry
    offsets (pins the offset terms of the supplementary point Jacobians)."""
    p = joint_mini
    X = p.init_poses
    r = oracle.eval_pair(p, X, s, t, p.params, grad_mode=1)
    assert r["n_valid"] > 50
    g_fd, flips = fd_grad_F(p, X, s, t, p.params)
    assert flips == 0
    g = 2 * r["b12"]
    assert np.abs(g - g_fd).max() < 2e-5 * np.abs(g_fd).max()


@pytest.mark.parametrize("fixture", ["rgbd_small", "lidar_mini"])
def test_hessian_matches_per_pixel_finite_differences(fixture, request):
    """H = sum w J^T Omega J rebuilt from per-pixel central differences of the residual vector
    (exact-slope mode), with the textbook Huber weight; F = sum of the textbook Huber rho."""
    p = request.getfixturevalue(fixture)
    prm = _params(p, **CH5)
    X = p.init_poses
    s, t = 1, 0
    h = 1e-7
    base = oracle.eval_pair(p, X, s, t, prm, pixels=True, grad_mode=1)
    valid = base["status"] == 0
    Jfd = np.zeros(valid.shape + (5, 12))
    keep = valid.copy()
    for k in range(12):
        res = []
        for sgn in (1, -1):
            dx = np.zeros(6 * p.n)
            dx[6 * s + k if k < 6 else 6 * t + k - 6] = sgn * h
            r = oracle.eval_pair(p, oracle.boxplus(X, dx), s, t, prm, pixels=True, grad_mode=1)
            keep &= r["status"] == 0
            res.append(r["res"])
        Jfd[..., k] = (res[0] - res[1]) / (2 * h)
    assert keep.sum() > 0.99 * valid.sum()
    e = base["res"][valid]
    om = np.array([prm["omega_intensity"], prm["omega_depth"]] + [prm["omega_normal"]] * 3)
    chi2 = (om * e * e).sum(1)
    delta = prm["huber_delta"]
    assert abs(_huber_rho(chi2, delta).sum() - base["F"]) < 1e-9 * base["F"]
    w = np.minimum(1.0, delta / np.sqrt(chi2))
    J = Jfd[valid]
    Hfd = np.einsum("p,c,pci,pcj->ij", w, om, J, J)
    bfd = np.einsum("p,c,pci,pc->i", w, om, J, e)
    assert np.abs(Hfd - base["H12"]).max() < 1e-3 * np.abs(base["H12"]).max()
    assert np.abs(bfd - base["b12"]).max() < 1e-3 * np.abs(base["b12"]).max()


def test_central_differences_exact_on_linear_ramps(rgbd_small):
    """On linear-ramp target channels the bilinear blend of central differences equals the slope of
    the bilinear interpolant, so both image-Jacobian modes give the same H and b; on the real
    (non-linear) texture they differ."""
    p = synth.make("rgbd_small")
    H, W = p.depth[0].shape
    rr, cc = np.mgrid[0:H, 0:W].astype(np.float64)
    # dyadic coefficients: the ramps are exactly representable in float32
    p.intensity[0] = (0.25 + cc / 512 - rr / 1024).astype(np.float32)
    p.depth[0] = (3.0 + cc / 128 + rr / 256).astype(np.float32)
    n = np.stack([0.125 + cc / 1024, -0.25 + rr / 512, -0.875 + (cc + rr) / 2048], -1)
    p.normals[0] = n.astype(np.float32)
    prm = _params(p, channels=5, occ_tau_pinhole=1e9, huber_delta=1e9)
    a = oracle.eval_pair(p, p.init_poses, 1, 0, prm, grad_mode=0)
    b = oracle.eval_pair(p, p.init_poses, 1, 0, prm, grad_mode=1)
    assert a["n_valid"] > 1000
    np.testing.assert_allclose(a["H12"], b["H12"], rtol=1e-9, atol=1e-9 * np.abs(b["H12"]).max())
    np.testing.assert_allclose(a["b12"], b["b12"], rtol=1e-9, atol=1e-9 * np.abs(b["b12"]).max())
    c = oracle.eval_pair(rgbd_small, rgbd_small.init_poses, 1, 0, _params(rgbd_small, **CH5), grad_mode=0)
    d = oracle.eval_pair(rgbd_small, rgbd_small.init_poses, 1, 0, _params(rgbd_small, **CH5), grad_mode=1)
    assert np.abs(c["H12"] - d["H12"]).max() > 1e-3 * np.abs(d["H12"]).max()


def _A_matrix(Xs, Xt):
    """J_s = J_t A for the relative platform pose (R, t) = X_t^-1 X_s: A = [[-R, 2 skewp(t) R], [0, -R]]."""
    Rs, ts = Xs[:9].reshape(3, 3), Xs[9:]
    Rt, tt = Xt[:9].reshape(3, 3), Xt[9:]
    R = Rt.T @ Rs
    t = Rt.T @ (ts - tt)
    skewp = np.array([[0, t[2], -t[1]], [-t[2], 0, t[0]], [t[1], -t[0], 0]])
    A = np.zeros((6, 6))
    A[:3, :3] = -R
    A[:3, 3:] = 2 * skewp @ R
    A[3:, 3:] = -R
    return A


@pytest.mark.parametrize("fixture,gm", [("rgbd_small", 0), ("lidar_mini", 0), ("lidar_mini", 1)])
def test_source_jacobian_is_target_jacobian_times_A(fixture, gm, request):
    """The source-pose rows follow from the target-pose rows: H_ss = A^T S A, H_st = A^T S,
    b_s = A^T b_t with S = H_tt (exact algebraic identity of the two supplementary formulas)."""
    p = request.getfixturevalue(fixture)
    X = p.init_poses
    r = oracle.eval_pair(p, X, 1, 0, _params(p, **CH5), grad_mode=gm)
    A = _A_matrix(X[1], X[0])
    S = r["H12"][6:, 6:]
    sc = np.abs(r["H12"]).max()
    np.testing.assert_allclose(r["H12"][:6, :6], A.T @ S @ A, atol=1e-9 * sc)
    np.testing.assert_allclose(r["H12"][:6, 6:], A.T @ S, atol=1e-9 * sc)
    np.testing.assert_allclose(r["b12"][:6], A.T @ r["b12"][6:], atol=1e-9 * np.abs(r["b12"]).max())


# ---------------------------------------------------------------- normal equations

def _global_motion(X, omega, tau):
    G = np.eye(4)
    G[:3, :3] = synth.rot_axis_angle(omega, np.linalg.norm(omega)) if np.linalg.norm(omega) > 0 else np.eye(3)
    G[:3, 3] = tau
    return np.stack([synth.mat_to_pose(G @ synth.pose_to_mat(x)) for x in X])


@pytest.mark.parametrize("fixture", ["rgbd_small", "lidar_mini"])
def test_gauge_invariance_and_symmetric_psd(fixture, request):
    """F depends only on relative poses: F(G X) = F(X) for a rigid G, and the tangent of a global
    motion is in the null space of H and orthogonal to b.  H is symmetric positive semidefinite."""
    p = request.getfixturevalue(fixture)
    prm = _params(p, **CH5)
    X = p.init_poses
    ev = oracle.evaluate(p, X, prm)
    ev2 = oracle.evaluate(p, _global_motion(X, np.array([0.02, -0.01, 0.03]), np.array([0.3, -0.2, 0.1])), prm)
    assert abs(ev2["F"] - ev["F"]) < 1e-9 * ev["F"]
    assert ev2["n_valid"] == ev["n_valid"]
    H, b = ev["H"], ev["b"]
    np.testing.assert_allclose(H, H.T, atol=1e-12 * np.abs(H).max())
    lam = np.linalg.eigvalsh(H)
    assert lam.min() > -1e-9 * lam.max()
    for tau, om in ((np.array([1.0, 0, 0]), np.zeros(3)), (np.array([0, 0.0, 1.0]), np.zeros(3)),
                    (np.zeros(3), np.array([0, 0, 1.0])), (np.zeros(3), np.array([1.0, 0.5, 0]))):
        v = np.zeros(6 * p.n)
        for k in range(p.n):
            R, t = X[k, :9].reshape(3, 3), X[k, 9:]
            v[6 * k:6 * k + 3] = R.T @ (tau + np.cross(om, t))
            v[6 * k + 3:6 * k + 6] = R.T @ om / 2.0      # rotation angle ~ 2 |dq|
        assert np.linalg.norm(H @ v) < 1e-8 * np.linalg.norm(H, 2) * np.linalg.norm(v)
        assert abs(b @ v) < 1e-8 * np.linalg.norm(b) * np.linalg.norm(v)


def test_full_system_gradient_is_half_dF(rgbd_small):
    """Assembled b (exact-slope mode) equals (1/2) dF/dx over all poses by central differences."""
    p = rgbd_small
    prm = _params(p, channels=2)
    X = p.init_poses
    ev = oracle.evaluate(p, X, prm, grad_mode=1)
    h = 1e-8
    rng = np.random.default_rng(0)
    for _ in range(4):
        v = rng.normal(size=6 * p.n)
        Fp = oracle.evaluate(p, oracle.boxplus(X, h * v), prm, grad_mode=1)
        Fm = oracle.evaluate(p, oracle.boxplus(X, -h * v), prm, grad_mode=1)
        assert Fp["n_valid"] == Fm["n_valid"]
        fd = (Fp["F"] - Fm["F"]) / (2 * h)
        assert abs(2 * ev["b"] @ v - fd) < 1e-5 * np.abs(2 * ev["b"]).sum() * np.abs(v).max()


def test_solve_step_residual_and_gauge(rgbd_small):
    """The LM/GN step solves (H + lambda diag H) dx = -b on the gauge-fixed system; anchor fixed."""
    p = rgbd_small
    ev = oracle.evaluate(p, p.init_poses)
    for lam in (0.0, 1e-4, 1.0):
        dx, ok = oracle.solve_step(ev["H"], ev["b"], lam, anchor=0)
        assert ok
        Hg, bg = oracle.gauge_fix(ev["H"], ev["b"], 0)
        A = Hg + lam * np.diag(np.diag(Hg))
        assert np.linalg.norm(A @ dx + bg) < 1e-10 * np.linalg.norm(bg)
        assert np.all(dx[:6] == 0)
        # a different factorisation (LU) gives the same step
        import scipy.linalg
        np.testing.assert_allclose(scipy.linalg.solve(A, -bg), dx, rtol=1e-8, atol=1e-12)
    dx, ok = oracle.solve_step(-np.eye(6 * p.n), ev["b"])
    assert not ok


# ---------------------------------------------------------------- update (Supplementary, boxplus)

def test_quaternion_rotation_against_scipy():
    """R(dq) for the unit quaternion (sqrt(1-|dq|^2), dq) equals scipy's quaternion rotation."""
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(1)
    for _ in range(50):
        dq = rng.normal(size=3)
        dq *= rng.uniform(0, 0.99) / np.linalg.norm(dq)
        w = math.sqrt(1 - dq @ dq)
        ref = Rotation.from_quat([dq[0], dq[1], dq[2], w]).as_matrix()
        np.testing.assert_allclose(oracle.quat_rot(dq), ref, atol=1e-14)
    dq = np.array([1.0, 2.0, -0.5])
    ref = Rotation.from_quat([dq[0], dq[1], dq[2], 1.0]).as_matrix()   # scipy normalises
    np.testing.assert_allclose(oracle.quat_rot(dq), ref, atol=1e-14)
    np.testing.assert_allclose(oracle.quat_rot(np.zeros(3)), np.eye(3), atol=0)


def test_boxplus_is_right_multiplication():
    """X boxplus dx = X exp(dx) with exp(dx) = [[R(dq), dt], [0, 1]] as 4x4 matrices; exp(0) = I."""
    rng = np.random.default_rng(2)
    X = np.stack([synth.mat_to_pose(np.block([[synth.rot_axis_angle(rng.normal(size=3), rng.uniform(0, 3)),
                                               rng.normal(size=(3, 1))], [np.zeros((1, 3)), np.ones((1, 1))]]))
                  for _ in range(3)])
    dx = rng.normal(size=18) * 0.1
    Y = oracle.boxplus(X, dx)
    for k in range(3):
        E = np.eye(4)
        E[:3, :3] = oracle.quat_rot(dx[6 * k + 3:6 * k + 6])
        E[:3, 3] = dx[6 * k:6 * k + 3]
        np.testing.assert_allclose(synth.pose_to_mat(Y[k]), synth.pose_to_mat(X[k]) @ E, atol=1e-14)
    np.testing.assert_array_equal(oracle.boxplus(X, np.zeros(18)), X)


# ---------------------------------------------------------------- ATE (Sec. V)

def test_horn_alignment_against_svd_and_rigid_copy():
    """Horn's quaternion alignment gives the same rotation as the SVD (Kabsch) solution, and a
    rigidly moved copy of a trajectory has ATE 0."""
    rng = np.random.default_rng(3)
    P = rng.normal(size=(40, 3)) * 5
    Rg = synth.rot_axis_angle(rng.normal(size=3), 1.1)
    Q = P @ Rg.T + np.array([3.0, -1.0, 2.0]) + rng.normal(size=P.shape) * 0.05
    R, t = oracle.horn_align(P, Q)
    mp, mq = P.mean(0), Q.mean(0)
    U, _, Vt = np.linalg.svd((P - mp).T @ (Q - mq))
    D = np.diag([1, 1, np.sign(np.linalg.det(Vt.T @ U.T))])
    Rk = Vt.T @ D @ U.T
    np.testing.assert_allclose(R, Rk, atol=1e-10)
    X = np.zeros((40, 12))
    X[:, 9:] = P
    Y = np.zeros((40, 12))
    Y[:, 9:] = P @ Rg.T + np.array([3.0, -1.0, 2.0])
    assert oracle.ate_rmse(X, Y) < 1e-12
    Y[:, 9:] = Q
    d = P @ Rk.T + (mq - Rk @ mp) - Q
    assert abs(oracle.ate_rmse(X, Y) - np.sqrt((d * d).sum(1).mean())) < 1e-12


# ---------------------------------------------------------------- convergence (Sec. IV-C)

def test_gauss_newton_converges_rgbd_small(rgbd_small):
    """Ten GN iterations from the 0.05 m / 2 deg perturbation reach the noise floor: the same ATE
    as optimising from the ground truth, far below the initial error."""
    p = rgbd_small
    ate0 = oracle.ate_rmse(p.init_poses, p.gt_poses)
    X, log = oracle.optimize(p, p.init_poses, iters=10, lm=False)
    Xg, _ = oracle.optimize(p, p.gt_poses, iters=3, lm=False)
    floor = oracle.ate_rmse(Xg, p.gt_poses)
    ate = oracle.ate_rmse(X, p.gt_poses)
    assert ate < ate0 / 20
    assert ate < 2 * floor + 1e-4
    assert log[0]["F"] < oracle.evaluate(p, p.init_poses)["F"]
    for k in range(1, p.n):
        assert rot_angle_deg(X[k, :9].reshape(3, 3), p.gt_poses[k, :9].reshape(3, 3)) < 0.1


def test_levenberg_marquardt_lidar_monotone(lidar_mini):
    """LM on a short LiDAR segment: F never increases on accepted steps and the pose errors drop."""
    p = lidar_mini
    X, log = oracle.optimize(p, p.init_poses, iters=8, lm=True)
    Fs = [oracle.evaluate(p, p.init_poses)["F"]] + [l["F"] for l in log]
    assert all(Fs[i + 1] <= Fs[i] for i in range(len(Fs) - 1))
    for k in range(1, p.n):
        e0 = np.linalg.norm(p.init_poses[k, 9:] - p.gt_poses[k, 9:])
        e1 = np.linalg.norm(X[k, 9:] - p.gt_poses[k, 9:])
        assert e1 < e0 / 3


# ---------------------------------------------------------------- loss gradient (adjoint)

def _loss_fd_delta(p, delta, k, j, h=1e-8):
    dp, dm = delta.copy(), delta.copy()
    dp[k, j] += h
    dm[k, j] -= h
    ep = oracle.evaluate(p, oracle.boxplus(p.init_poses, dp.ravel()))
    em = oracle.evaluate(p, oracle.boxplus(p.init_poses, dm.ravel()))
    if ep["n_valid"] != em["n_valid"]:
        return None
    return (ep["F"] - em["F"]) / (2 * h)


@pytest.mark.parametrize("fixture", ["rgbd_small", "lidar_mini"])
def test_loss_gradient_wrt_delta_matches_fd(fixture, request):
    """dF/d delta of F(X0 boxplus delta) at a non-zero delta: chain rule through R(q) and the
    quaternion right Jacobian L(q), checked by central differences."""
    p = request.getfixturevalue(fixture)
    prm = _params(p, **CH5)
    q = synth.Problem(p.name, p.sensors, p.kf_sensor, p.gt_poses, p.init_poses, p.pairs, prm)
    q.intensity, q.depth, q.normals = p.intensity, p.depth, p.normals
    delta = np.random.default_rng(0).normal(size=(q.n, 6)) * 1e-3
    r = oracle.loss_and_grad(q, q.init_poses, delta)
    scale = np.abs(r["g_delta"]).max()
    checked = 0
    for k in range(q.n):
        for j in range(6):
            fd = _loss_fd_delta(q, delta, k, j)
            if fd is None:
                continue
            checked += 1
            assert abs(fd - r["g_delta"][k, j]) < 2e-5 * scale, (k, j, fd, r["g_delta"][k, j])
    assert checked >= 6 * q.n - 2


@pytest.mark.parametrize("fixture", ["rgbd_small", "lidar_mini"])
def test_loss_gradient_wrt_images_matches_fd(fixture, request):
    """dF/d(image texel) for intensity, depth and normals of a source and a target keyframe, at
    the texels with the largest gradients, by central differences (masks frozen: cases where
    the perturbation changes a mask are skipped)."""
    p = request.getfixturevalue(fixture)
    q = synth.Problem(p.name, p.sensors, p.kf_sensor, p.gt_poses, p.init_poses, p.pairs, _params(p, **CH5))
    q.intensity, q.depth, q.normals = list(p.intensity), list(p.depth), list(p.normals)
    delta = np.random.default_rng(1).normal(size=(q.n, 6)) * 1e-3
    r = oracle.loss_and_grad(q, q.init_poses, delta)
    X = oracle.boxplus(q.init_poses, delta.ravel())
    checked = 0
    for arr, garr in (("intensity", "gI"), ("depth", "gD"), ("normals", "gN")):
        for kf in (0, 1):
            g = r[garr][kf]
            for i in np.argsort(-np.abs(g).ravel())[:3]:
                imgs = getattr(q, arr)
                orig = imgs[kf]
                vals = []
                for sgn in (1, -1):
                    a = orig.copy()
                    a.ravel()[i] += sgn * 1e-4
                    imgs[kf] = a
                    vals.append(oracle.evaluate(q, X))
                imgs[kf] = orig
                if vals[0]["n_valid"] != vals[1]["n_valid"]:
                    continue
                hp = float(np.float32(orig.ravel()[i] + 1e-4) - np.float32(orig.ravel()[i] - 1e-4))
                fd = (vals[0]["F"] - vals[1]["F"]) / hp
                assert abs(fd - g.ravel()[i]) < 1e-3 * abs(g.ravel()[i]), (arr, kf, i, fd, g.ravel()[i])
                checked += 1
    assert checked >= 15
