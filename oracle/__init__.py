"""Plain FP64 CPU oracle of photometric LiDAR / RGB-D bundle adjustment.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import this package.  The product library
(paper_2303_16878_amd) shares no code with it and never calls it.

What it computes (paper section in brackets):
  * per pair and pixel: warp, projection, multi-cue residuals, Huber weight,
    Jacobians w.r.t. both poses, written out in pba_oracle.c
    [Sec. III, Sec. IV-C Eqs. (uprime), (total-error-multicue), Supplementary];
  * the 6N x 6N normal equations H dx = -b assembled from the per-pair 12x12
    blocks in pair order [Sec. IV-C: Levenberg-Marquardt over all poses];
  * the gauge: the anchor pose is held fixed (identity rows, zero gradient);
  * the Levenberg-Marquardt / Gauss-Newton step (H + lambda diag H) dx = -b,
    solved by a Cholesky factorisation (library primitive);
  * the pose update X <- X exp(dx) with exp(dx) = [R(dq), dt], R(dq) the
    rotation of the unit quaternion with imaginary part dq [Supplementary];
  * ATE RMSE after Horn's closed-form SE(3) alignment [Sec. V];
  * optionally, occlusion suppression by a z-buffer of the pair's own warped source points in
    addition to the depth-consistency gate [Sec. IV-C: occluded portions are suppressed; the
    mechanism is a reading].

Every function here is pinned by tests/test_oracle_pins.py against facts that
do not come from the oracle itself (finite differences, closed forms,
invariants, a different alignment algorithm, convergence to ground truth).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

# per-pixel status codes written by orc_eval_pair
ST_VALID, ST_NODEPTH, ST_NOPROJ, ST_OUTSIDE, ST_BADTAP, ST_OCCLUDED, ST_SKIPPED, ST_ZOCCLUDED = range(8)


class OrcSensor(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("fx", ctypes.c_double), ("fy", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double), ("dmin", ctypes.c_double),
                ("dmax", ctypes.c_double), ("Ro", ctypes.c_double * 9), ("to", ctypes.c_double * 3)]


class OrcParams(ctypes.Structure):
    _fields_ = [("channels", ctypes.c_int32), ("grad_mode", ctypes.c_int32),
                ("omega", ctypes.c_double * 3), ("huber", ctypes.c_double), ("occ_tau", ctypes.c_double),
                ("zbuffer", ctypes.c_int32), ("pad", ctypes.c_int32)]


class OrcPairOut(ctypes.Structure):
    _fields_ = [("H", ctypes.c_double * 144), ("b", ctypes.c_double * 12), ("F", ctypes.c_double),
                ("n_eval", ctypes.c_int64), ("n_valid", ctypes.c_int64), ("babs", ctypes.c_double * 12)]


class OrcImageGrad(ctypes.Structure):
    _fields_ = [("gIs", ctypes.c_void_p), ("gDs", ctypes.c_void_p), ("gNs", ctypes.c_void_p),
                ("gIt", ctypes.c_void_p), ("gDt", ctypes.c_void_p), ("gNt", ctypes.c_void_p)]


class OrcFrame(ctypes.Structure):
    _fields_ = [("I", ctypes.c_void_p), ("D", ctypes.c_void_p), ("N", ctypes.c_void_p),
                ("sensor", ctypes.c_int32), ("pad", ctypes.c_int32)]


def build_lib(force: bool = False) -> str:
    src = os.path.join(_HERE, "pba_oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def use_library(path):
    """Load the oracle from another build of pba_oracle.c (tests plant mistakes in copies)."""
    global _lib, _LIB_PATH
    _lib = None
    _LIB_PATH = path
    return _load()


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_lib()
        lib = ctypes.CDLL(_LIB_PATH)
        vp = ctypes.c_void_p
        lib.orc_eval_pair.restype = ctypes.c_int
        lib.orc_eval_pair.argtypes = [ctypes.POINTER(OrcSensor), vp, vp, vp, ctypes.POINTER(OrcSensor), vp, vp,
                                      vp, vp, vp, ctypes.POINTER(OrcParams), vp, vp,
                                      ctypes.POINTER(OrcPairOut), vp, vp, vp, vp]
        lib.orc_eval_pair_grad.restype = ctypes.c_int
        lib.orc_eval_pair_grad.argtypes = lib.orc_eval_pair.argtypes + [vp, ctypes.POINTER(OrcImageGrad)]
        lib.orc_zbuffer.restype = None
        lib.orc_zbuffer.argtypes = [ctypes.POINTER(OrcSensor), vp, ctypes.POINTER(OrcSensor), vp, vp, vp]
        lib.orc_eval_pairs.restype = ctypes.c_int
        lib.orc_eval_pairs.argtypes = [vp, vp, vp, ctypes.c_int, vp, vp, ctypes.POINTER(OrcParams),
                                       ctypes.POINTER(OrcParams), vp]
        _lib = lib
    return _lib


# ------------------------------------------------------------------ marshalling

def sensor_struct(sen) -> OrcSensor:
    s = OrcSensor()
    s.model, s.H, s.W = int(sen["model"]), int(sen["H"]), int(sen["W"])
    s.fx, s.fy, s.cx, s.cy = float(sen["fx"]), float(sen["fy"]), float(sen["cx"]), float(sen["cy"])
    s.dmin, s.dmax = float(sen["min_depth"]), float(sen["max_depth"])
    off = np.asarray(sen["offset"], np.float64)
    for i in range(9):
        s.Ro[i] = off[i]
    for i in range(3):
        s.to[i] = off[9 + i]
    return s


def params_struct(params: dict, model: int, grad_mode: int = 0) -> OrcParams:
    p = OrcParams()
    p.channels = int(params["channels"])
    p.grad_mode = int(params.get("grad_mode", grad_mode))
    p.omega[0] = params["omega_intensity"]
    p.omega[1] = params["omega_depth"]
    p.omega[2] = params["omega_normal"]
    p.huber = params["huber_delta"]
    p.occ_tau = params["occ_tau_pinhole"] if model == 0 else params["occ_tau_spherical"]
    p.zbuffer = int(params.get("occlusion_zbuffer", 0))
    return p


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# ------------------------------------------------------------------ evaluation

def eval_pair(prob, poses, s, t, params=None, force_valid=None, force_cell=None, pixels=False,
              grad_mode=0):
    """One ordered pair (s -> t).

    Returns dict(H12, b12, babs12, F, n_eval, n_valid[, status, uv, res, margin, G]); G is the
    per-pixel image Jacobian [H, W, 5, 2] (d/dcol, d/drow of each channel at u'; NaN where not valid)."""
    lib = _load()
    params = prob.params if params is None else params
    ss, st = prob.sensors[prob.kf_sensor[s]], prob.sensors[prob.kf_sensor[t]]
    Is, Ds, Ns = _c(prob.intensity[s], np.float32), _c(prob.depth[s], np.float32), _c(prob.normals[s], np.float32)
    It, Dt, Nt = _c(prob.intensity[t], np.float32), _c(prob.depth[t], np.float32), _c(prob.normals[t], np.float32)
    Xs, Xt = _c(poses[s], np.float64), _c(poses[t], np.float64)
    prm = params_struct(params, st["model"], grad_mode)
    out = OrcPairOut()
    Hs, Ws = ss["H"], ss["W"]
    status = np.empty((Hs, Ws), np.uint8) if pixels else None
    uv = np.empty((Hs, Ws, 2), np.float64) if pixels else None
    res = np.empty((Hs, Ws, 5), np.float64) if pixels else None
    margin = np.empty((Hs, Ws), np.float64) if pixels else None
    gimg = np.empty((Hs, Ws, 5, 2), np.float64) if pixels else None
    fv = _c(force_valid, np.uint8) if force_valid is not None else None
    fc = _c(force_cell, np.int32) if force_cell is not None else None
    rc = lib.orc_eval_pair_grad(ctypes.byref(sensor_struct(ss)), Is.ctypes.data, Ds.ctypes.data, Ns.ctypes.data,
                                ctypes.byref(sensor_struct(st)), It.ctypes.data, Dt.ctypes.data, Nt.ctypes.data,
                                Xs.ctypes.data, Xt.ctypes.data, ctypes.byref(prm),
                                fv.ctypes.data if fv is not None else None,
                                fc.ctypes.data if fc is not None else None,
                                ctypes.byref(out),
                                status.ctypes.data if pixels else None,
                                uv.ctypes.data if pixels else None,
                                res.ctypes.data if pixels else None,
                                margin.ctypes.data if pixels else None,
                                gimg.ctypes.data if pixels else None, None)
    if rc != 0:
        raise RuntimeError("orc_eval_pair failed (%d)" % rc)
    r = dict(H12=np.array(out.H).reshape(12, 12), b12=np.array(out.b), babs12=np.array(out.babs), F=out.F,
             n_eval=out.n_eval, n_valid=out.n_valid)
    if pixels:
        r.update(status=status, uv=uv, res=res, margin=margin, G=gimg)
    return r


def zbuffer(prob, poses, s, t):
    """The source z-buffer of the ordered pair (s -> t) used by the z-buffer occlusion variant:
    [Ht, Wt] float32, per target cell the smallest predicted depth (FP32) of the pair's source
    points whose integer cell lies in the evaluated region, +inf elsewhere (orc_zbuffer)."""
    lib = _load()
    ss, st = prob.sensors[prob.kf_sensor[s]], prob.sensors[prob.kf_sensor[t]]
    Ds = _c(prob.depth[s], np.float32)
    Xs, Xt = _c(poses[s], np.float64), _c(poses[t], np.float64)
    Z = np.empty((st["H"], st["W"]), np.float32)
    lib.orc_zbuffer(ctypes.byref(sensor_struct(ss)), Ds.ctypes.data, ctypes.byref(sensor_struct(st)),
                    Xs.ctypes.data, Xt.ctypes.data, Z.ctypes.data)
    return Z


def eval_pairs(prob, poses, params=None, pairs=None, grad_mode=0):
    """All pairs, OpenMP over pairs.  Returns per-pair arrays H12 [P,12,12], b12 [P,12], F, n_eval, n_valid."""
    lib = _load()
    params = prob.params if params is None else params
    pairs = prob.pairs if pairs is None else np.asarray(pairs, np.int32)
    sens = (OrcSensor * len(prob.sensors))(*[sensor_struct(s) for s in prob.sensors])
    keep = []
    frames = (OrcFrame * prob.n)()
    for k in range(prob.n):
        if prob.depth[k] is None:
            continue
        I, D, N = _c(prob.intensity[k], np.float32), _c(prob.depth[k], np.float32), _c(prob.normals[k], np.float32)
        keep += [I, D, N]
        frames[k].I, frames[k].D, frames[k].N = I.ctypes.data, D.ctypes.data, N.ctypes.data
        frames[k].sensor = int(prob.kf_sensor[k])
    poses = _c(poses, np.float64)
    src, tgt = _c(pairs[:, 0], np.int32), _c(pairs[:, 1], np.int32)
    outs = (OrcPairOut * len(pairs))()
    pp, ps = params_struct(params, 0, grad_mode), params_struct(params, 1, grad_mode)
    rc = lib.orc_eval_pairs(ctypes.cast(sens, ctypes.c_void_p), ctypes.cast(frames, ctypes.c_void_p),
                            poses.ctypes.data, len(pairs), src.ctypes.data, tgt.ctypes.data,
                            ctypes.byref(pp), ctypes.byref(ps), ctypes.cast(outs, ctypes.c_void_p))
    if rc != 0:
        raise RuntimeError("orc_eval_pairs failed")
    P = len(pairs)
    H12 = np.array([np.array(o.H) for o in outs]).reshape(P, 12, 12)
    b12 = np.array([np.array(o.b) for o in outs]).reshape(P, 12)
    return dict(H12=H12, b12=b12, F=np.array([o.F for o in outs]),
                n_eval=np.array([o.n_eval for o in outs]), n_valid=np.array([o.n_valid for o in outs]))


def assemble(pair_res, pairs, n, pose_of=None):
    """Sum per-pair 12x12 blocks into the 6n x 6n system in pair order.  With pose_of (keyframe ->
    pose variable, for keyframes that share a rig pose), the source and target blocks go to their
    keyframes' variables: the chain rule for X_kf = X_var under a common right perturbation, so a
    pair inside one variable adds all four of its 6x6 blocks to that variable's diagonal block."""
    H = np.zeros((6 * n, 6 * n))
    b = np.zeros(6 * n)
    for p, (s, t) in enumerate(np.asarray(pairs)):
        v = (int(s), int(t)) if pose_of is None else (int(pose_of[s]), int(pose_of[t]))
        for a in range(2):
            b[6 * v[a]:6 * v[a] + 6] += pair_res["b12"][p][6 * a:6 * a + 6]
            for c in range(2):
                H[6 * v[a]:6 * v[a] + 6, 6 * v[c]:6 * v[c] + 6] += pair_res["H12"][p][6 * a:6 * a + 6, 6 * c:6 * c + 6]
    return H, b


def evaluate(prob, poses, params=None, pairs=None, grad_mode=0):
    """The system at `poses`: one pose per keyframe, or per pose variable when prob.pose_of is set."""
    pairs = prob.pairs if pairs is None else pairs
    pose_of = getattr(prob, "pose_of", None)
    kfp = np.asarray(poses, np.float64) if pose_of is None else np.asarray(poses, np.float64)[np.asarray(pose_of)]
    pr = eval_pairs(prob, kfp, params, pairs, grad_mode)
    H, b = assemble(pr, pairs, prob.n if pose_of is None else int(np.max(pose_of)) + 1, pose_of)
    return dict(H=H, b=b, F=float(pr["F"].sum()), n_eval=int(pr["n_eval"].sum()),
                n_valid=int(pr["n_valid"].sum()), pairs=pr)


# ------------------------------------------------------------------ solve and update

def gauge_fix(H, b, anchor=0):
    """Hold the anchor pose fixed: its rows/columns become identity and its gradient zero."""
    H = H.copy()
    b = b.copy()
    sl = slice(6 * anchor, 6 * anchor + 6)
    H[sl, :] = 0.0
    H[:, sl] = 0.0
    H[sl, sl] = np.eye(6)
    b[sl] = 0.0
    return H, b


def solve_step(H, b, lam=0.0, anchor=0):
    """Solve (H + lam diag(H)) dx = -b with the anchor fixed; Cholesky factorisation.

    Returns (dx, ok); ok is False when the damped matrix is not positive definite."""
    Hg, bg = gauge_fix(H, b, anchor)
    A = Hg + lam * np.diag(np.diag(Hg))
    try:
        L = np.linalg.cholesky(A)
    except np.linalg.LinAlgError:
        return np.zeros_like(b), False
    y = np.linalg.solve(L, -bg)       # L y = -b   (dense, triangular L)
    dx = np.linalg.solve(L.T, y)      # L^T dx = y
    return dx, True


def quat_rot(dq):
    """Rotation of the unit quaternion (w, dq), w = sqrt(1 - |dq|^2); if |dq| >= 1, (1, dq) normalised."""
    qx, qy, qz = (float(v) for v in dq)
    n2 = qx * qx + qy * qy + qz * qz
    if n2 < 1.0:
        w = math.sqrt(1.0 - n2)
    else:
        s = 1.0 / math.sqrt(1.0 + n2)
        w, qx, qy, qz = s, qx * s, qy * s, qz * s
    return np.array([
        [1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qz * w), 2 * (qx * qz + qy * w)],
        [2 * (qx * qy + qz * w), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qx * w)],
        [2 * (qx * qz - qy * w), 2 * (qy * qz + qx * w), 1 - 2 * (qx * qx + qy * qy)]])


def boxplus(poses, dx):
    """X_k <- X_k exp(dx_k): R_k <- R_k R(dq_k), t_k <- t_k + R_k dt_k (dx_k = [dt, dq])."""
    out = np.array(poses, np.float64, copy=True)
    for k in range(len(out)):
        R = out[k, :9].reshape(3, 3)
        t = out[k, 9:12]
        d = dx[6 * k:6 * k + 6]
        out[k, 9:12] = t + R @ d[:3]
        out[k, :9] = (R @ quat_rot(d[3:])).reshape(-1)
    return out


def optimize(prob, poses0, iters=10, lm=False, params=None, lam0=1e-4, anchor=0, pairs=None):
    """Gauss-Newton (lm=False) or Levenberg-Marquardt iterations.

    LM: a step is accepted if F decreases (lambda /= 10, floor 1e-12), else rejected
    (lambda *= 10).  GN: every step is taken.  Returns (poses, log)."""
    X = np.array(poses0, np.float64, copy=True)
    ev = evaluate(prob, X, params, pairs)
    lam = lam0 if lm else 0.0
    log = []
    for it in range(iters):
        dx, ok = solve_step(ev["H"], ev["b"], lam, anchor)
        if not ok:
            if not lm:
                raise np.linalg.LinAlgError("GN system not positive definite")
            lam *= 10.0
            log.append(dict(F=ev["F"], lam=lam, accepted=False, step=0.0, n_valid=ev["n_valid"]))
            continue
        Xc = boxplus(X, dx)
        evc = evaluate(prob, Xc, params, pairs)
        accept = (not lm) or (evc["F"] < ev["F"])
        if accept:
            X, ev = Xc, evc
            if lm:
                lam = max(lam / 10.0, 1e-12)
        else:
            lam *= 10.0
        log.append(dict(F=ev["F"], lam=lam, accepted=accept, step=float(np.linalg.norm(dx)),
                        n_valid=ev["n_valid"]))
    return X, log


# ------------------------------------------------------------------ normal estimation

def unproject_image(sen, D):
    """Points q = pi^-1(u, d) [H, W, 3] of a depth image in the sensor frame (Sec. III)."""
    H, W = D.shape
    r, c = np.mgrid[0:H, 0:W].astype(np.float64)
    d = np.asarray(D, np.float64)
    if sen["model"] == 0:
        return np.stack([d * (c - sen["cx"]) / sen["fx"], d * (r - sen["cy"]) / sen["fy"], d], -1)
    az, el = (c - sen["cx"]) / sen["fx"], (r - sen["cy"]) / sen["fy"]
    return np.stack([d * np.cos(el) * np.cos(az), d * np.cos(el) * np.sin(az), d * np.sin(el)], -1)


def estimate_normals(sen, D, radius_m=0.1, min_px=2.0, max_px=5.0, tau=0.5, min_count=5):
    """Sec. IV-A: the normal at u is the normal of the plane that best fits the unprojected
    neighbours u' with |u - u'| < tau_u, tau_u inversely proportional to the range at u, oriented
    towards the observer.  Readings: tau_u = clamp(radius_m |fx| / d(u), min_px, max_px) pixels (a
    fixed metric radius seen at range d, at least the 8-neighbourhood); neighbours need valid depth within tau of d(u) (no fit across a
    depth edge); best fit = least squares, i.e. the eigenvector of the smallest eigenvalue of the
    neighbours' covariance (library eigendecomposition); at least min_count points and a second
    eigenvalue above 1e-12 of the trace; oriented so that n . q_u < 0 (the sensor at the origin).
    Pixels without a normal get 0.  FP64; returns (normals FP32 [H, W, 3], has-normal mask,
    covariance eigenvalues [H, W, 3] ascending, neighbour counts)."""
    H, W = D.shape
    d = np.asarray(D, np.float64)
    valid = np.isfinite(d) & (d > 0) & (d >= sen["min_depth"]) & (d <= sen["max_depth"])
    q = unproject_image(sen, np.where(valid, d, 0.0))
    rad = np.where(valid, np.clip(radius_m * abs(sen["fx"]) / np.where(valid, d, 1.0), min_px, max_px), 0.0)
    R = int(np.floor(max_px))
    n = np.zeros((H, W))
    s1 = np.zeros((H, W, 3))
    s2 = np.zeros((H, W, 3, 3))
    for dy in range(-R, R + 1):
        for dx in range(-R, R + 1):
            dist = np.hypot(dx, dy)
            ys, xs = slice(max(0, -dy), min(H, H - dy)), slice(max(0, -dx), min(W, W - dx))
            yn, xn = slice(max(0, dy), min(H, H + dy)), slice(max(0, dx), min(W, W + dx))
            m = valid[ys, xs] & valid[yn, xn] & (dist < rad[ys, xs]) & (np.abs(d[yn, xn] - d[ys, xs]) <= tau)
            qq = np.where(m[..., None], q[yn, xn], 0.0)
            n[ys, xs] += m
            s1[ys, xs] += qq
            s2[ys, xs] += qq[..., :, None] * qq[..., None, :]
    cnt = np.maximum(n, 1)
    mean = s1 / cnt[..., None]
    cov = s2 / cnt[..., None, None] - mean[..., :, None] * mean[..., None, :]
    w, v = np.linalg.eigh(cov)
    nrm = v[..., :, 0]
    ok = valid & (n >= min_count) & (w[..., 1] > 1e-12 * np.maximum(np.trace(cov, axis1=-2, axis2=-1), 1e-300))
    flip = np.sum(nrm * q, -1) > 0
    nrm = np.where(flip[..., None], -nrm, nrm)
    return np.where(ok[..., None], nrm, 0.0).astype(np.float32), ok, w, n


# ------------------------------------------------------------------ image pyramid

def level_sensor(sen):
    """Intrinsics of the half-resolution level above `sen` (Sec. IV-A: each pyramid level has
    half the resolution of the one below).  Texel j of the new level covers texels 2j and 2j + 1
    of the old one, whose centres lie at 2j and 2j + 1, so the coordinates are related by
    u_old = 2 u_new + 1/2.  Both projections are affine in the image coordinates (pinhole K,
    spherical K_[1,2]), so the new level keeps the model with fx/2, fy/2, (cx - 1/2)/2,
    (cy - 1/2)/2 and floor(H/2) x floor(W/2) texels; depth limits and offset are unchanged."""
    out = dict(sen)
    out["H"], out["W"] = int(sen["H"]) // 2, int(sen["W"]) // 2
    out["fx"], out["fy"] = sen["fx"] / 2.0, sen["fy"] / 2.0
    out["cx"], out["cy"] = (sen["cx"] - 0.5) / 2.0, (sen["cy"] - 0.5) / 2.0
    return out


def downsample_keyframe(I, D, N, sen, tau):
    """One level up: each 2x2 block of texels becomes one (an odd last row or column is dropped).

    Depth: the block's mean if all four depths are valid (finite, inside the sensor's depth
    interval) and their spread max - min is at most tau, else no measurement (0): a block that
    straddles a depth edge has no single surface to stand for.  Intensity: the mean of the four.
    Normals: the mean of the four scaled to unit length.  Texels without depth get intensity and
    normal 0; they are never read (a source pixel needs depth, and so does every target tap).
    Means are taken in FP64 and rounded once to FP32."""
    H2, W2 = D.shape[0] // 2, D.shape[1] // 2
    d = np.asarray(D, np.float64)[:2 * H2, :2 * W2]
    ok = np.isfinite(d) & (d > 0) & (d >= sen["min_depth"]) & (d <= sen["max_depth"])
    blocks = lambda a: np.stack([a[0::2, 0::2], a[0::2, 1::2], a[1::2, 0::2], a[1::2, 1::2]], 0)
    db, okb = blocks(np.where(ok, d, 0.0)), blocks(ok)
    valid = okb.all(0) & ((db.max(0) - db.min(0)) <= tau)
    D2 = np.where(valid, db.sum(0) / 4.0, 0.0)
    I2 = np.where(valid, blocks(np.asarray(I, np.float64)[:2 * H2, :2 * W2]).sum(0) / 4.0, 0.0)
    N2 = np.zeros((H2, W2, 3))
    if N is not None:
        n = np.asarray(N, np.float64)[:2 * H2, :2 * W2]
        mean = np.stack([blocks(n[..., k]).sum(0) / 4.0 for k in range(3)], -1)
        norm = np.sqrt(np.sum(mean * mean, -1))
        good = valid & (norm > 0)
        N2[good] = mean[good] / norm[good][:, None]
    return I2.astype(np.float32), D2.astype(np.float32), N2.astype(np.float32)


def pyramid(prob, n_levels):
    """[level 0 (= prob), level 1, ...]: copies of the problem with downsampled keyframes and
    level intrinsics; poses and pairs are shared."""
    import copy
    levels = [prob]
    for _ in range(1, n_levels):
        lo = levels[-1]
        up = copy.copy(lo)
        up.sensors = [level_sensor(sn) for sn in lo.sensors]
        up.intensity, up.depth, up.normals = [], [], []
        for k in range(lo.n):
            sn = lo.sensors[lo.kf_sensor[k]]
            tau = lo.params["occ_tau_pinhole"] if sn["model"] == 0 else lo.params["occ_tau_spherical"]
            i2, d2, n2 = downsample_keyframe(lo.intensity[k], lo.depth[k],
                                             lo.normals[k] if lo.normals else None, sn, tau)
            up.intensity.append(i2)
            up.depth.append(d2)
            up.normals.append(n2)
        levels.append(up)
    return levels


def optimize_coarse_to_fine(prob, poses0, n_levels=3, iters=(2, 5, 10), rel_tol=1e-3, lm=True, params=None,
                            lam0=1e-4, anchor=0):
    """Sec. IV-C: optimise the coarsest level first and move one level finer when the error stops
    changing -- here when an accepted iteration lowers F by less than rel_tol relative, or after
    iters[level] iterations (iters[0] is the finest level).  LM (or GN) as in optimize(); lambda
    restarts at lam0 on every level.  Returns (poses, log) with the level in each log row."""
    levels = pyramid(prob, n_levels)
    X = np.array(poses0, np.float64, copy=True)
    log = []
    for lev in range(n_levels - 1, -1, -1):
        pl = levels[lev]
        ev = evaluate(pl, X, params)
        lam = lam0 if lm else 0.0
        for it in range(iters[lev]):
            dx, ok = solve_step(ev["H"], ev["b"], lam, anchor)
            if not ok:
                if not lm:
                    raise np.linalg.LinAlgError("GN system not positive definite")
                lam *= 10.0
                log.append(dict(level=lev, F=ev["F"], lam=lam, accepted=False, step=0.0))
                continue
            Xc = boxplus(X, dx)
            evc = evaluate(pl, Xc, params)
            accept = (not lm) or (evc["F"] < ev["F"])
            drop = (ev["F"] - evc["F"]) / ev["F"] if ev["F"] > 0 else 0.0
            if accept:
                X, ev = Xc, evc
                if lm:
                    lam = max(lam / 10.0, 1e-12)
            else:
                lam *= 10.0
            log.append(dict(level=lev, F=ev["F"], lam=lam, accepted=accept, step=float(np.linalg.norm(dx))))
            if accept and drop < rel_tol:
                break
    return X, log


# ------------------------------------------------------------------ pair graph

def pose_angle(Xa, Xb):
    """Rotation angle (rad) between the orientations of two poses: the angle of Ra^T Rb."""
    Ra, Rb = np.asarray(Xa[:9]).reshape(3, 3), np.asarray(Xb[:9]).reshape(3, 3)
    c = (np.trace(Ra.T @ Rb) - 1.0) / 2.0
    return float(np.arccos(np.clip(c, -1.0, 1.0)))


def build_pairs(prob, poses, max_angle=np.radians(30.0), max_dist=1.0, min_ratio=1.0 / 3.0, sequential=True,
                params=None):
    """Sec. IV-B: the matching pairs.  An ordered pair (s, t) of keyframes is kept if the angle
    between their orientations is below max_angle, the distance between their positions below
    max_dist, and the fraction of s's pixels with depth that reproject validly into t (n_valid /
    n_eval of the evaluation at `poses`) at least min_ratio; with `sequential`, (k, k + 1) and
    (k + 1, k) are kept whatever the criteria say (odometry-like links).  Returns int32 [P, 2] in
    (s, t) order and, for every ordered pair that passed the pose tests, its ratio."""
    X = np.asarray(poses, np.float64)
    n = prob.n
    kept, ratios = [], {}
    for s in range(n):
        for t in range(n):
            if s == t:
                continue
            seq = sequential and abs(s - t) == 1
            close = (pose_angle(X[s], X[t]) < max_angle and
                     np.linalg.norm(X[s, 9:] - X[t, 9:]) < max_dist)
            if close:
                r = eval_pair(prob, X, s, t, params)
                ratios[(s, t)] = r["n_valid"] / r["n_eval"] if r["n_eval"] > 0 else 0.0
            if seq or (close and ratios[(s, t)] >= min_ratio):
                kept.append((s, t))
    return np.array(kept, np.int32).reshape(-1, 2), ratios


# ------------------------------------------------------------------ trajectory error

def horn_align(P, Q):
    """Rigid (R, t) minimising sum |R P_k + t - Q_k|^2, Horn's unit-quaternion closed form."""
    P = np.asarray(P, np.float64)
    Q = np.asarray(Q, np.float64)
    mp, mq = P.mean(0), Q.mean(0)
    S = (P - mp).T @ (Q - mq)
    Sxx, Sxy, Sxz = S[0]
    Syx, Syy, Syz = S[1]
    Szx, Szy, Szz = S[2]
    N = np.array([
        [Sxx + Syy + Szz, Syz - Szy, Szx - Sxz, Sxy - Syx],
        [Syz - Szy, Sxx - Syy - Szz, Sxy + Syx, Szx + Sxz],
        [Szx - Sxz, Sxy + Syx, -Sxx + Syy - Szz, Syz + Szy],
        [Sxy - Syx, Szx + Sxz, Syz + Szy, -Sxx - Syy + Szz]])
    w, V = np.linalg.eigh(N)
    q0, qx, qy, qz = V[:, np.argmax(w)]
    R = np.array([
        [q0 * q0 + qx * qx - qy * qy - qz * qz, 2 * (qx * qy - q0 * qz), 2 * (qx * qz + q0 * qy)],
        [2 * (qy * qx + q0 * qz), q0 * q0 - qx * qx + qy * qy - qz * qz, 2 * (qy * qz - q0 * qx)],
        [2 * (qz * qx - q0 * qy), 2 * (qz * qy + q0 * qx), q0 * q0 - qx * qx - qy * qy + qz * qz]])
    t = mq - R @ mp
    return R, t


def ate_rmse(est_poses, gt_poses):
    """RMSE of translational differences after Horn SE(3) alignment (Sec. V)."""
    P = np.asarray(est_poses)[:, 9:12]
    Q = np.asarray(gt_poses)[:, 9:12]
    R, t = horn_align(P, Q)
    d = (P @ R.T + t) - Q
    return float(np.sqrt(np.mean(np.sum(d * d, axis=1))))


# ------------------------------------------------------------------ loss and its gradient

def quat_right_jacobian(dq):
    """L(q) with R(q + dq') = R(q) R(L(q) dq') to first order: the body-frame quaternion increment
    vec(Q* (x) dQ) of the unit quaternion Q = (w, q), w = sqrt(1 - |q|^2)."""
    q = np.asarray(dq, np.float64)
    w = math.sqrt(1.0 - float(q @ q))
    S = np.array([[0, -q[2], q[1]], [q[2], 0, -q[0]], [-q[1], q[0], 0]])
    return w * np.eye(3) + np.outer(q, q) / w - S


def loss_and_grad(prob, poses0, delta, params=None, pairs=None):
    """F(X0 boxplus delta) = sum of rho over pairs and valid pixels, and its exact gradients.

    delta: [N, 6] per pose [dt, dq] (per pose variable when prob.pose_of is set).  Returns
    dict(F, g_delta [N,6], gI, gD, gN per keyframe).
    The derivative of F is taken with the slope of the bilinear interpolant (the sampled images
    are what F depends on); masks and integer cells are those of the evaluation at X."""
    lib = _load()
    params = prob.params if params is None else params
    pairs = prob.pairs if pairs is None else np.asarray(pairs, np.int32)
    pose_of = getattr(prob, "pose_of", None)
    nv = prob.n if pose_of is None else int(np.max(pose_of)) + 1
    var = np.arange(prob.n) if pose_of is None else np.asarray(pose_of)
    delta = np.asarray(delta, np.float64).reshape(nv, 6)
    X = boxplus(poses0, delta.reshape(-1))[var]
    gI = [np.zeros(prob.depth[k].shape) for k in range(prob.n)]
    gD = [np.zeros(prob.depth[k].shape) for k in range(prob.n)]
    gN = [np.zeros(prob.depth[k].shape + (3,)) for k in range(prob.n)]
    b = np.zeros(6 * nv)
    F = 0.0
    for (s, t) in pairs:
        s, t = int(s), int(t)
        ss, st = prob.sensors[prob.kf_sensor[s]], prob.sensors[prob.kf_sensor[t]]
        imgs = [_c(a, np.float32) for a in (prob.intensity[s], prob.depth[s], prob.normals[s],
                                             prob.intensity[t], prob.depth[t], prob.normals[t])]
        ig = OrcImageGrad(gI[s].ctypes.data, gD[s].ctypes.data, gN[s].ctypes.data,
                          gI[t].ctypes.data, gD[t].ctypes.data, gN[t].ctypes.data)
        out = OrcPairOut()
        Xs, Xt = _c(X[s], np.float64), _c(X[t], np.float64)
        rc = lib.orc_eval_pair_grad(ctypes.byref(sensor_struct(ss)), imgs[0].ctypes.data, imgs[1].ctypes.data,
                                    imgs[2].ctypes.data, ctypes.byref(sensor_struct(st)), imgs[3].ctypes.data,
                                    imgs[4].ctypes.data, imgs[5].ctypes.data, Xs.ctypes.data, Xt.ctypes.data,
                                    ctypes.byref(params_struct(params, st["model"], 1)), None, None,
                                    ctypes.byref(out), None, None, None, None, None, ctypes.byref(ig))
        if rc != 0:
            raise RuntimeError("orc_eval_pair_grad failed (%d)" % rc)
        F += out.F
        bb = np.array(out.b)
        b[6 * var[s]:6 * var[s] + 6] += bb[:6]
        b[6 * var[t]:6 * var[t] + 6] += bb[6:]
    # dF/d(right perturbation at X) = 2 b; chain rule through X0 boxplus delta
    g = np.zeros((nv, 6))
    for k in range(nv):
        q = delta[k, 3:]
        g[k, :3] = quat_rot(q) @ (2.0 * b[6 * k:6 * k + 3])
        g[k, 3:] = quat_right_jacobian(q).T @ (2.0 * b[6 * k + 3:6 * k + 6])
    return dict(F=F, g_delta=g, gI=gI, gD=gD, gN=gN)
