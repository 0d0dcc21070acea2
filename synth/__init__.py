"""Seeded synthetic keyframe generator shared by the tests, the oracle checks and bench.py.

The scenes stand in for the paper's workloads (Sec. V): an RGB-D camera in a
cluttered room (ETH3D-like, 640x480) and a 128- or 64-beam spinning LiDAR
driving a 2 km loop between buildings (Newer College / OS0-128-like).  None of
those datasets is used; everything here is procedural and seeded.

This module renders inputs only.  It contains none of the bundle-adjustment
arithmetic (warp, sampling of keyframes, residuals, Jacobians, reductions,
solve or pose update): the oracle and the HIP library each implement those on
their own.  Random numbers the method itself would draw do not exist; the only
randomness is in the scene, the trajectory, the image noise and the initial
pose perturbation, all fixed by the seed.

Pose convention: a pose is 12 float64 numbers, row-major R (3x3) then t, and
maps the platform frame to the world frame (p_w = R p + t).  A sensor offset
maps the sensor frame to the platform frame in the same layout.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None

NSIN = 8
PINHOLE, SPHERICAL = 0, 1

RECT_DTYPE = np.dtype([
    ("c", "f8", 3), ("e1", "f8", 3), ("e2", "f8", 3), ("n", "f8", 3),
    ("h1", "f8"), ("h2", "f8"), ("radius", "f8"), ("tex", "f8", (NSIN, 4)),
])


class _Cam(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int), ("H", ctypes.c_int), ("W", ctypes.c_int),
                ("fx", ctypes.c_double), ("fy", ctypes.c_double), ("cx", ctypes.c_double),
                ("cy", ctypes.c_double), ("max_depth", ctypes.c_double)]


def build_lib(force: bool = False) -> str:
    """Compile the ray-caster (gcc, OpenMP) next to this file."""
    src = os.path.join(_HERE, "raycast.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_lib()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.synth_render.restype = ctypes.c_int
        lib.synth_render.argtypes = [
            ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(_Cam),
            ctypes.c_int, ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
            ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


# ------------------------------------------------------------------ geometry helpers

def rot_axis_angle(axis, angle):
    """Rodrigues rotation (generator-side; used to build and perturb poses)."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * (K @ K)


def pose_to_mat(p):
    p = np.asarray(p, dtype=np.float64)
    T = np.eye(4)
    T[:3, :3] = p[:9].reshape(3, 3)
    T[:3, 3] = p[9:12]
    return T


def mat_to_pose(T):
    return np.concatenate([T[:3, :3].reshape(-1), T[:3, 3]])


def _orthonormal_frame(normal, rng):
    n = normal / np.linalg.norm(normal)
    a = rng.normal(size=3)
    a -= a.dot(n) * n
    e1 = a / np.linalg.norm(a)
    e2 = np.cross(n, e1)
    return e1, e2, n


def _random_texture(rng):
    t = np.zeros((NSIN, 4))
    f = rng.uniform(0.5, 4.0, NSIN)
    th = rng.uniform(0, 2 * np.pi, NSIN)
    t[:, 0] = f * np.cos(th)
    t[:, 1] = f * np.sin(th)
    t[:, 2] = rng.uniform(0, 2 * np.pi, NSIN)
    t[:, 3] = rng.uniform(0.5, 1.0, NSIN)
    return t


def _rect(c, e1, e2, h1, h2, tex):
    r = np.zeros((), dtype=RECT_DTYPE)
    r["c"] = c
    r["e1"] = e1
    r["e2"] = e2
    r["n"] = np.cross(e1, e2)
    r["h1"] = h1
    r["h2"] = h2
    r["radius"] = math.hypot(h1, h2)
    r["tex"] = tex
    return r


# ------------------------------------------------------------------ sensors

def pinhole_sensor(H, W, fx, fy, cx, cy, min_depth=0.1, max_depth=10.0, offset=None):
    return dict(model=PINHOLE, H=H, W=W, fx=fx, fy=fy, cx=cx, cy=cy, min_depth=min_depth,
                max_depth=max_depth,
                offset=np.array(offset if offset is not None else [1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0],
                                dtype=np.float64))


def spherical_sensor(H, W, el_up_deg=8.0, el_down_deg=-25.0, min_depth=0.5, max_depth=80.0,
                     offset=None):
    """Spherical (LiDAR) intrinsics: column 0 looks at azimuth +pi, row 0 at the top elevation."""
    up, dn = math.radians(el_up_deg), math.radians(el_down_deg)
    fx = -W / (2 * math.pi)
    cx = W / 2.0
    fy = -(H - 1) / (up - dn)
    cy = (H - 1) * up / (up - dn)
    return dict(model=SPHERICAL, H=H, W=W, fx=fx, fy=fy, cx=cx, cy=cy, min_depth=min_depth,
                max_depth=max_depth,
                offset=np.array(offset if offset is not None else [1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0],
                                dtype=np.float64))


# ------------------------------------------------------------------ problem container

@dataclass
class Problem:
    name: str
    sensors: list
    kf_sensor: np.ndarray          # int32 [N]
    gt_poses: np.ndarray           # float64 [N,12] platform -> world
    init_poses: np.ndarray         # float64 [N,12]
    pairs: np.ndarray              # int32 [P,2] (source, target)
    params: dict
    intensity: list = field(default_factory=list)   # per keyframe float32 [H,W] (None if not rendered)
    depth: list = field(default_factory=list)
    normals: list = field(default_factory=list)     # float32 [H,W,3]
    scene: dict = field(default_factory=dict)
    # keyframe -> pose variable (several sensors of one rig frame share a pose); None: one pose
    # per keyframe.  With it, gt_poses / init_poses hold one pose per variable.
    pose_of: np.ndarray = None

    @property
    def n(self):
        return len(self.kf_sensor)

    @property
    def n_poses(self):
        return self.n if self.pose_of is None else int(np.max(self.pose_of)) + 1

    def kf_poses(self, X):
        """Per-keyframe poses from per-variable poses."""
        X = np.asarray(X, np.float64)
        return X if self.pose_of is None else X[np.asarray(self.pose_of)]

    def subset(self, kfs):
        """Problem restricted to keyframes `kfs` (re-indexed), keeping pairs among them."""
        kfs = list(kfs)
        remap = {k: i for i, k in enumerate(kfs)}
        pairs = np.array([(remap[s], remap[t]) for s, t in self.pairs if s in remap and t in remap],
                         np.int32).reshape(-1, 2)
        assert self.pose_of is None, "subset of a problem with shared poses"
        sub = Problem(self.name + "_sub", self.sensors, self.kf_sensor[kfs].copy(), self.gt_poses[kfs].copy(),
                      self.init_poses[kfs].copy(), pairs, dict(self.params), scene=self.scene)
        if self.intensity:
            sub.intensity = [self.intensity[k] for k in kfs]
            sub.depth = [self.depth[k] for k in kfs]
            sub.normals = [self.normals[k] for k in kfs]
        return sub

    def px_pairs_upper(self):
        return int(sum(self.sensors[self.kf_sensor[s]]["H"] * self.sensors[self.kf_sensor[s]]["W"]
                       for s, _ in self.pairs))


def _sensor_pose(platform_pose, offset):
    return mat_to_pose(pose_to_mat(platform_pose) @ pose_to_mat(offset))


def render(prob: Problem, kfs=None, noise=True, poses=None):
    """Render keyframes `kfs` (default all) into prob.intensity/depth/normals."""
    lib = _load()
    N = prob.n
    if not prob.intensity:
        prob.intensity = [None] * N
        prob.depth = [None] * N
        prob.normals = [None] * N
    kfs = list(range(N)) if kfs is None else list(kfs)
    poses = prob.kf_poses(prob.gt_poses if poses is None else poses)
    sc = prob.scene
    rects = np.ascontiguousarray(sc["rects"])
    gtex = np.ascontiguousarray(sc["ground_tex"], dtype=np.float64)
    for sid, sen in enumerate(prob.sensors):
        ks = [k for k in kfs if prob.kf_sensor[k] == sid]
        if not ks:
            continue
        H, W = sen["H"], sen["W"]
        cam = _Cam(sen["model"], H, W, sen["fx"], sen["fy"], sen["cx"], sen["cy"], sen["max_depth"])
        sp = np.ascontiguousarray(np.stack([_sensor_pose(poses[k], sen["offset"]) for k in ks]))
        # render in chunks so the same keyframe gets the same noise whatever the subset
        for k, spk in zip(ks, sp):
            I = np.empty((H, W), np.float32)
            D = np.empty((H, W), np.float32)
            Nn = np.empty((H, W, 3), np.float32)
            spk = np.ascontiguousarray(spk[None])
            rc = lib.synth_render(rects.ctypes.data, len(rects), int(sc["ground"]), gtex.ctypes.data,
                                  ctypes.byref(cam), 1, spk.ctypes.data,
                                  sc["noise_i"] if noise else 0.0, sc["noise_d"] if noise else 0.0,
                                  int(sc["seed"]), int(k), I.ctypes.data, D.ctypes.data, Nn.ctypes.data)
            if rc != 0:
                raise RuntimeError("synth_render failed")
            prob.intensity[k], prob.depth[k], prob.normals[k] = I, D, Nn
    return prob


def _perturb(gt, rng, mag_t, mag_r_deg, anchor=0):
    out = gt.copy()
    for k in range(len(gt)):
        if k == anchor:
            continue
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        ax = rng.normal(size=3)
        dT = np.eye(4)
        dT[:3, :3] = rot_axis_angle(ax, math.radians(mag_r_deg))
        dT[:3, 3] = mag_t * d
        out[k] = mat_to_pose(pose_to_mat(gt[k]) @ dT)
    return out


def _look_frame_camera(forward, up=(0, 0, 1)):
    """Pinhole camera axes (x right, y down, z forward) as columns of R."""
    f = np.asarray(forward, np.float64)
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, np.float64))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    return np.stack([r, d, f], axis=1)


def _look_frame_lidar(forward, up=(0, 0, 1)):
    """LiDAR axes (x forward, y left, z up) as columns of R."""
    f = np.asarray(forward, np.float64)
    u = np.asarray(up, np.float64)
    f = f - f.dot(u) * u
    f /= np.linalg.norm(f)
    left = np.cross(u, f)
    return np.stack([f, left, u], axis=1)


DEFAULT_PARAMS = dict(omega_intensity=1.0, omega_depth=1.0, omega_normal=1.0, huber_delta=0.1,
                      occ_tau_pinhole=0.5, occ_tau_spherical=1.0, anchor=0)


# ------------------------------------------------------------------ configs

def rgbd_small(seed=1, H=120, W=160, n_kf=5):
    """Five 160x120 RGB-D keyframes on a 1 m arc looking into a 6 m box of 50 textured rectangles."""
    rng = np.random.default_rng(seed)
    scale = W / 160.0
    sen = pinhole_sensor(H, W, 120.0 * scale, 120.0 * scale, 80.0 * scale, 60.0 * (H / 120.0),
                         min_depth=0.1, max_depth=20.0)
    # poses: radius 2 m around the origin, 1 m of arc, looking at the centre
    span = 1.0 / 2.0
    th = np.linspace(-span / 2, span / 2, n_kf) + rng.uniform(0, 2 * np.pi)
    gt = []
    for a in th:
        pos = np.array([2.0 * math.cos(a), 2.0 * math.sin(a), 0.0])
        R = _look_frame_camera(-pos)
        gt.append(np.concatenate([R.reshape(-1), pos]))
    gt = np.array(gt)
    rects = []
    while len(rects) < 50:
        c = rng.uniform(-3, 3, 3)
        e1, e2, n = _orthonormal_frame(rng.normal(size=3), rng)
        h1, h2 = rng.uniform(0.25, 1.25, 2)
        if np.min(np.linalg.norm(gt[:, 9:] - c, axis=1)) < math.hypot(h1, h2) + 0.4:
            continue
        rects.append(_rect(c, e1, e2, h1, h2, _random_texture(rng)))
    # enclosing walls of the box so every ray returns
    L = 4.0
    for ax in range(3):
        for sgn in (-1, 1):
            n = np.zeros(3)
            n[ax] = -sgn
            c = np.zeros(3)
            c[ax] = sgn * L
            e1 = np.zeros(3)
            e1[(ax + 1) % 3] = 1
            e2 = np.cross(n, e1)
            rects.append(_rect(c, e1, e2, L, L, _random_texture(rng)))
    rects = np.array(rects, dtype=RECT_DTYPE)
    pairs = np.array([(i, j) for i in range(n_kf) for j in range(n_kf) if i != j], np.int32)
    init = _perturb(gt, np.random.default_rng(100 + 0), 0.05, 2.0)
    params = dict(DEFAULT_PARAMS, channels=2, iterations=10, lm=False)
    scene = dict(rects=rects, ground=0, ground_tex=np.zeros((NSIN, 4)), noise_i=0.01, noise_d=0.005,
                 seed=seed)
    return Problem("rgbd_small", [sen], np.zeros(n_kf, np.int32), gt, init, pairs, params, scene=scene)


def _closed_curve(n, length, ax, by, wig, rng, p=2.0):
    """Closed planar curve of the given length: superellipse with seeded wiggles."""
    t = np.linspace(0, 2 * np.pi, 20001)[:-1]
    c, s = np.cos(t), np.sin(t)
    x = ax * np.sign(c) * np.abs(c) ** (2.0 / p)
    y = by * np.sign(s) * np.abs(s) ** (2.0 / p)
    for (amp, k, ph) in wig:
        x = x + amp * np.sin(k * t + ph)
        y = y + amp * np.cos((k + 1) * t + 0.7 * ph)
    pts = np.stack([x, y], 1)
    seg = np.linalg.norm(np.diff(np.vstack([pts, pts[:1]]), axis=0), axis=1)
    L = seg.sum()
    pts = pts * (length / L)
    seg = seg * (length / L)
    cum = np.concatenate([[0], np.cumsum(seg)])
    return pts, cum


def _sample_curve(pts, cum, s):
    L = cum[-1]
    s = np.mod(s, L)
    i = np.searchsorted(cum, s, side="right") - 1
    i = np.clip(i, 0, len(pts) - 1)
    j = (i + 1) % len(pts)
    f = (s - cum[i]) / np.maximum(cum[i + 1] - cum[i], 1e-12)
    p = pts[i] * (1 - f)[:, None] + pts[j] * f[:, None]
    tan = pts[j] - pts[i]
    tan /= np.linalg.norm(tan, axis=1, keepdims=True)
    return p, tan


def rgbd_room(seed=2, H=480, W=640, n_kf=100, knn=10):
    """640x480 RGB-D keyframes along a 30 m smooth path in a room with 300 textured planes."""
    rng = np.random.default_rng(seed)
    sen = pinhole_sensor(H, W, 525.0 * W / 640, 525.0 * W / 640, (W - 1) / 2.0, (H - 1) / 2.0,
                         min_depth=0.1, max_depth=10.0)
    pts, cum = _closed_curve(n_kf, 30.0, 5.5, 3.5,
                             [(0.4, 3, rng.uniform(0, 6.28)), (0.3, 5, rng.uniform(0, 6.28))], rng)
    s = np.arange(n_kf) * (30.0 / n_kf)
    p2, tan = _sample_curve(pts, cum, s)
    gt = []
    for k in range(n_kf):
        z = 1.5 + 0.2 * math.sin(2 * math.pi * s[k] / 30.0 * 2)
        yaw = math.radians(20.0) * math.sin(2 * math.pi * s[k] / 30.0 * 3)
        f = np.array([tan[k, 0], tan[k, 1], 0.0])
        f = rot_axis_angle([0, 0, 1], yaw) @ f
        f[2] = math.tan(math.radians(-5.0 * math.cos(2 * math.pi * s[k] / 10.0)))
        R = _look_frame_camera(f)
        gt.append(np.concatenate([R.reshape(-1), [p2[k, 0], p2[k, 1], z]]))
    gt = np.array(gt)
    hx, hy, hz = 8.0, 6.0, 3.0
    rects = []
    while len(rects) < 300:
        c = np.array([rng.uniform(-hx + 0.5, hx - 0.5), rng.uniform(-hy + 0.5, hy - 0.5), rng.uniform(0.3, 2.7)])
        e1, e2, n = _orthonormal_frame(rng.normal(size=3), rng)
        h1, h2 = rng.uniform(0.15, 0.75, 2)
        if np.min(np.linalg.norm(gt[:, 9:] - c, axis=1)) < math.hypot(h1, h2) + 0.6:
            continue
        rects.append(_rect(c, e1, e2, h1, h2, _random_texture(rng)))
    box = [((0, 0, 0), (1, 0, 0), (0, 1, 0), hx, hy),     # floor
           ((0, 0, hz), (0, 1, 0), (1, 0, 0), hy, hx),    # ceiling (normal -z)
           ((hx, 0, hz / 2), (0, 0, 1), (0, 1, 0), hz / 2, hy),
           ((-hx, 0, hz / 2), (0, 1, 0), (0, 0, 1), hy, hz / 2),
           ((0, hy, hz / 2), (1, 0, 0), (0, 0, 1), hx, hz / 2),
           ((0, -hy, hz / 2), (0, 0, 1), (1, 0, 0), hz / 2, hx)]
    for c, e1, e2, a, b in box:
        rects.append(_rect(np.array(c, float), np.array(e1, float), np.array(e2, float), a, b,
                           _random_texture(rng)))
    rects = np.array(rects, dtype=RECT_DTYPE)
    pos = gt[:, 9:]
    d = np.linalg.norm(pos[:, None] - pos[None], axis=2)
    pairs = []
    for k in range(n_kf):
        order = np.argsort(d[k], kind="stable")
        for j in [j for j in order if j != k][:knn]:
            pairs.append((k, j))
    pairs = np.array(pairs, np.int32)
    init = _perturb(gt, np.random.default_rng(100 + 1), 0.1, 3.0)
    params = dict(DEFAULT_PARAMS, channels=5, iterations=10, lm=True)
    scene = dict(rects=rects, ground=0, ground_tex=np.zeros((NSIN, 4)), noise_i=0.01, noise_d=0.005,
                 seed=seed)
    return Problem("rgbd_room", [sen], np.zeros(n_kf, np.int32), gt, init, pairs, params, scene=scene)


def _driving_world(rng, n_struct, length=2000.0):
    pts, cum = _closed_curve(0, length, 400.0, 200.0,
                             [(15.0, 3, rng.uniform(0, 6.28)), (8.0, 7, rng.uniform(0, 6.28))], rng, p=4.0)
    rects = []
    s = rng.uniform(0, length, n_struct)
    p2, tan = _sample_curve(pts, cum, s)
    for i in range(n_struct):
        side = 1.0 if rng.uniform() < 0.5 else -1.0
        nrm = np.array([-tan[i, 1], tan[i, 0]]) * side
        yaw_t = math.atan2(tan[i, 1], tan[i, 0])
        tex = _random_texture
        if rng.uniform() < 0.7:   # box: 4 sides + roof
            a, b = rng.uniform(1.0, 5.0, 2)
            h = rng.uniform(2.0, 12.0)
            lat = max(rng.uniform(5.0, 40.0), 3.5 + math.hypot(a, b))
            cxy = p2[i] + lat * nrm
            yaw = yaw_t + rng.uniform(-0.5, 0.5)
            ex = np.array([math.cos(yaw), math.sin(yaw), 0.0])
            ey = np.array([-math.sin(yaw), math.cos(yaw), 0.0])
            ez = np.array([0.0, 0.0, 1.0])
            c0 = np.array([cxy[0], cxy[1], h / 2])
            for (ax, half, o1, h1) in ((ex, a, ey, b), (ey, b, ex, a)):
                for sg in (-1, 1):
                    c = c0 + sg * half * ax
                    n = sg * ax
                    e1 = np.cross(ez, n)
                    rects.append(_rect(c, e1, ez, h1, h / 2, tex(rng)))
            rects.append(_rect(c0 + ez * h / 2, ex, ey, a, b, tex(rng)))
        else:                      # free-standing wall
            L2 = rng.uniform(2.5, 10.0)
            h = rng.uniform(2.0, 8.0)
            lat = max(rng.uniform(5.0, 40.0), 3.5 + L2)
            cxy = p2[i] + lat * nrm
            yaw = yaw_t + rng.normal(0, math.radians(15.0))
            e1 = np.array([math.cos(yaw), math.sin(yaw), 0.0])
            rects.append(_rect(np.array([cxy[0], cxy[1], h / 2]), e1, np.array([0.0, 0.0, 1.0]), L2, h / 2,
                               tex(rng)))
    return pts, cum, np.array(rects, dtype=RECT_DTYPE)


def lidar_loop(name, seed, H, W, n_kf, radius=30.0, n_struct=5000, length=2000.0):
    rng = np.random.default_rng(seed)
    sen = spherical_sensor(H, W)
    pts, cum, rects = _driving_world(rng, n_struct, length)
    s = np.arange(n_kf) * (length / n_kf)
    p2, tan = _sample_curve(pts, cum, s)
    gt = []
    for k in range(n_kf):
        R = _look_frame_lidar([tan[k, 0], tan[k, 1], 0.0])
        gt.append(np.concatenate([R.reshape(-1), [p2[k, 0], p2[k, 1], 1.8]]))
    gt = np.array(gt)
    pos = gt[:, 9:]
    d = np.linalg.norm(pos[:, None] - pos[None], axis=2)
    pairs = np.array([(i, j) for i in range(n_kf) for j in range(n_kf) if i != j and d[i, j] < radius],
                     np.int32)
    # 0.05 m / 1 deg: inside the single-resolution photometric basin at 128x2048 (a 3 deg start
    # stalls without a coarse-to-fine pyramid)
    init = _perturb(gt, np.random.default_rng(100 + seed), 0.05, 1.0)
    params = dict(DEFAULT_PARAMS, channels=5, iterations=10, lm=True)
    scene = dict(rects=rects, ground=1, ground_tex=_random_texture(rng), noise_i=0.01, noise_d=0.01,
                 seed=seed)
    return Problem(name, [sen], np.zeros(n_kf, np.int32), gt, init, pairs, params, scene=scene)


def lidar64(seed=3, **kw):
    """64x1024 spherical LiDAR, 500 keyframes on a 2 km loop, pairs within 30 m."""
    kw.setdefault("H", 64)
    kw.setdefault("W", 1024)
    kw.setdefault("n_kf", 500)
    return lidar_loop("lidar64", seed, **kw)


def lidar128(seed=4, **kw):
    """128x2048 spherical LiDAR, 300 keyframes on a 2 km loop, pairs within 30 m."""
    kw.setdefault("H", 128)
    kw.setdefault("W", 2048)
    kw.setdefault("n_kf", 300)
    return lidar_loop("lidar128", seed, **kw)


def joint(seed=5, n_lidar=200, n_rgbd=400, H_l=128, W_l=1024, H_c=480, W_c=640, radius=20.0, length=2000.0,
          n_struct=5000):
    """Joint LiDAR + RGB-D rig on the 2 km driving loop: a spherical LiDAR (el -25..+8 deg) and a
    forward-looking pinhole camera (fx = fy = 525 at 640x480, scaled with the size) mounted on one
    platform with fixed seeded extrinsics (sensor -> platform offsets).  n_lidar LiDAR keyframes
    and n_rgbd camera keyframes spaced along the loop; every ordered pair of keyframes within
    `radius` metres is used, same-sensor and cross-sensor alike."""
    rng = np.random.default_rng(seed)
    pts, cum, rects = _driving_world(rng, n_struct, length)
    # extrinsics: LiDAR 0.3 m above the platform origin; camera forward-looking with a small
    # seeded misalignment, 0.2 m ahead
    lid_off = np.concatenate([np.eye(3).reshape(-1), [0.0, 0.0, 0.3]])
    Rc = np.array([[0.0, 0.0, 1.0], [-1.0, 0.0, 0.0], [0.0, -1.0, 0.0]])     # columns: right, down, forward
    Rc = rot_axis_angle(rng.normal(size=3), math.radians(2.0)) @ Rc
    cam_off = np.concatenate([Rc.reshape(-1), [0.2, rng.uniform(-0.1, 0.1), 0.1]])
    sc = W_c / 640.0
    lid = spherical_sensor(H_l, W_l, offset=lid_off)
    cam = pinhole_sensor(H_c, W_c, 525.0 * sc, 525.0 * sc, (W_c - 1) / 2.0, (H_c - 1) / 2.0, min_depth=0.3,
                         max_depth=40.0, offset=cam_off)
    s_l = np.arange(n_lidar) * (length / max(n_lidar, 1))
    s_c = (np.arange(n_rgbd) + 0.5) * (length / max(n_rgbd, 1))
    p2, tan = _sample_curve(pts, cum, np.concatenate([s_l, s_c]))
    gt = []
    for k in range(len(p2)):
        R = _look_frame_lidar([tan[k, 0], tan[k, 1], 0.0])
        gt.append(np.concatenate([R.reshape(-1), [p2[k, 0], p2[k, 1], 1.5]]))
    gt = np.array(gt)
    kf_sensor = np.array([0] * n_lidar + [1] * n_rgbd, np.int32)
    pos = gt[:, 9:]
    d = np.linalg.norm(pos[:, None] - pos[None], axis=2)
    n = len(gt)
    pairs = np.array([(i, j) for i in range(n) for j in range(n) if i != j and d[i, j] < radius], np.int32)
    init = _perturb(gt, np.random.default_rng(100 + seed), 0.05, 1.0)
    params = dict(DEFAULT_PARAMS, channels=5, iterations=20, lm=True)
    scene = dict(rects=rects, ground=1, ground_tex=_random_texture(rng), noise_i=0.01, noise_d=0.01, seed=seed)
    return Problem("joint", [lid, cam], kf_sensor, gt, init, pairs, params, scene=scene)


def rig_pair(seed=5, H_l=64, W_l=512, H_c=240, W_c=320, station=300.0, perturb_t=0.1, perturb_deg=3.0,
             perturb_seed=0):
    """One frame of the joint LiDAR + RGB-D rig (the joint loop's world and extrinsics) and a copy
    of it: keyframes [LiDAR, camera] of frame 0 and the same images again as frame 1, each frame
    one pose variable (pose_of = [0, 0, 1, 1]).  Frame 0 is held at the true pose; frame 1 starts
    from it moved by perturb_t metres and perturb_deg degrees in seeded directions, so aligning the
    frame to itself should return the identity.  Pairs: LiDAR 0 <-> 2, camera 1 <-> 3."""
    base = joint(seed=seed, n_lidar=1, n_rgbd=1, H_l=H_l, W_l=W_l, H_c=H_c, W_c=W_c)
    # the platform at `station` metres along the loop
    rng = np.random.default_rng(seed)
    pts, cum, _ = _driving_world(rng, 5000, 2000.0)
    p2, tan = _sample_curve(pts, cum, np.array([station]))
    X = np.concatenate([_look_frame_lidar([tan[0, 0], tan[0, 1], 0.0]).reshape(-1), [p2[0, 0], p2[0, 1], 1.5]])
    gt = np.array([X, X])
    init = _perturb(gt, np.random.default_rng(1000 + perturb_seed), perturb_t, perturb_deg, anchor=0)
    prob = Problem("rig_pair", base.sensors, np.array([0, 1, 0, 1], np.int32), gt, init,
                   np.array([(0, 2), (2, 0), (1, 3), (3, 1)], np.int32), dict(base.params, iterations=30),
                   scene=base.scene, pose_of=np.array([0, 0, 1, 1], np.int32))
    prob._copy_images = {2: 0, 3: 1}
    return prob


def plane_pair(model="pinhole", seed=7):
    """One large textured plane seen by three keyframes; keyframe 0 is the only source and keeps
    depth only in a central window (outside it the depth is 0, i.e. no measurement), keyframes 1 and 2 are targets whose whole view is the plane.  With small pose
    offsets every source pixel warps well inside the targets and no tap meets a depth edge, so the
    set of valid correspondences does not change under small pose steps (a fixture for finite
    differences of the loss with respect to the poses)."""
    rng = np.random.default_rng(seed)
    if model == "pinhole":
        sen = pinhole_sensor(96, 128, 100.0, 100.0, 64.0, 48.0, min_depth=0.1, max_depth=20.0)
        fwd = np.array([0.0, 1.0, 0.0])
        c = np.array([0.0, 3.0, 0.0])
        look = _look_frame_camera
        h1 = h2 = 6.0
        margin = (0.25, 0.25)
    else:
        sen = spherical_sensor(32, 512, el_up_deg=8.0, el_down_deg=-25.0, min_depth=0.5, max_depth=40.0)
        fwd = np.array([1.0, 0.0, 0.0])
        c = np.array([8.0, 0.0, -1.5])
        look = _look_frame_lidar
        h1, h2 = 30.0, 8.0
        margin = (0.25, 0.42)
    # plane facing the sensors: e1 horizontal, e2 = n x e1
    e1 = np.array([1.0, 0.0, 0.0]) if model == "pinhole" else np.array([0.0, 1.0, 0.0])
    e2 = np.cross(-fwd, e1)
    rect = _rect(c, e1, e2, h1, h2, _random_texture(rng))
    gt = []
    for k in range(3):
        pos = np.array([0.0, 0.0, 0.0]) + 0.15 * np.array([math.cos(2.1 * k), 0.0, math.sin(2.1 * k)]) * (k > 0)
        pos = pos if model == "pinhole" else pos[[1, 0, 2]]
        gt.append(np.concatenate([look(fwd).reshape(-1), pos]))
    gt = np.array(gt)
    init = _perturb(gt, np.random.default_rng(200 + seed), 0.02, 0.5, anchor=-1)
    params = dict(DEFAULT_PARAMS, channels=5, iterations=5, lm=False)
    scene = dict(rects=np.array([rect], dtype=RECT_DTYPE), ground=0, ground_tex=np.zeros((NSIN, 4)), noise_i=0.01,
                 noise_d=0.005, seed=seed)
    prob = Problem("plane_pair_" + model, [sen], np.zeros(3, np.int32), gt, init,
                   np.array([(0, 1), (0, 2)], np.int32), params, scene=scene)
    prob._source_margin = margin
    return prob


def _mask_source(prob):
    m = getattr(prob, "_source_margin", None)
    if m is None or not prob.depth or prob.depth[0] is None:
        return prob
    H, W = prob.depth[0].shape
    keep = np.zeros((H, W), bool)
    keep[int(m[0] * H):H - int(m[0] * H), int(m[1] * W):W - int(m[1] * W)] = True
    prob.depth[0] = np.where(keep, prob.depth[0], np.float32(0.0)).astype(np.float32)
    return prob


CONFIGS = {"rgbd_small": rgbd_small, "rgbd_room": rgbd_room, "lidar64": lidar64, "lidar128": lidar128, "joint": joint,
           "plane_pair": plane_pair, "rig_pair": rig_pair}


def make(name, render_images=True, noise=True, kfs=None, **kw):
    prob = CONFIGS[name](**kw)
    if render_images:
        copies = getattr(prob, "_copy_images", {})
        render(prob, kfs=[k for k in (range(prob.n) if kfs is None else kfs) if k not in copies], noise=noise)
        for k, src in copies.items():
            prob.intensity[k], prob.depth[k], prob.normals[k] = prob.intensity[src], prob.depth[src], prob.normals[src]
        _mask_source(prob)
    return prob
