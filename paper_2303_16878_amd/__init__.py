"""Python binding of libpba, the MI355X photometric bundle-adjustment library.

The names mirror the C ABI in include/pba.h; this module only marshals
arguments through ctypes.  Every step of the computation runs in the HIP
kernels of libpba.so; if the library is not built, importing the binding's
entry points raises instead of falling back to anything else.

Arrays may be numpy arrays (host) or torch CUDA tensors (device memory; the
library then reads them in place on the given stream).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpba.so")

PBA_OK, PBA_EINVAL, PBA_ENOMEM, PBA_EDEVICE, PBA_ESTATE, PBA_ENOTPD, PBA_ENOVALID = 0, -1, -2, -3, -4, -5, -6
PBA_PINHOLE, PBA_SPHERICAL = 0, 1
PBA_F32, PBA_F64 = 0, 1
PBA_ORDER_AUTO, PBA_ORDER_NATURAL, PBA_ORDER_ND = 0, 1, 2
PBA_PAIR_OUT_LEN = 160
PBA_NOALLOC_SCRATCH_BYTES = 128 << 20

# names declared in include/pba.h
ABI_FUNCTIONS = (
    "pba_config_default", "pba_create", "pba_destroy", "pba_add_sensor", "pba_load_keyframes",
    "pba_set_poses", "pba_get_poses", "pba_set_pose_groups", "pba_set_pairs", "pba_evaluate",
    "pba_evaluate_noalloc", "pba_solve_step",
    "pba_apply_step", "pba_iterate", "pba_loss_forward", "pba_loss_backward", "pba_build_pyramid",
    "pba_set_level", "pba_optimize_pyramid", "pba_get_level_image", "pba_autotune", "pba_build_pairs", "pba_estimate_normals", "pba_debug_pair",
    "pba_get_timings", "pba_status_string", "pba_last_error",
)


class pba_sensor(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("height", ctypes.c_int32), ("width", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("fx", ctypes.c_double), ("fy", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double), ("min_depth", ctypes.c_double),
                ("max_depth", ctypes.c_double), ("offset", ctypes.c_double * 12)]


class pba_config(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("precision", ctypes.c_int32), ("channels", ctypes.c_int32),
                ("grad_mode", ctypes.c_int32), ("anchor", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("omega_intensity", ctypes.c_double),
                ("omega_depth", ctypes.c_double), ("omega_normal", ctypes.c_double),
                ("huber_delta", ctypes.c_double), ("occlusion_tau_pinhole", ctypes.c_double),
                ("occlusion_tau_spherical", ctypes.c_double), ("occlusion_zbuffer", ctypes.c_int32),
                ("storage_bf16", ctypes.c_int32), ("solve_order", ctypes.c_int32), ("dev_alloc", ctypes.c_void_p),
                ("dev_free", ctypes.c_void_p),
                ("alloc_user", ctypes.c_void_p)]


class pba_eval_out(ctypes.Structure):
    _fields_ = [("F", ctypes.c_double), ("n_evaluated", ctypes.c_int64), ("n_valid", ctypes.c_int64),
                ("n_boundary_band", ctypes.c_int64), ("H", ctypes.c_void_p), ("b", ctypes.c_void_p),
                ("pair_out", ctypes.c_void_p), ("on_device", ctypes.c_int32), ("pad", ctypes.c_int32)]


class pba_iter_log(ctypes.Structure):
    _fields_ = [("F", ctypes.c_double), ("lambda_", ctypes.c_double), ("step_norm", ctypes.c_double),
                ("n_valid", ctypes.c_int64), ("accepted", ctypes.c_int32), ("ms", ctypes.c_float)]


class pba_tune_point(ctypes.Structure):
    _fields_ = [("items_px", ctypes.c_int32), ("grid", ctypes.c_int32), ("eval_ms", ctypes.c_double)]


class pba_timings(ctypes.Structure):
    _fields_ = [("eval_ms", ctypes.c_double), ("eval_launches", ctypes.c_int64), ("iterate_ms", ctypes.c_double),
                ("iterations", ctypes.c_int64), ("n_items", ctypes.c_int64), ("items_px", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("iter_eval_ms", ctypes.c_double), ("iter_evals", ctypes.c_int64),
                ("solve_n", ctypes.c_int32), ("solve_steps", ctypes.c_int32), ("solve_nd", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


_lib = None

# device allocator callbacks of pba_config (dev_alloc, dev_free)
_ALLOC_T = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_T = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)


class TorchAllocator:
    """Routes the library's device allocations through torch's caching allocator (on the
    context's device and stream).  Holds the ctypes callbacks alive for the context's life."""

    def __init__(self, device, stream):
        import torch
        self._torch = torch
        self.device = device
        self.stream = stream          # torch.cuda.Stream the library works on
        self.live = {}

        def _alloc(nbytes, user):
            try:
                ptr = int(torch.cuda.caching_allocator_alloc(int(nbytes), device=self.device, stream=self.stream))
            except Exception:
                return None
            self.live[ptr] = int(nbytes)
            return ptr

        def _free(ptr, nbytes, user):
            if ptr and self.live.pop(int(ptr), None) is not None:
                torch.cuda.caching_allocator_delete(int(ptr))

        self.alloc_cb = _ALLOC_T(_alloc)
        self.free_cb = _FREE_T(_free)

    def install(self, cfg):
        cfg.dev_alloc = ctypes.cast(self.alloc_cb, ctypes.c_void_p)
        cfg.dev_free = ctypes.cast(self.free_cb, ctypes.c_void_p)
        cfg.alloc_user = None


_open_contexts = None


def _close_open_contexts():
    # contexts whose memory belongs to torch's allocator are destroyed before torch shuts down
    for ctx in list(_open_contexts or ()):
        try:
            ctx.close()
        except Exception:
            pass


def load_library(path: str = LIB_PATH):
    """Load libpba.so; raises if it has not been built (there is no other implementation)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libpba.so is not built (%s): run __graft_entry__.build() or "
                           "python -m paper_2303_16878_amd.build" % path)
    # torch ships its own copy of the HIP runtime library; the process must use one runtime for
    # the tensors it hands over and for this library, so torch (if present) is loaded first and
    # its runtime then also serves libpba
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp, i32, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    sig = {
        "pba_config_default": (None, [ctypes.POINTER(pba_config)]),
        "pba_create": (i32, [ctypes.POINTER(pba_config), ctypes.POINTER(vp)]),
        "pba_destroy": (i32, [vp]),
        "pba_add_sensor": (i32, [vp, ctypes.POINTER(pba_sensor), ctypes.POINTER(i32)]),
        "pba_load_keyframes": (i32, [vp, i32, vp, vp, vp, vp, i32]),
        "pba_set_poses": (i32, [vp, i32, vp, i32]),
        "pba_get_poses": (i32, [vp, vp, i32]),
        "pba_set_pairs": (i32, [vp, i32, vp, vp]),
        "pba_set_pose_groups": (i32, [vp, vp, i32]),
        "pba_evaluate": (i32, [vp, ctypes.POINTER(pba_eval_out)]),
        "pba_evaluate_noalloc": (i32, [vp, ctypes.POINTER(pba_eval_out)]),
        "pba_solve_step": (i32, [vp, f64, vp, i32]),
        "pba_apply_step": (i32, [vp, vp, i32]),
        "pba_iterate": (i32, [vp, i32, i32, f64, vp]),
        "pba_loss_forward": (i32, [vp, vp, i32, ctypes.POINTER(f64), ctypes.POINTER(ctypes.c_int64)]),
        "pba_loss_backward": (i32, [vp, f64, vp, vp, vp, vp, i32]),
        "pba_build_pyramid": (i32, [vp, i32]),
        "pba_set_level": (i32, [vp, i32]),
        "pba_optimize_pyramid": (i32, [vp, vp, f64, i32, f64, vp, vp, vp]),
        "pba_get_level_image": (i32, [vp, i32, i32, vp, vp, vp, vp]),
        "pba_autotune": (i32, [vp, vp, i32, vp]),
        "pba_build_pairs": (i32, [vp, f64, f64, f64, i32, i32, vp, vp, vp]),
        "pba_estimate_normals": (i32, [vp, f64, f64, f64, i32]),
        "pba_debug_pair": (i32, [vp, i32, vp, vp, vp, vp]),
        "pba_get_timings": (i32, [vp, ctypes.POINTER(pba_timings), i32]),
        "pba_status_string": (ctypes.c_char_p, [i32]),
        "pba_last_error": (ctypes.c_char_p, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class PbaError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s (%d): %s" % (load_library().pba_status_string(status).decode(), status, message))
        self.status = status


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _ptr(x, dtype):
    """(pointer, on_device, keepalive) for a numpy array or a torch tensor."""
    if x is None:
        return None, 0, None
    if _is_torch(x):
        import torch
        tdt = {np.float32: torch.float32, np.float64: torch.float64, np.int32: torch.int32}[dtype]
        if x.dtype != tdt or not x.is_contiguous():
            raise TypeError("expected a contiguous %s tensor" % tdt)
        return x.data_ptr(), int(x.is_cuda), x
    a = np.ascontiguousarray(x, dtype=dtype)
    return a.ctypes.data, 0, a


def config_default():
    cfg = pba_config()
    load_library().pba_config_default(ctypes.byref(cfg))
    return cfg


class Context:
    """Owns one pba_ctx.  Methods map one-to-one onto the C ABI calls."""

    def __init__(self, device=0, precision=PBA_F32, channels=5, grad_mode=0, anchor=0, stream=None,
                 omega_intensity=1.0, omega_depth=1.0, omega_normal=1.0, huber_delta=0.1,
                 occlusion_tau_pinhole=0.5, occlusion_tau_spherical=1.0, use_graph=True, occlusion_zbuffer=False,
                 storage_bf16=False, solve_order=PBA_ORDER_AUTO, allocator="torch"):
        """allocator: "torch" -- device memory from torch's caching allocator (when torch sees a GPU
        and no raw stream handle is given), "hip" -- the library's own hipMalloc.  solve_order:
        PBA_ORDER_AUTO, PBA_ORDER_NATURAL or PBA_ORDER_ND (elimination order of the step's solve)."""
        self.lib = load_library()
        self.h = None
        self.allocator = None
        cfg = config_default()
        cfg.device, cfg.precision, cfg.channels, cfg.grad_mode, cfg.anchor = device, precision, channels, grad_mode, anchor
        cfg.use_graph = int(bool(use_graph))
        tstream = None
        if stream is None:
            try:
                import torch
                if torch.cuda.is_available():
                    tstream = torch.cuda.current_stream(device)
                    stream = tstream.cuda_stream
            except ImportError:
                stream = None
        cfg.stream = stream
        if allocator == "torch" and tstream is not None:
            self.allocator = TorchAllocator(device, tstream)
            self.allocator.install(cfg)
        elif allocator not in ("torch", "hip"):
            raise ValueError("allocator must be 'torch' or 'hip'")
        cfg.omega_intensity, cfg.omega_depth, cfg.omega_normal = omega_intensity, omega_depth, omega_normal
        cfg.huber_delta = huber_delta
        cfg.occlusion_tau_pinhole, cfg.occlusion_tau_spherical = occlusion_tau_pinhole, occlusion_tau_spherical
        cfg.occlusion_zbuffer = int(bool(occlusion_zbuffer))
        cfg.storage_bf16 = int(bool(storage_bf16))
        cfg.solve_order = int(solve_order)
        self.cfg = cfg
        h = ctypes.c_void_p()
        self._check(self.lib.pba_create(ctypes.byref(cfg), ctypes.byref(h)), ctx=None)
        self.h = h
        global _open_contexts
        if _open_contexts is None:
            import atexit
            import weakref
            _open_contexts = weakref.WeakSet()
            atexit.register(_close_open_contexts)
        _open_contexts.add(self)
        self.n = 0
        self.n_poses = 0
        self.p = 0
        self.sensor_sizes = []
        self.kf_sensor = None

    def _check(self, st, ctx="self"):
        if st != PBA_OK:
            msg = self.lib.pba_last_error(self.h if ctx == "self" else None).decode()
            raise PbaError(st, msg)

    def close(self):
        if getattr(self, "h", None):
            self.lib.pba_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def add_sensor(self, model, height, width, fx, fy, cx, cy, min_depth, max_depth, offset=None):
        s = pba_sensor()
        s.model, s.height, s.width = model, height, width
        s.fx, s.fy, s.cx, s.cy, s.min_depth, s.max_depth = fx, fy, cx, cy, min_depth, max_depth
        off = np.eye(3).reshape(-1).tolist() + [0.0, 0.0, 0.0] if offset is None else list(np.asarray(offset, float))
        for i in range(12):
            s.offset[i] = off[i]
        sid = ctypes.c_int32()
        self._check(self.lib.pba_add_sensor(self.h, ctypes.byref(s), ctypes.byref(sid)))
        self.sensor_sizes.append((height, width))
        return sid.value

    def load_keyframes(self, sensor_ids, intensity, depth, normals=None):
        n = len(sensor_ids)
        keep = []
        ptrs = {}
        on_dev = None
        for name, arrs in (("I", intensity), ("D", depth), ("N", normals)):
            if arrs is None:
                ptrs[name] = None
                continue
            ps = (ctypes.c_void_p * n)()
            for k in range(n):
                p, dev, ka = _ptr(arrs[k], np.float32)
                keep.append(ka)
                ps[k] = p
                if on_dev is None:
                    on_dev = dev
                elif on_dev != dev:
                    raise ValueError("mixing host and device images")
            ptrs[name] = ps
        sid = np.ascontiguousarray(sensor_ids, np.int32)
        self._check(self.lib.pba_load_keyframes(
            self.h, n, sid.ctypes.data, ctypes.cast(ptrs["I"], ctypes.c_void_p),
            ctypes.cast(ptrs["D"], ctypes.c_void_p),
            ctypes.cast(ptrs["N"], ctypes.c_void_p) if ptrs["N"] is not None else None, int(on_dev or 0)))
        self.n = n
        self.n_poses = n
        self.kf_sensor = sid.copy()

    def set_poses(self, poses):
        p, dev, ka = _ptr(poses, np.float64)
        self._check(self.lib.pba_set_poses(self.h, self.n_poses, p, dev))

    def get_poses(self, out=None):
        if out is None:
            out = np.empty((self.n_poses, 12), np.float64)
        p, dev, ka = _ptr(out, np.float64)
        self._check(self.lib.pba_get_poses(self.h, p, dev))
        return out

    def set_pose_groups(self, pose_of=None):
        """Keyframes sharing pose variables (pose_of[k] = variable of keyframe k); None restores one
        pose per keyframe.  Poses must be set again afterwards (one per variable)."""
        if pose_of is None:
            self._check(self.lib.pba_set_pose_groups(self.h, None, 0))
            self.n_poses = self.n
            return
        g = np.ascontiguousarray(pose_of, np.int32).reshape(-1)
        if len(g) != self.n:
            raise ValueError("pose_of needs one entry per keyframe")
        npv = int(g.max()) + 1 if len(g) else 0
        self._check(self.lib.pba_set_pose_groups(self.h, g.ctypes.data, npv))
        self.n_poses = npv

    def set_pairs(self, pairs):
        pairs = np.ascontiguousarray(pairs, np.int32).reshape(-1, 2)
        s = np.ascontiguousarray(pairs[:, 0])
        t = np.ascontiguousarray(pairs[:, 1])
        self._check(self.lib.pba_set_pairs(self.h, len(pairs), s.ctypes.data, t.ctypes.data))
        self.p = len(pairs)

    def evaluate(self, want_system=False, want_pairs=False, noalloc=False):
        """pba_evaluate, or pba_evaluate_noalloc (noalloc=True: working memory from the library's fixed
        scratch array; same results)."""
        out = pba_eval_out()
        H = b = po = None
        if want_system:
            H = np.empty((6 * self.n_poses, 6 * self.n_poses), np.float64)
            b = np.empty(6 * self.n_poses, np.float64)
            out.H, out.b = H.ctypes.data, b.ctypes.data
        if want_pairs:
            po = np.empty((self.p, PBA_PAIR_OUT_LEN), np.float64)
            out.pair_out = po.ctypes.data
        out.on_device = 0
        fn = self.lib.pba_evaluate_noalloc if noalloc else self.lib.pba_evaluate
        self._check(fn(self.h, ctypes.byref(out)))
        r = dict(F=out.F, n_evaluated=out.n_evaluated, n_valid=out.n_valid, n_boundary_band=out.n_boundary_band)
        if want_system:
            r.update(H=H, b=b)
        if want_pairs:
            r["pairs"] = po
        return r

    def solve_step(self, lam=0.0):
        dx = np.empty(6 * self.n_poses, np.float64)
        self._check(self.lib.pba_solve_step(self.h, float(lam), dx.ctypes.data, 0))
        return dx

    def apply_step(self, dx=None):
        if dx is None:
            self._check(self.lib.pba_apply_step(self.h, None, 0))
        else:
            p, dev, ka = _ptr(dx, np.float64)
            self._check(self.lib.pba_apply_step(self.h, p, dev))

    def iterate(self, n_iters, use_lm=False, lambda0=1e-4):
        logs = (pba_iter_log * max(1, n_iters))()
        self._check(self.lib.pba_iterate(self.h, int(n_iters), int(bool(use_lm)), float(lambda0),
                                         ctypes.cast(logs, ctypes.c_void_p)))
        return [dict(F=l.F, lam=l.lambda_, step=l.step_norm, n_valid=l.n_valid, accepted=bool(l.accepted), ms=l.ms)
                for l in logs[:n_iters]]

    def estimate_normals(self, radius_m=0.1, min_px=2.0, max_px=5.0, min_count=5):
        """Replace the keyframes' normal images with plane fits to the depth (Sec. IV-A)."""
        self._check(self.lib.pba_estimate_normals(self.h, float(radius_m), float(min_px), float(max_px),
                                                  int(min_count)))

    def build_pairs(self, max_angle=np.radians(30.0), max_dist=1.0, min_ratio=1.0 / 3.0, sequential=True):
        """Matching pairs from the current poses (angle, distance, valid-reprojection ratio,
        sequential links); they replace the context's pairs.  Returns int32 [P, 2]."""
        n = ctypes.c_int32()
        cap = max(1, self.n * (self.n - 1))
        src = np.zeros(cap, np.int32)
        tgt = np.zeros(cap, np.int32)
        self._check(self.lib.pba_build_pairs(self.h, float(max_angle), float(max_dist), float(min_ratio),
                                             int(bool(sequential)), cap, src.ctypes.data, tgt.ctypes.data,
                                             ctypes.byref(n)))
        self.p = n.value
        return np.stack([src[:n.value], tgt[:n.value]], 1)

    def autotune(self):
        """Time the evaluation launch over item sizes and grids, keep the fastest; returns the
        measured points [(items_px, grid, eval_ms)]."""
        pts = (pba_tune_point * 64)()
        n = ctypes.c_int32()
        self._check(self.lib.pba_autotune(self.h, ctypes.cast(pts, ctypes.c_void_p), 64, ctypes.byref(n)))
        return [(pts[i].items_px, pts[i].grid, pts[i].eval_ms) for i in range(n.value)]

    def build_pyramid(self, n_levels):
        """Levels 1 .. n_levels - 1 as 2x2 reductions of the loaded images (level 0)."""
        self._check(self.lib.pba_build_pyramid(self.h, int(n_levels)))
        self.n_levels = int(n_levels)

    def set_level(self, level):
        self._check(self.lib.pba_set_level(self.h, int(level)))

    def optimize_pyramid(self, iters, rel_tol=1e-3, use_lm=True, lambda0=1e-4):
        """Coarse to fine over the built levels; iters[l] bounds the iterations of level l
        (iters[0] is the finest).  Returns the log rows, each with its level."""
        it = np.ascontiguousarray(iters, np.int32)
        total = max(1, int(it.sum()))
        logs = (pba_iter_log * total)()
        lev = np.zeros(total, np.int32)
        done = ctypes.c_int32()
        self._check(self.lib.pba_optimize_pyramid(self.h, it.ctypes.data, float(rel_tol), int(bool(use_lm)),
                                                  float(lambda0), ctypes.cast(logs, ctypes.c_void_p),
                                                  lev.ctypes.data, ctypes.byref(done)))
        return [dict(level=int(lev[i]), F=logs[i].F, lam=logs[i].lambda_, step=logs[i].step_norm,
                     n_valid=logs[i].n_valid, accepted=bool(logs[i].accepted)) for i in range(done.value)]

    def get_level_image(self, level, kf):
        """(intensity [H,W], depth [H,W] (0 = no measurement), normals [H,W,3]) of keyframe kf at
        a pyramid level, copied to the host."""
        dims = np.zeros(2, np.int32)
        self._check(self.lib.pba_get_level_image(self.h, int(level), int(kf), None, None, None, dims.ctypes.data))
        H, W = int(dims[0]), int(dims[1])
        I = np.empty((H, W), np.float32)
        D = np.empty((H, W), np.float32)
        N = np.empty((H, W, 3), np.float32)
        self._check(self.lib.pba_get_level_image(self.h, int(level), int(kf), I.ctypes.data, D.ctypes.data,
                                                 N.ctypes.data, None))
        return I, D, N

    def loss_forward(self, delta, with_count=False):
        """F(X0 boxplus delta) (delta: [N, 6] float32 numpy array or CUDA tensor); with_count also
        returns the number of valid correspondences."""
        p, dev, ka = _ptr(delta, np.float32)
        F = ctypes.c_double()
        nv = ctypes.c_int64()
        self._check(self.lib.pba_loss_forward(self.h, p, dev, ctypes.byref(F), ctypes.byref(nv)))
        return (F.value, nv.value) if with_count else F.value

    def loss_backward(self, grad_F=1.0, grad_delta=None, grad_images=None):
        """Gradients of grad_F * F at the last forward's delta.  grad_delta: [N, 6] float32 output
        (numpy or CUDA tensor); grad_images: (I_list, D_list, N_list) of outputs (entries may be
        None).  Outputs must all live on the same side (host or device)."""
        keep = []
        dev_flags = set()
        gd = None
        if grad_delta is not None:
            gd, dev, ka = _ptr(grad_delta, np.float32)
            keep.append(ka)
            dev_flags.add(dev)
        arrs = [None, None, None]
        if grad_images is not None:
            for j, lst in enumerate(grad_images):
                if lst is None:
                    continue
                ps = (ctypes.c_void_p * self.n)()
                for k, t in enumerate(lst):
                    if t is None:
                        continue
                    if not _is_torch(t) and not (isinstance(t, np.ndarray) and t.dtype == np.float32
                                                 and t.flags["C_CONTIGUOUS"]):
                        raise TypeError("gradient outputs must be C-contiguous float32 arrays or tensors")
                    p, dev, ka = _ptr(t, np.float32)
                    keep.append(ka)
                    dev_flags.add(dev)
                    ps[k] = p
                arrs[j] = ps
        if len(dev_flags) > 1:
            raise ValueError("mixing host and device gradient outputs")
        on_dev = dev_flags.pop() if dev_flags else 0
        cast = lambda a: ctypes.cast(a, ctypes.c_void_p) if a is not None else None
        self._check(self.lib.pba_loss_backward(self.h, float(grad_F), gd, cast(arrs[0]), cast(arrs[1]),
                                               cast(arrs[2]), on_dev))

    def debug_pair(self, pair, src_shape):
        H, W = src_shape
        status = np.empty((H, W), np.uint8)
        uv = np.empty((H, W, 2), np.float32)
        cell = np.empty((H, W, 2), np.int32)
        res = np.empty((H, W, 5), np.float32)
        self._check(self.lib.pba_debug_pair(self.h, int(pair), status.ctypes.data, uv.ctypes.data,
                                            cell.ctypes.data, res.ctypes.data))
        return dict(status=status, uv=uv, cell=cell, res=res)

    def timings(self, reset=False):
        t = pba_timings()
        self._check(self.lib.pba_get_timings(self.h, ctypes.byref(t), int(bool(reset))))
        return dict(eval_ms=t.eval_ms, eval_launches=t.eval_launches, iterate_ms=t.iterate_ms,
                    iterations=t.iterations, n_items=t.n_items, items_px=t.items_px, grid=t.grid,
                    iter_eval_ms=t.iter_eval_ms, iter_evals=t.iter_evals, solve_n=t.solve_n,
                    solve_steps=t.solve_steps, solve_nd=bool(t.solve_nd))


def context_for_problem(prob, precision=PBA_F32, channels=None, grad_mode=0, device=0, poses=None, images=None,
                        **kw):
    """Create a context holding a synthetic problem's sensors, keyframes, poses and pairs.

    `prob` follows the layout of the seeded generator (sensors, kf_sensor, images, poses, pairs);
    `images` optionally overrides the per-keyframe (intensity, depth, normals) lists (e.g. torch
    CUDA tensors).  Only argument marshalling happens here."""
    prm = prob.params
    ch = channels if channels is not None else prm["channels"]
    ctx = Context(device=device, precision=precision, channels=ch, grad_mode=grad_mode,
                  anchor=kw.pop("anchor", prm.get("anchor", 0)),
                  omega_intensity=prm["omega_intensity"], omega_depth=prm["omega_depth"],
                  omega_normal=prm["omega_normal"], huber_delta=prm["huber_delta"],
                  occlusion_tau_pinhole=prm["occ_tau_pinhole"], occlusion_tau_spherical=prm["occ_tau_spherical"],
                  **dict(dict(occlusion_zbuffer=bool(prm.get("occlusion_zbuffer", 0)),
                              storage_bf16=bool(prm.get("storage_bf16", 0))), **kw))
    for s in prob.sensors:
        ctx.add_sensor(s["model"], s["H"], s["W"], s["fx"], s["fy"], s["cx"], s["cy"], s["min_depth"],
                       s["max_depth"], s["offset"])
    I, D, N = images if images is not None else (prob.intensity, prob.depth, prob.normals)
    ctx.load_keyframes(prob.kf_sensor, I, D, N if ch == 5 else None)
    if getattr(prob, "pose_of", None) is not None:
        ctx.set_pose_groups(prob.pose_of)
    ctx.set_poses(prob.init_poses if poses is None else poses)
    ctx.set_pairs(prob.pairs)
    return ctx


# ------------------------------------------------------------------ autograd

def _photometric_loss_function():
    import torch

    class PhotometricLoss(torch.autograd.Function):
        """F(X0 boxplus delta, images) as a torch.autograd.Function.

        forward(ctx, pba_context, delta, *images): images are the flat list
        [I_0..I_{N-1}, D_0..D_{N-1}, N_0..N_{N-1}] of CUDA float32 tensors the context holds
        (they are re-loaded into the context, so edits between calls are seen), or empty to use
        the images already loaded.  Returns F as a 0-d float64 tensor on delta's device.
        backward returns dF/d delta and dF/d image for every image tensor given."""

        @staticmethod
        def forward(ctx, pctx, delta, *images):
            n = pctx.n
            if images:
                if len(images) not in (2 * n, 3 * n):
                    raise ValueError("expected 2N or 3N image tensors")
                I, D = list(images[:n]), list(images[n:2 * n])
                Nn = list(images[2 * n:]) if len(images) == 3 * n else None
                pctx.load_keyframes(pctx.kf_sensor, I, D, Nn)
            d = delta.detach().to(torch.float32).contiguous()
            F = pctx.loss_forward(d)
            ctx.pctx = pctx
            ctx.n_images = len(images)
            ctx.shapes = [t.shape for t in images]
            ctx.device = delta.device
            ctx.delta_dtype = delta.dtype
            return torch.tensor(F, dtype=torch.float64, device=delta.device)

        @staticmethod
        def backward(ctx, grad_out):
            pctx = ctx.pctx
            n = pctx.n
            g_delta = torch.empty((pctx.n_poses, 6), dtype=torch.float32, device=ctx.device)
            outs = [torch.empty(sh, dtype=torch.float32, device=ctx.device) for sh in ctx.shapes]
            lists = None
            if ctx.n_images:
                lists = (outs[:n], outs[n:2 * n], outs[2 * n:] if ctx.n_images == 3 * n else None)
            torch.cuda.current_stream(ctx.device).synchronize()
            pctx.loss_backward(float(grad_out.item()), g_delta, lists)
            return (None, g_delta.to(ctx.delta_dtype)) + tuple(outs)

    return PhotometricLoss


_PL = None


def photometric_loss(pctx, delta, images=()):
    """F(X0 boxplus delta) with gradients for delta and the given image tensors (see PhotometricLoss)."""
    global _PL
    if _PL is None:
        _PL = _photometric_loss_function()
    return _PL.apply(pctx, delta, *images)
