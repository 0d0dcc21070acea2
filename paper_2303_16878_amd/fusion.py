"""LiDAR + RGB-D fusion schedules on a rig whose sensors share one pose per frame.

The fusion experiments refine a rig frame against photometric errors of both sensors in two ways:
coupled, minimising F^r(X) + F^l(X) together, and consecutive, minimising F^l alone and then F^r
starting from that result.  Both run here through the library's LM iterations on the context's
pose variables (pba_set_pose_groups); which pairs belong to which sensor is read from the sensor
models of their keyframes (spherical: LiDAR, pinhole: RGB-D).

`python -m paper_2303_16878_amd.fusion` runs the convergence-basin study on the synthetic rig:
one frame of the joint LiDAR + camera rig aligned to a copy of itself from growing perturbations,
for LiDAR alone, RGB-D alone, coupled and consecutive, reporting the final error.
"""
import argparse
import math
import sys

import numpy as np

SCHEDULES = ("lidar", "rgbd", "coupled", "consecutive")


def split_pairs(pairs, kf_model):
    """Same-sensor pairs by model: (LiDAR pairs, RGB-D pairs); cross-sensor pairs are dropped."""
    pairs = np.asarray(pairs, np.int32).reshape(-1, 2)
    ms, mt = kf_model[pairs[:, 0]], kf_model[pairs[:, 1]]
    return pairs[(ms == 1) & (mt == 1)], pairs[(ms == 0) & (mt == 0)]


def run_schedule(ctx, schedule, lidar_pairs, rgbd_pairs, iters=30, lambda0=1e-4):
    """Refine the context's current poses with one schedule; returns (poses, logs)."""
    if schedule not in SCHEDULES:
        raise ValueError("unknown schedule %r" % schedule)
    stages = {"lidar": [lidar_pairs], "rgbd": [rgbd_pairs],
              "coupled": [np.concatenate([lidar_pairs, rgbd_pairs])],
              "consecutive": [lidar_pairs, rgbd_pairs]}[schedule]
    logs = []
    for pairs in stages:
        ctx.set_pairs(pairs)
        logs += ctx.iterate(iters, use_lm=True, lambda0=lambda0)
    return ctx.get_poses(), logs


def frame_error(X, ref=0, other=1):
    """Translation (m) and rotation (rad) of frame `other` relative to frame `ref`."""
    X = np.asarray(X, np.float64)
    dt = float(np.linalg.norm(X[other, 9:] - X[ref, 9:]))
    c = (np.trace(X[ref, :9].reshape(3, 3).T @ X[other, :9].reshape(3, 3)) - 1.0) / 2.0
    return dt, float(math.acos(min(1.0, max(-1.0, c))))


def basin_study(pba, synth, trans=(0.02, 0.05, 0.1, 0.2, 0.4), rots_deg=(0.5, 1.0, 2.0, 4.0, 8.0), seeds=(0, 1, 2),
                iters=30, precision=None, out=sys.stdout):
    """Final error of each schedule on the self-aligned rig frame, per perturbation (t, r): the
    median over seeds of the mean of the translation (m) and rotation (rad) errors."""
    prob = synth.make("rig_pair")
    kf_model = np.array([prob.sensors[s]["model"] for s in prob.kf_sensor])
    lid, cam = split_pairs(prob.pairs, kf_model)
    table = {}
    for t in trans:
        for r in rots_deg:
            res = {s: [] for s in SCHEDULES}
            for seed in seeds:
                p0 = synth.rig_pair(perturb_t=t, perturb_deg=r, perturb_seed=seed)
                for sched in SCHEDULES:
                    kw = {} if precision is None else dict(precision=precision)
                    with pba.context_for_problem(prob, poses=p0.init_poses, **kw) as ctx:
                        X, _ = run_schedule(ctx, sched, lid, cam, iters=iters)
                    et, er = frame_error(X)
                    res[sched].append(0.5 * (et + er))
            table[(t, r)] = {s: float(np.median(v)) for s, v in res.items()}
            print("t %.2f m, r %.1f deg: " % (t, r) + ", ".join("%s %.1e" % (s, table[(t, r)][s]) for s in SCHEDULES),
                  file=out, flush=True)
    return table


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--iters", type=int, default=30)
    ap.add_argument("--seeds", type=int, default=3)
    args = ap.parse_args(argv)
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import synth
    import paper_2303_16878_amd as pba
    pba.load_library()
    basin_study(pba, synth, seeds=tuple(range(args.seeds)), iters=args.iters)


if __name__ == "__main__":
    main()
