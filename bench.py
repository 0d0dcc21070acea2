#!/usr/bin/env python3
"""Benchmark: photometric BA iterations on one MI355X.

Workload (default): 128x2048 spherical LiDAR keyframes, 300 of them on a seeded 2 km loop,
2406 ordered pairs within 30 m, 5 channels (intensity, range, normal xyz), Levenberg-Marquardt.
One step = one full iteration: damped FP64 Cholesky solve at the current poses, pose update,
evaluation of residuals/Jacobians/H/b at the candidate over every pair and valid source pixel,
device-side accept/reject.  Inputs are resident on the GPU before timing starts.

Prints one JSON line on stdout.  value = px-pair evaluations per second over whole iterations
(FP32 evaluation path); the FP64 path, the evaluation-kernel roofline and the FP64 CPU oracle
on a bounded sample are reported beside it.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 vector peak without packed math (packed FP32 is disabled for every HIP object of the library):
# 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP (FMA) x 2.4 GHz; FP64 vector issues at the same rate
VALU_PEAK_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bytes_per_px_pair(channels, bf16=0):
    # source texel + one target texel per evaluation: FP32 depth plus the other cues in FP32 or BF16
    return 2 * (4 + (2 if bf16 else 4) * (channels - 1))


def flops_split(channels, target_model):
    """Algorithmic FLOPs (FMA = 2) of one px-pair: (every evaluated px-pair: transform 18, projection
    36 spherical / 10 pinhole, the 12-tap occlusion bound 24; every valid correspondence: the rest --
    bilinear samples with central differences, residuals, Huber, projective Jacobian, Jacobian rows
    and the 27-term accumulation), totalling about 720 for 5 cue rows into a spherical target, 690
    into a pinhole one, 300 for 2 rows."""
    first = 18 + (36 if target_model == 1 else 10) + 24
    total = 300 if channels == 2 else (720 if target_model == 1 else 690)
    return first, total - first


PROFILE_KERNEL = "void pba::eval_kernel<float, 5, 1, 1, 0, false, false, false, false>(pba::EvalArgs, int, int)"


def measured_counters(root):
    """PMC figures of the evaluation kernel on the 128x2048 LiDAR workload from the committed summary:
    HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's reading) and the VALU
    busy fraction, or {} when the kernel source or the dispatched kernel differs from the one
    profiled."""
    import hashlib
    path = os.path.join(root, "profiles", "eval_kernel_lidar128_counters.md")
    src = os.path.join(root, "paper_2303_16878_amd", "csrc", "eval.hip")
    try:
        fields = dict(line.split(": ", 1) for line in open(path).read().splitlines() if ": " in line)
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if fields.get("eval_source_sha256", "").strip() != sha or fields.get("kernel", "").strip() != PROFILE_KERNEL:
            return {}
        return {"traffic_bytes_per_launch": int(fields["traffic_bytes_per_launch"]),
                "valu_busy": float(fields["valu_busy"]),
                "valu_insts_per_launch": int(fields["valu_insts_per_launch"])}
    except (OSError, KeyError, ValueError):
        return {}


def run_path(pba, prob, precision, warmup, steps, autotune=True, use_lm=True, solve_order=0):
    import numpy as np
    import torch
    with pba.context_for_problem(prob, precision=precision, solve_order=solve_order) as ctx:
        torch.cuda.synchronize()
        tune = ctx.autotune() if autotune else []
        # the system at the initial poses, for FP32 vs FP64; per-pair counts for the FLOP figure
        ev_init = ctx.evaluate(want_system=True, want_pairs=True)
        if warmup:
            ctx.iterate(warmup, use_lm=use_lm, lambda0=1e-4)
        ev = ctx.evaluate(want_pairs=True)       # system at the current poses; counts per evaluation
        torch.cuda.synchronize()
        ctx.timings(reset=True)
        t0 = time.perf_counter()
        logs = ctx.iterate(steps, use_lm=use_lm, lambda0=0.0)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        # the evaluation inside each timed iteration, bracketed on the library's stream by device
        # wall-clock stamps (one duration per graph replay)
        tm_it = ctx.timings(reset=True)
        assert tm_it["iter_evals"] == steps, tm_it
        # cross-check: the evaluation alone, timed with HIP events on the same stream
        n_eval_runs = 5
        for _ in range(n_eval_runs):
            ctx.evaluate()
        tm = ctx.timings(reset=True)
        poses = ctx.get_poses()
    return dict(elapsed=elapsed, logs=logs, n_evaluated=ev["n_evaluated"], n_valid=ev["n_valid"], init=ev_init, tune=tune,
                pair_eval=ev["pairs"][:, 157].copy(), pair_valid=ev["pairs"][:, 158].copy(),
                eval_ms=tm_it["iter_eval_ms"] / steps, eval_ms_events=tm["eval_ms"] / n_eval_runs,
                n_items=tm["n_items"], items_px=tm["items_px"], grid=tm["grid"], poses=poses, F=logs[-1]["F"],
                solve_n=tm["solve_n"], solve_steps=tm["solve_steps"], solve_nd=tm["solve_nd"])


def bf16_round(x):
    """float32 -> nearest-even BF16 values, held in float32 (input preparation for the FP64 path)."""
    import numpy as np
    b = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    return (((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16).astype(np.uint32).view(np.float32).reshape(np.shape(x))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(prob, pairs):
    import oracle
    t0 = time.perf_counter()
    r = oracle.eval_pairs(prob, prob.init_poses, pairs=pairs)
    dt = time.perf_counter() - t0
    return int(r["n_eval"].sum()), dt


def cpu_baseline(prob, workload, target_s=15.0):
    """The FP64 oracle, as it is, on a bounded sample of pairs of the same workload: with the host's
    OpenMP threads, and once more on one thread in a child process (sample of ~3 s)."""
    import subprocess
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    pairs = prob.pairs
    n0 = min(len(pairs), max(threads, 8))
    px, dt = _oracle_rate(prob, pairs[:n0])
    n1 = int(min(len(pairs), max(n0, n0 * target_s / max(dt, 1e-3))))
    if n1 > n0:
        px, dt = _oracle_rate(prob, pairs[n0:n1])
        n0 = n1 - n0
    reps = 1
    if n0 == len(pairs) or dt < 0.2 * target_s:   # a small workload: whole evaluations, repeated
        px, dt = 0, 0.0
        n0 = len(pairs)
        while dt < 0.2 * target_s:
            p1, d1 = _oracle_rate(prob, pairs)
            px, dt, reps = px + p1, dt + d1, reps + (1 if px else 0)
    out = dict(value=px / dt, unit="px-pair evals/s", cores=threads, kind="oracle", cpu=cpu_model(),
               sample="%d of %d pairs%s, FP64 evaluation (residuals, Jacobians of both poses, 12x12 blocks) at "
                      "the initial poses, %.1f s" % (n0, len(pairs), " x %d" % reps if reps > 1 else "", dt))
    # one thread: a child process renders only the keyframes of a few pairs
    n_one = max(1, int(3.0 * (px / dt) / threads / max(1.0, px / n0)))
    n_one = min(n_one, len(pairs))
    code = ("import sys, json, time; sys.path.insert(0, %r); import synth, oracle; import numpy as np\n"
            "pairs = np.asarray(synth.make(%r, render_images=False).pairs)[:%d]\n"
            "kfs = sorted(set(int(k) for k in pairs.ravel()))\n"
            "prob = synth.make(%r, kfs=kfs)\n"
            "px, dt, reps = 0, 0.0, 0\n"
            "while dt < 2.0:\n"
            "    t0 = time.perf_counter(); r = oracle.eval_pairs(prob, prob.init_poses, pairs=pairs)\n"
            "    dt += time.perf_counter() - t0; px += int(r['n_eval'].sum()); reps += 1\n"
            "print(json.dumps(dict(px=px, dt=dt, reps=reps)))\n" % (ROOT, workload, n_one, workload))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
        one = json.loads(res.stdout.strip().splitlines()[-1])
        out["single_thread"] = dict(value=one["px"] / one["dt"], unit="px-pair evals/s", cores=1,
                                    sample="first %d pairs%s, %.1f s" % (
                                        n_one, " x %d" % one["reps"] if one["reps"] > 1 else "", one["dt"]))
    except (subprocess.SubprocessError, ValueError, IndexError, KeyError) as e:
        out["single_thread"] = dict(error=str(e)[:200])
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="lidar128",
                    choices=["lidar128", "lidar64", "rgbd_room", "rgbd_small", "joint"])
    ap.add_argument("--bf16", type=int, default=None, metavar="0|1",
                    help="BF16 storage of intensity / normal images (default: 1 for joint, else 0); the FP64 "
                         "path then reads the same images rounded to BF16, held in FP32")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--gn", action="store_true", help="Gauss-Newton iterations (every step taken) instead of LM")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default item size and grid")
    ap.add_argument("--zbuffer", action="store_true",
                    help="the z-buffer occlusion variant (an extra projection-only pass per evaluation)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (5 times), to calibrate byte counters")
    ap.add_argument("--solve-order", default="auto", choices=["auto", "natural", "nd"],
                    help="elimination order of the step's Cholesky solve (auto: nested dissection when it at "
                         "least halves the factorisation's dependent steps)")
    ap.add_argument("--profile-evals", type=int, default=0, metavar="K",
                    help="only load the workload and run K evaluations at the initial poses on the FP32 path "
                         "(default item size and grid): a short command for counter profiles")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copied %d MiB x 5" % args.copy_calibration)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    import paper_2303_16878_amd as pba

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    pba.load_library()
    t0 = time.perf_counter()
    prob = synth.make(args.workload)
    log("generated %s: %d keyframes, %d pairs in %.1f s" % (args.workload, prob.n, len(prob.pairs),
                                                             time.perf_counter() - t0))
    if args.zbuffer:
        prob.params["occlusion_zbuffer"] = 1
    bf16 = args.bf16 if args.bf16 is not None else int(args.workload == "joint")
    prob.params["storage_bf16"] = bf16
    if args.profile_evals:
        with pba.context_for_problem(prob, precision=pba.PBA_F32) as ctx:
            for i in range(args.profile_evals):
                ev = ctx.evaluate()
                log("evaluation %d: %d px-pairs, %d valid" % (i, ev["n_evaluated"], ev["n_valid"]))
        return
    ch = prob.params["channels"]
    sen = prob.sensors[0]

    log("FP32 path: warmup %d, timed %d iterations" % (args.warmup, args.steps))
    order = {"auto": pba.PBA_ORDER_AUTO, "natural": pba.PBA_ORDER_NATURAL, "nd": pba.PBA_ORDER_ND}[args.solve_order]
    r32 = run_path(pba, prob, pba.PBA_F32, args.warmup, args.steps, not args.no_autotune, use_lm=not args.gn,
                   solve_order=order)
    ms_step = 1e3 * r32["elapsed"] / args.steps
    value = r32["n_evaluated"] * args.steps / r32["elapsed"]
    eval_s = r32["eval_ms"] / 1e3
    achieved = bytes_per_px_pair(ch, bf16) * r32["n_evaluated"] / eval_s / 1e9
    # algorithmic FLOPs of one evaluation at the poses the timed iterations start from, pair by pair
    tmodel = [prob.sensors[prob.kf_sensor[int(t)]]["model"] for _, t in prob.pairs]
    flop_launch = float(sum(e * flops_split(ch, m)[0] + v * flops_split(ch, m)[1]
                            for e, v, m in zip(r32["pair_eval"], r32["pair_valid"], tmodel)))
    flop = flop_launch / r32["n_evaluated"]
    tflops = flop_launch / eval_s / 1e12
    log("FP32: %.2f ms/iter, %.3e px-pair/s; eval kernel %.3f ms in the iterations, %.3f ms alone "
        "(%.3e px-pair/s, %.0f GB/s algorithmic)" % (ms_step, value, r32["eval_ms"], r32["eval_ms_events"],
                                                     r32["n_evaluated"] / eval_s, achieved))

    from paper_2303_16878_amd.metrics import ate_rmse
    out = {
        "metric": "px residual+Jacobian evals/s and s/GN-iter, FP32 vs FP64 path, equal final RMSE",
        "value": value,
        "unit": "px-pair evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "%s: %s %dx%d, %d keyframes, %d ordered pairs, %d channels, %s iterations" % (
                args.workload, "spherical" if sen["model"] == 1 else "pinhole", sen["H"], sen["W"], prob.n,
                len(prob.pairs), ch, "GN" if args.gn else "LM"),
            "px_pairs_per_step": r32["n_evaluated"],
            "valid_per_step": r32["n_valid"],
            "work_items": r32["n_items"],
            "items_px": r32["items_px"],
            "grid": r32["grid"],
            "autotune": "item size and grid chosen by pba_autotune over %d points" % len(r32["tune"])
            if r32["tune"] else "off",
            "occlusion": "depth gate + z-buffer of the pair's source points" if args.zbuffer else "depth gate",
            "image_storage": "BF16 intensity / normals, FP32 depth" if bf16 else "FP32",
            "sensors": ["%s %dx%d" % ("spherical" if x["model"] == 1 else "pinhole", x["H"], x["W"])
                        for x in prob.sensors],
            "solve": "%s order: FP64 Cholesky of order %d in %d dependent steps" % (
                "nested-dissection" if r32["solve_nd"] else "natural", r32["solve_n"], r32["solve_steps"]),
        },
        "roofline": {
            # the evaluation kernel is bound by vector-ALU issue (measured VALU busy below); the HBM
            # figure the headline target is quoted on sits beside it
            "bound": "alu",
            "achieved": tflops,
            "peak": VALU_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": tflops / VALU_PEAK_TFLOPS,
            "traffic": None,
            "flop_per_px_pair": flop,
            "flop_model": "per evaluated px-pair: transform + projection + 12-tap occlusion bound (78 spherical, "
                          "52 pinhole); per valid correspondence: the rest of ~720 / 690 / 300 (5 rows spherical / "
                          "pinhole, 2 rows)",
            "valu_busy_counter": None,
            "hbm": {"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                    "bytes_per_px_pair": bytes_per_px_pair(ch, bf16)},
            "kernel": ("eval_kernel<float,%d,%s,%s> (persistent)" % (
                ch, "sph" if sen["model"] == 1 else "pin", "sph" if sen["model"] == 1 else "pin")
                if len(prob.sensors) == 1 else
                "eval_kernel<float,%d,*,*> (persistent; one launch per source/target model pair)" % ch),
            "kernel_ms": r32["eval_ms"],
            "kernel_ms_source": "mean over the timed iterations of device wall-clock stamps around the "
                                "evaluation launches, on the library's stream",
            "kernel_ms_hip_events": r32["eval_ms_events"],
        },
        "s_per_iter": {"f32": r32["elapsed"] / args.steps},
        # the rest of an iteration besides the evaluation launches: damped copy, factorisation,
        # triangular solves, pose update, per-pair reduction, assembly, accept/reject, launch gaps
        "ms_per_iter_outside_eval": {"f32": ms_step - r32["eval_ms"]},
        "eval_px_pairs_per_s": {"f32": r32["n_evaluated"] / eval_s},
        "final_ate_rmse": {"f32": ate_rmse(r32["poses"], prob.gt_poses),
                           "init": ate_rmse(prob.init_poses, prob.gt_poses)},
    }
    pmc = measured_counters(ROOT) if args.workload == "lidar128" and not args.zbuffer else {}
    if pmc:   # HBM bytes per launch (PMC, scaled by a 1 GiB copy) over the same launch time; VALU busy
        tb = pmc["traffic_bytes_per_launch"]
        out["roofline"]["traffic"] = tb / eval_s / 1e9
        out["roofline"]["traffic_bytes_per_launch"] = tb
        out["roofline"]["algorithmic_bytes_per_launch"] = bytes_per_px_pair(ch, bf16) * r32["n_evaluated"]
        out["roofline"]["valu_busy_counter"] = pmc["valu_busy"]
        out["roofline"]["valu_insts_per_launch"] = pmc["valu_insts_per_launch"]
    if not args.no_fp64:
        log("FP64 path: warmup %d, timed %d iterations" % (args.warmup, args.steps))
        prob64 = prob
        if bf16:   # the FP64 path reads FP32 images: the same values, rounded to BF16 here
            import copy
            prob64 = copy.copy(prob)
            prob64.params = dict(prob.params, storage_bf16=0)
            prob64.intensity = [bf16_round(x) for x in prob.intensity]
            prob64.normals = [bf16_round(x) for x in prob.normals]
        r64 = run_path(pba, prob64, pba.PBA_F64, args.warmup, args.steps, not args.no_autotune, use_lm=not args.gn,
                       solve_order=order)
        out["s_per_iter"]["f64"] = r64["elapsed"] / args.steps
        out["eval_px_pairs_per_s"]["f64"] = r64["n_evaluated"] / (r64["eval_ms"] / 1e3)
        out["fp64_value"] = r64["n_evaluated"] * args.steps / r64["elapsed"]
        out["final_ate_rmse"]["f64"] = ate_rmse(r64["poses"], prob.gt_poses)
        out["final_ate_rmse"]["abs_diff"] = abs(out["final_ate_rmse"]["f64"] - out["final_ate_rmse"]["f32"])
        a, b = r32["init"], r64["init"]
        out["fp32_vs_fp64"] = {
            "at": "initial poses, then after the timed iterations",
            "F_rel": abs(a["F"] - b["F"]) / abs(b["F"]),
            "H_rel_max": float(np.abs(a["H"] - b["H"]).max() / np.abs(b["H"]).max()),
            "b_rel_max": float(np.abs(a["b"] - b["b"]).max() / np.abs(b["b"]).max()),
            "valid_diff": int(a["n_valid"]) - int(b["n_valid"]),
            "final_pose_max_dt_m": float(np.abs(r32["poses"][:, 9:] - r64["poses"][:, 9:]).max()),
        }
        log("FP64: %.2f ms/iter; FP32 vs FP64: %s" % (1e3 * r64["elapsed"] / args.steps, out["fp32_vs_fp64"]))
    if not args.no_cpu:
        log("CPU oracle baseline (bounded sample)")
        out["cpu_baseline"] = cpu_baseline(prob, args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
