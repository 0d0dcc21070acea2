"""Host logic of the nested-dissection solve (no GPU): the plan built by the library's own C++ code
(nested-dissection blocks, padded positions, tile pattern with fill and elimination-tree levels,
per-level task lists) drives a CPU run of the level-scheduled factorisation and triangular solves
in the device launches' order; the result equals numpy's dense solve of the same gauge-fixed,
damped system (a library routine independent of both the plan and the oracle) to 1e-12 of its
largest entry.  Entries outside the plan's pattern are NaN in that run, so a read outside the
pattern fails the comparison; invariants of the plan are checked inside the program.

Systems: a random symmetric positive definite matrix with the block pattern of each pose graph
(one 12x12 Gram block per pair plus a diagonal shift), on the full-size LiDAR loop and joint-rig
graphs, a cycle with chords, two disconnected paths with an isolated vertex, and the smallest
graphs.
"""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2303_16878_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc) and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("ndplan") / "nd_plan_check")
    cmd = [hipcc, "--offload-arch=gfx950", "-O2", "-std=c++17", "-I", CSRC, "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "nd_plan_check.cpp"), os.path.join(CSRC, "ordering.hip"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return exe


def _run(exe, N, pairs, anchor=0, lam=0.0, seed=1):
    rng = np.random.default_rng(seed)
    n0 = 6 * N
    H = np.zeros((n0, n0))
    for s, t in pairs:
        J = rng.standard_normal((12, 12))
        idx = np.r_[6 * s:6 * s + 6, 6 * t:6 * t + 6]
        H[np.ix_(idx, idx)] += J.T @ J
    H += 5 * np.eye(n0)
    b = rng.standard_normal(n0)
    buf = struct.pack("<ii", N, len(pairs)) + b"".join(struct.pack("<ii", s, t) for s, t in pairs)
    buf += struct.pack("<iid", n0, anchor, lam) + H.astype("<f8").tobytes() + b.astype("<f8").tobytes()
    r = subprocess.run([exe], input=buf, capture_output=True, timeout=300)
    assert r.returncode == 0, r.stderr.decode()
    x = np.frombuffer(r.stdout, "<f8")
    A = H.copy()
    a0 = 6 * anchor
    A[a0:a0 + 6, :] = 0.0
    A[:, a0:a0 + 6] = 0.0
    A[a0:a0 + 6, a0:a0 + 6] = np.eye(6)
    A[np.diag_indices(n0)] *= 1.0 + lam
    rhs = -b
    rhs[a0:a0 + 6] = 0.0
    ref = np.linalg.solve(A, rhs)
    err = np.abs(x - ref).max() / (np.abs(ref).max() or 1.0)   # a lone anchored pose: dx = 0
    info = r.stderr.decode().split()
    stats = {info[i]: int(info[i + 1]) for i in range(0, len(info) - 1, 2)}
    return err, stats


def _graph(name):
    import synth
    prob = synth.make(name, render_images=False)
    return prob.n, [(int(s), int(t)) for s, t in prob.pairs]


@pytest.mark.parametrize("name,levels", [("lidar128", 6), ("joint", 8)])
def test_full_size_pose_graphs(checker, name, levels):
    N, pairs = _graph(name)
    err, st = _run(checker, N, pairs, anchor=0, lam=1e-4)
    assert st["levels"] == levels and st["n"] % 64 == 0
    assert err <= 1e-12, err


@pytest.mark.parametrize("graph,anchor,lam", [
    ((120, [(i, i + 1) for i in range(119)] + [(0, 119), (10, 80)]), 7, 0.0),       # cycle with a chord
    ((41, [(i, i + 1) for i in range(19)] + [(i, i + 1) for i in range(20, 39)]), 0, 1e-3),  # 2 paths + 1 isolated
    ((2, [(0, 1)]), 1, 0.0),
    ((1, []), 0, 0.0),
])
def test_small_graphs(checker, graph, anchor, lam):
    N, pairs = graph
    err, st = _run(checker, N, pairs, anchor=anchor, lam=lam)
    assert err <= 1e-12, err
    assert st["n"] >= 6 * N
