"""GPU: the damped step's solve in the nested-dissection order against the natural order and the
oracle's dense solve of the same system.

The factorisation and triangular solves change order and schedule (one launch per elimination-tree
level instead of one per 64-row block column) but not the system: the step must equal the dense
Cholesky solve of the evaluated H, b within 1e-8 of its largest entry in either order (both are
backward-stable FP64 Cholesky solves of systems with condition numbers far below 1e8), and the
iterations that use it must reach the same poses.
"""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


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


def _check_step(dx, H, b, lam, anchor):
    ref, ok = oracle.solve_step(H, b, lam, anchor=anchor)
    assert ok
    err = np.abs(dx - ref).max() / np.abs(ref).max()
    assert err <= 1e-8, err
    return err


# full-size pose graphs: natural block columns (dependent steps) and levels of the dissection
FULL = [("lidar128", 29, 6), ("joint", 57, 8)]


@pytest.mark.parametrize("name,nat_steps,nd_steps", FULL)
def test_full_size_orders_agree(name, nat_steps, nd_steps, pba):
    """Full-size pose graphs (300 LiDAR keyframes with loop closures; the 600-keyframe joint rig):
    the automatic order picks nested dissection, and its step equals the natural order's and the
    dense solve's, undamped and damped."""
    _log("case", name)
    prob = synth.make(name)
    kw = dict(storage_bf16=True) if name == "joint" else {}
    with pba.context_for_problem(prob, **kw) as ca, \
            pba.context_for_problem(prob, solve_order=pba.PBA_ORDER_NATURAL, **kw) as cn:
        ea, en = ca.evaluate(want_system=True), cn.evaluate(want_system=True)
        assert np.array_equal(ea["H"], en["H"]) and np.array_equal(ea["b"], en["b"])
        for lam in (0.0, 1e-4):
            da, dn = ca.solve_step(lam), cn.solve_step(lam)
            e_a = _check_step(da, ea["H"], ea["b"], lam, prob.params.get("anchor", 0))
            e_n = _check_step(dn, en["H"], en["b"], lam, prob.params.get("anchor", 0))
            _log("  lam %g: nested dissection err %.2e, natural err %.2e" % (lam, e_a, e_n))
        ta, tn = ca.timings(), cn.timings()
    _log("  nd order n %d, %d levels; natural n %d, %d block columns" % (ta["solve_n"], ta["solve_steps"],
                                                                        tn["solve_n"], tn["solve_steps"]))
    assert ta["solve_nd"] and not tn["solve_nd"]
    assert tn["solve_n"] == 6 * prob.n and tn["solve_steps"] == nat_steps
    assert ta["solve_steps"] == nd_steps and ta["solve_n"] % 64 == 0 and ta["solve_n"] <= 2 * 6 * prob.n + 64


@pytest.mark.parametrize("fixture", ["rgbd_small", "lidar_mini", "joint_mini"])
@pytest.mark.parametrize("anchor", [0, 2])
def test_forced_nested_dissection_small(fixture, anchor, request, pba):
    """Nested dissection forced on small pose graphs (a single padded tile, or a few): the step
    equals the dense solve with the gauge anchor at keyframe 0 or 2, and pba_apply_step of the
    returned step gives the same poses as the natural order's."""
    prob = request.getfixturevalue(fixture)
    _log("case", fixture, "anchor", anchor)
    poses = []
    for order in (pba.PBA_ORDER_ND, pba.PBA_ORDER_NATURAL):
        with pba.context_for_problem(prob, precision=pba.PBA_F64, anchor=anchor, solve_order=order) as ctx:
            ev = ctx.evaluate(want_system=True)
            for lam in (0.0, 1e-3):
                dx = ctx.solve_step(lam)
                _check_step(dx, ev["H"], ev["b"], lam, anchor)
                assert np.all(dx[6 * anchor:6 * anchor + 6] == 0.0)
            ctx.apply_step(dx)
            poses.append(ctx.get_poses())
            assert ctx.timings()["solve_nd"] == (order == pba.PBA_ORDER_ND)
    assert np.abs(poses[0] - poses[1]).max() < 1e-12


def test_forced_nested_dissection_multiblock_lm(pba):
    """40 LiDAR keyframes (n = 240): LM iterations in the nested-dissection order accept and reject
    as in the natural order and end at the same poses."""
    full = synth.make("lidar128", kfs=range(40), H=32, W=512)
    prob = full.subset(range(40))
    res = {}
    for order in (pba.PBA_ORDER_ND, pba.PBA_ORDER_NATURAL):
        with pba.context_for_problem(prob, precision=pba.PBA_F64, solve_order=order) as ctx:
            ev = ctx.evaluate(want_system=True)
            _check_step(ctx.solve_step(1e-4), ev["H"], ev["b"], 1e-4, 0)
            logs = ctx.iterate(3, use_lm=True, lambda0=1e-4)
            res[order] = (ctx.get_poses(), [l["accepted"] for l in logs], ctx.timings())
    Xd, acc_d, td = res[pba.PBA_ORDER_ND]
    Xn, acc_n, tn = res[pba.PBA_ORDER_NATURAL]
    _log("nd: n %d, %d levels; natural: %d block columns" % (td["solve_n"], td["solve_steps"], tn["solve_steps"]))
    assert td["solve_nd"] and acc_d == acc_n
    assert np.abs(Xd - Xn).max() < 1e-9


def test_nested_dissection_not_positive_definite_then_recovers(lidar_mini, pba):
    """A keyframe in no pair makes the damped system singular: the nested-dissection solve reports
    PBA_ENOTPD with a zero step, and after the pairs are restored it solves again (the flag, which
    this order clears ahead of the factorisation, does not stick)."""
    prob = lidar_mini
    pairs = np.asarray(prob.pairs, np.int32)
    lone = prob.n - 1
    keep = pairs[(pairs[:, 0] != lone) & (pairs[:, 1] != lone)]
    with pba.context_for_problem(prob, precision=pba.PBA_F64, solve_order=pba.PBA_ORDER_ND) as ctx:
        ctx.set_pairs(keep)
        dx = np.full(6 * ctx.n_poses, np.nan)
        assert ctx.lib.pba_solve_step(ctx.h, 1e-3, dx.ctypes.data, 0) == pba.PBA_ENOTPD
        assert np.all(dx == 0.0)
        ctx.set_pairs(pairs)
        ev = ctx.evaluate(want_system=True)
        _check_step(ctx.solve_step(1e-3), ev["H"], ev["b"], 1e-3, 0)


def test_nested_dissection_graph_replays_match_eager(pba):
    """40 LiDAR keyframes (several levels, so level updates too): the captured iteration graph with
    the level launches gives bitwise the poses and log of the same launches made one by one, replay
    after replay."""
    prob = synth.make("lidar128", kfs=range(40), H=32, W=512).subset(range(40))
    kw = dict(solve_order=pba.PBA_ORDER_ND)
    with pba.context_for_problem(prob, use_graph=True, **kw) as cg, \
            pba.context_for_problem(prob, use_graph=False, **kw) as ce:
        for it in range(4):
            lg = cg.iterate(1, use_lm=True, lambda0=1e-4 if it == 0 else 0.0)
            le = ce.iterate(1, use_lm=True, lambda0=1e-4 if it == 0 else 0.0)
            assert np.array_equal(cg.get_poses(), ce.get_poses()), it
            assert [dict(l, ms=0) for l in lg] == [dict(l, ms=0) for l in le], it
        assert cg.timings()["solve_steps"] > 1


def test_nested_dissection_step_to_device_memory(rgbd_small, pba):
    """pba_solve_step with a device output pointer writes the step in pose order there."""
    import torch
    with pba.context_for_problem(rgbd_small, precision=pba.PBA_F64, solve_order=pba.PBA_ORDER_ND) as ctx:
        ev = ctx.evaluate(want_system=True)
        host = ctx.solve_step(1e-3)
        dev = torch.full((6 * ctx.n_poses,), float("nan"), dtype=torch.float64, device="cuda")
        st = ctx.lib.pba_solve_step(ctx.h, 1e-3, dev.data_ptr(), 1)
        torch.cuda.synchronize()
        assert st == pba.PBA_OK
        assert np.array_equal(dev.cpu().numpy(), host)
        _check_step(host, ev["H"], ev["b"], 1e-3, 0)


@pytest.mark.parametrize("order", [-1, 3])
def test_unknown_solve_order_is_rejected(order, pba):
    import ctypes
    cfg = pba.config_default()
    cfg.solve_order = order
    h = ctypes.c_void_p()
    assert pba.load_library().pba_create(ctypes.byref(cfg), ctypes.byref(h)) == pba.PBA_EINVAL
