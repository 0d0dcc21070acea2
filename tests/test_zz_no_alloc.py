"""pba_evaluate_noalloc through the C ABI: the evaluation whose working memory is the library's
fixed scratch array gives bitwise pba_evaluate's results, on two calls in a row -- the second on a
smaller work queue, so it runs over what the first left in the array -- and on a second context;
a work queue larger than the array is refused with PBA_EINVAL and leaves the context usable."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pba():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2303_16878_amd as pba
    pba.load_library()
    return pba


def _same(a, b):
    assert a["F"] == b["F"] and a["n_valid"] == b["n_valid"] and a["n_evaluated"] == b["n_evaluated"]
    assert a["n_boundary_band"] == b["n_boundary_band"]
    assert np.array_equal(a["H"], b["H"]) and np.array_equal(a["b"], b["b"])
    assert np.array_equal(a["pairs"], b["pairs"])


def test_noalloc_matches_evaluate_twice_then_smaller(lidar_mini, rgbd_small, pba):
    big, small = lidar_mini, rgbd_small
    print("noalloc: lidar_mini (%d pairs) then rgbd_small subset" % len(big.pairs), flush=True)
    with pba.context_for_problem(big) as ctx:
        ref = ctx.evaluate(want_system=True, want_pairs=True)
        first = ctx.evaluate(want_system=True, want_pairs=True, noalloc=True)
        _same(first, ref)
        assert first["n_valid"] > 0
    # a smaller queue on another context: the array still holds the first call's partial sums
    with pba.context_for_problem(small) as ctx:
        ctx.set_pairs(small.pairs[:7])
        ref = ctx.evaluate(want_system=True, want_pairs=True)
        second = ctx.evaluate(want_system=True, want_pairs=True, noalloc=True)
        _same(second, ref)
        # the system kept by the context is the evaluated one: a step from it equals the usual one
        dx_noalloc = ctx.solve_step(1e-4)
        ctx.evaluate()
        assert np.array_equal(dx_noalloc, ctx.solve_step(1e-4))


def test_noalloc_fp64_path(rgbd_small, pba):
    with pba.context_for_problem(rgbd_small, precision=pba.PBA_F64) as ctx:
        ref = ctx.evaluate(want_system=True, want_pairs=True)
        _same(ctx.evaluate(want_system=True, want_pairs=True, noalloc=True), ref)


def test_noalloc_refuses_a_queue_beyond_the_array(rgbd_small, pba):
    """60000 pairs of 160x120 keyframes: 300000 work items (4096 source pixels per wave) and 60000 pair
    records need ~154 MB, more than the 128 MiB array."""
    pairs = np.tile(np.asarray(rgbd_small.pairs, np.int32), (3000, 1))
    with pba.context_for_problem(rgbd_small) as ctx:
        ctx.set_pairs(pairs)
        with pytest.raises(pba.PbaError) as e:
            ctx.evaluate(noalloc=True)
        assert e.value.status == pba.PBA_EINVAL
        assert "scratch" in str(e.value)
        ctx.set_pairs(rgbd_small.pairs)
        ref = ctx.evaluate(want_system=True, want_pairs=True)
        _same(ctx.evaluate(want_system=True, want_pairs=True, noalloc=True), ref)
