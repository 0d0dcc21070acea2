"""Boundary features of the C ABI on the GPU: device memory through the caller's allocator
callbacks (torch's caching allocator in the binding), per-iteration device times in the LM log."""
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


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_torch_caching_allocator_backs_the_context(rgbd_small, pba):
    """With the torch allocator every device buffer of the context is a torch allocation (torch's
    count of allocated bytes covers them while the context lives and returns to its old value
    after pba_destroy), and the results equal those of a context on the library's own hipMalloc."""
    import torch
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    with pba.context_for_problem(rgbd_small, allocator="torch") as ctx:
        ev = ctx.evaluate(want_system=True)
        log = ctx.iterate(2, use_lm=True)
        torch.cuda.synchronize()
        during = torch.cuda.memory_allocated()
        live = sum(ctx.allocator.live.values())
        # packed planes: depth (4 B) plus intensity (4 B) with 2 cues, {intensity, normal} (16 B) with 5
        images = sum(d.size for d in rgbd_small.depth) * (8 if rgbd_small.params["channels"] == 2 else 20)
        _log("torch allocator: %d buffers, %d bytes; torch counts %d more bytes" % (len(ctx.allocator.live), live,
                                                                                  during - before))
        assert live >= images
        assert during - before >= live
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
    with pba.context_for_problem(rgbd_small, allocator="hip") as ctx2:
        ev2 = ctx2.evaluate(want_system=True)
        log2 = ctx2.iterate(2, use_lm=True)
    assert ev["F"] == ev2["F"] and ev["n_valid"] == ev2["n_valid"]
    assert np.array_equal(ev["H"], ev2["H"]) and np.array_equal(ev["b"], ev2["b"])
    assert [l["F"] for l in log] == [l["F"] for l in log2]


def test_iteration_log_carries_device_time(lidar_mini, pba):
    """Every log row of pba_iterate holds that iteration's device time (wall-clock stamps at its
    first and last launch); their sum is within the HIP-event time of the whole call."""
    with pba.context_for_problem(lidar_mini) as ctx:
        ctx.iterate(1, use_lm=True)
        ctx.timings(reset=True)
        log = ctx.iterate(4, use_lm=True)
        tm = ctx.timings(reset=True)
    ms = [l["ms"] for l in log]
    _log("iteration ms", ms, "events", tm["iterate_ms"])
    assert all(m > 0 for m in ms)
    assert sum(ms) <= tm["iterate_ms"] * 1.05 + 0.05
    assert sum(ms) >= 0.5 * tm["iterate_ms"]
