"""The allocation-free entry point gt_plan_norm_estimate_noalloc against gt_plan_norm_estimate
(the same kernels with per-call buffers): two calls in a row, the second on a smaller
plan, through the C ABI; nothing is allocated during the calls; a plan too large for the
fixed region is rejected with GT_EINVAL."""
import numpy as np
import pytest

import workloads as W
from oracle import index_set as oidx
from paper_2010_10199_amd import lib
from tests.gpu_util import TOL, dtype_code, say, to_dev

pytestmark = pytest.mark.gpu


def _plan(d, ds, N, M, R, prec, seed):
    x = W.uniform_nodes(W.rng(seed, W.P_NODES), M, d, prec)
    p, keep = lib.make_problem(d, ds, N, M=M, R=R, dtype=dtype_code(prec))
    return lib.Plan(p, to_dev(x), keepalive=keep)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_noalloc_norm_estimate_matches_allocating_entry_point(gpu_lib, prec):
    import torch
    torch.cuda.set_device(0)
    cases = [((10, 2, (64, 16), 50000, 1), 61), ((4, 3, (8, 6, 4), 3000, 2), 62)]   # the second is smaller
    for (d, ds, N, M, R), seed in cases:
        plan = _plan(d, ds, N, M, R, prec, seed)
        ref = plan.norm_estimate(30)
        lib.debug_fail_alloc(0)
        got = plan.norm_estimate_noalloc(30)
        nalloc = lib.debug_alloc_count()
        e = abs(got - ref) / ref
        say(f"[noalloc] {prec} d={d} M={M} R={R}: {got:.12e} vs {ref:.12e} rel {e:.2e}, allocations {nalloc}")
        assert nalloc == 0
        assert e <= TOL[prec]
        plan.close()
    torch.cuda.synchronize()


def test_noalloc_rejects_plans_beyond_the_region(gpu_lib):
    """R M complex values alone exceed 16 MiB: 2 right-hand sides x 600,000 nodes in FP64."""
    import torch
    plan = _plan(3, 1, (8,), 600000, 2, "f64", 63)
    with pytest.raises(lib.GroupedError) as e:
        plan.norm_estimate_noalloc(5)
    say(f"[noalloc] rejected: {e.value}")
    assert e.value.code == lib.GT_EINVAL and "exceed" in str(e.value)
    plan.close()
    torch.cuda.synchronize()
