"""Inspection hooks on the device: the set's double binary tree as the
library built it, against the oracle's construction (Section II-C), and the
per-workgroup profile of a launch."""
import numpy as np
import pytest

from oracle import topology as topo
from tests import gpu_harness as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vccl():
    import paper_2507_04786_amd as v
    return v


@pytest.mark.parametrize("R", [2, 3, 4, 7, 8, 12, 16])
def test_trees_match_the_oracle(vccl, R):
    comms = vccl.vcclCommInitAll(R)
    try:
        trees = topo.double_binary_tree(R, 1)
        for t in (0, 1):
            got = vccl.vcclCommGetTree(comms[0], t)
            want = [-1] * R
            for v in range(R):
                for k in trees[t]["children"][v]:
                    want[k] = v
            assert got == want, (R, t, got, want)
    finally:
        for c in comms:
            vccl.vcclCommDestroy(c)


def test_profile_records_every_workgroup(vccl):
    """A profiled ring AllReduce of 8 ranks on 4 channels: one record per
    (lane, rank) of the launch, each with a positive span, its counter waits
    within it and one item; profiling off again, the next launch leaves the
    records alone."""
    t = H.torch()
    R, n = 8, 1 << 20
    comms = vccl.vcclCommInitAll(R)
    try:
        x = [t.full((n,), r, dtype=t.int32, device="cuda") for r in range(R)]
        y = [t.empty(n, dtype=t.int32, device="cuda") for _ in range(R)]
        H.tune(vccl, comms, "ring", "simple", nchannels=4)
        vccl.vcclCommDebugProfile(comms[0], True)
        H.call(vccl, comms, "allreduce", x, y, n, "int32")
        t.cuda.synchronize()
        recs = vccl.vcclCommDebugReadProfile(comms[0], 64 * R)
        vccl.vcclCommDebugProfile(comms[0], False)
        assert len(recs) == 4 * R
        for k, (t0, t1, wait, items) in enumerate(recs):
            assert items == 1 and t1 > t0 and wait <= t1 - t0, (k, t0, t1, wait, items)
        assert int(y[3][5].item()) == R * (R - 1) // 2
        assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess
    finally:
        H.untune(vccl, comms)
        for c in comms:
            vccl.vcclCommDestroy(c)
