"""Failure handling (Section II-A: Abort terminates and cancels ongoing work
to avoid deadlock).  Every condition is forced from the host: a rank whose
workgroups skip their work (test hook) with a short wait timeout, an abort
raised while peers wait, and argument / matching errors.  Every kernel still
exits on its own bounded waits."""
import time

import numpy as np
import pytest

from tests import gpu_harness as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vccl():
    import paper_2507_04786_amd as v
    return v


def test_dead_rank_times_out_with_remote_error(vccl):
    t = H.torch()
    comms = vccl.vcclCommInitAll(4)
    try:
        vccl.vcclCommSetTimeout(comms[0], 20000)  # 20 ms per wait
        vccl.vcclCommDebugSetDeadRanks(comms[0], 1 << 2)
        xs = [t.ones(4096, device="cuda") for _ in range(4)]
        for r in range(4):
            vccl.vcclAllReduce(xs[r], xs[r], 4096, vccl.vcclFloat32, vccl.vcclSum, comms[r])
        t0 = time.time()
        t.cuda.synchronize()
        assert time.time() - t0 < 30
        assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclRemoteError
        with pytest.raises(vccl.VcclError) as e:  # the set refuses further work
            for r in range(4):
                vccl.vcclAllReduce(xs[r], xs[r], 4096, vccl.vcclFloat32, vccl.vcclSum, comms[r])
        assert e.value.code == vccl.vcclRemoteError
    finally:
        for c in comms:
            vccl.vcclCommDestroy(c)


def test_abort_releases_waiting_peers(vccl):
    t = H.torch()
    comms = vccl.vcclCommInitAll(4)
    try:
        vccl.vcclCommSetTimeout(comms[0], 20_000_000)  # 20 s: only the abort can end the wait early
        vccl.vcclCommDebugSetDeadRanks(comms[0], 1 << 1)
        xs = [t.ones(1 << 16, device="cuda") for _ in range(4)]
        for r in range(4):
            vccl.vcclAllReduce(xs[r], xs[r], 1 << 16, vccl.vcclFloat32, vccl.vcclSum, comms[r])
        time.sleep(0.2)
        t0 = time.time()
        vccl.vcclCommAbort(comms[0])  # sets the abort word, then waits for the device
        assert time.time() - t0 < 10
        assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclRemoteError
    finally:
        for c in comms:
            vccl.vcclCommDestroy(c)


def test_argument_and_matching_errors(vccl):
    t = H.torch()
    comms = vccl.vcclCommInitAll(2)
    try:
        x = t.zeros(64, device="cuda")
        y = t.zeros(64, device="cuda", dtype=t.int16)
        bad = [
            lambda: vccl.vcclAllReduce(x, x, 64, 7, vccl.vcclSum, comms[0]),            # dtype
            lambda: vccl.vcclAllReduce(x, x, 64, vccl.vcclFloat32, 9, comms[0]),        # op
            lambda: vccl.vcclBroadcast(x, x, 64, vccl.vcclFloat32, 5, comms[0]),        # root
            lambda: vccl.vcclAllReduce(None, x, 64, vccl.vcclFloat32, vccl.vcclSum, comms[0]),
            lambda: vccl.vcclAllReduce(y[1:], x, 8, vccl.vcclFloat32, vccl.vcclSum, comms[0]),  # misaligned
        ]
        for f in bad:
            with pytest.raises(vccl.VcclError) as e:
                f()
            assert e.value.code == vccl.vcclInvalidArgument
        # mismatched counts across ranks: reported to the call completing the set
        vccl.vcclAllReduce(x, x, 64, vccl.vcclFloat32, vccl.vcclSum, comms[0])
        with pytest.raises(vccl.VcclError) as e:
            vccl.vcclAllReduce(x, x, 32, vccl.vcclFloat32, vccl.vcclSum, comms[1])
        assert e.value.code == vccl.vcclInvalidUsage
        # tree is AllReduce-only; forcing it elsewhere falls back to the ring
        vccl.vcclCommSetTuning(comms[0], algo=vccl.vcclAlgoTree)
        ag = [t.zeros(64, device="cuda") for _ in range(2)]
        vccl.vcclAllGather(x[:32], ag[0], 32, vccl.vcclFloat32, comms[0])
        vccl.vcclAllGather(x[32:], ag[1], 32, vccl.vcclFloat32, comms[1])
        t.cuda.synchronize()
        assert vccl.vcclCommGetLastPlan(comms[0])["algo"] == 0
        vccl.vcclCommSetTuning(comms[0])
        assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess
        with pytest.raises(vccl.VcclError):
            vccl.vcclCommSetTuning(comms[0], chunkBytes=100)  # not a multiple of 16
    finally:
        for c in comms:
            vccl.vcclCommDestroy(c)


def test_different_streams_are_joined(vccl):
    t = H.torch()
    comms = vccl.vcclCommInitAll(4)
    try:
        streams = [t.cuda.Stream() for _ in range(4)]
        xs = [t.full((5000,), float(r), device="cuda") for r in range(4)]
        t.cuda.synchronize()
        for r in range(4):
            vccl.vcclAllReduce(xs[r], xs[r], 5000, vccl.vcclFloat32, vccl.vcclSum, comms[r], streams[r])
        for r in range(4):
            streams[r].synchronize()
            assert bool((xs[r] == 6.0).all())
    finally:
        for c in comms:
            vccl.vcclCommDestroy(c)
