"""Robustness of the lock-free protocol and of the library's lifetime:

* a collective launched while a torch kernel occupies the device from
  another stream still completes with the definition's result (its
  workgroups wait for compute units, and every wait is bounded)."""
import numpy as np
import pytest

import synthetic_inputs as si
from oracle import definitions as defs
from tests import gpu_harness as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vccl():
    import paper_2507_04786_amd as v
    return v


@pytest.mark.parametrize("coll", ["allreduce", "reducescatter", "allgather"])
def test_collective_beside_a_busy_stream(vccl, coll):
    t = H.torch()
    R, n = 8, 1 << 20
    xs = si.rank_inputs(si.WL_GROUPED, R, "int32", H.send_len(coll, n, R), lo=-2**20, hi=2**20, extra=4242)
    comms = vccl.vcclCommInitAll(R)
    try:
        sends = [H.to_dev(x) for x in xs]
        recvs = [H.empty_dev(H.recv_len(coll, n, R), "int32") for _ in range(R)]
        a = t.randn(8192, 8192, device="cuda")
        b = t.randn(8192, 8192, device="cuda")
        t.cuda.synchronize()
        busy = t.cuda.Stream()
        mine = t.cuda.Stream()
        with t.cuda.stream(busy):
            for _ in range(4):
                c = a @ b  # about 0.5 TFLOP each, queued ahead of the collective
        with t.cuda.stream(mine):
            H.call(vccl, comms, coll, sends, recvs, n, "int32", stream=mine)
        t.cuda.synchronize()
        del c
        assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess
        if coll == "allreduce":
            want = defs.allreduce(xs, "sum", "int32")
        elif coll == "reducescatter":
            want = defs.reducescatter(xs, "sum", "int32")
        else:
            want = defs.allgather(xs)
        for r in range(R):
            assert np.array_equal(H.from_dev(recvs[r], "int32"), want[r]), r
    finally:
        for c in comms:
            vccl.vcclCommDestroy(c)
