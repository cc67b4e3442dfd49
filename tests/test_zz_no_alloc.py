"""The allocation-free AllReduce (vcclAllReduceNoAlloc) against vcclAllReduce,
the entry point it is a variant of: two calls in a row, the second with a
smaller input, each bit for bit equal to vcclAllReduce run with the plan the
allocation-free call reports, and to the oracle's ring fold for that plan."""
import numpy as np
import pytest

import synthetic_inputs as si
from oracle import definitions as defs
from oracle import folds
from tests import gpu_harness as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vccl():
    import paper_2507_04786_amd as v
    return v


def _run(vccl, comms, R, dtype, op, n, extra, in_place=False):
    t = H.torch()
    kw = dict(lo=-2**20, hi=2**20) if dtype == "int32" else {}
    xs = si.rank_inputs(si.WL_RING_AR_SWEEP, R, dtype, n, extra=extra, **kw)
    sends = [H.to_dev(x) for x in xs]
    recvs = sends if in_place else [H.empty_dev(n, dtype) for _ in range(R)]
    code = vccl.DTYPE_NAMES[dtype]
    o = vccl.OP_NAMES[op]
    print(f"no-alloc AllReduce: R={R} {dtype} {op} n={n} in_place={in_place}", flush=True)
    plan = vccl.vcclAllReduceNoAlloc(sends, recvs, n, code, o)
    t.cuda.synchronize()
    got = [H.from_dev(r, dtype).copy() for r in recvs]
    assert plan["algo"] == vccl.vcclAlgoRing and plan["proto"] in (vccl.vcclProtoSimple, vccl.vcclProtoLL), plan
    assert 1 <= plan["nchannels"] <= min(32, 128 // R) and plan["chunkBytes"] <= 32 * 1024, plan
    # the entry point it is a variant of, with the same plan
    sends2 = [H.to_dev(x) for x in xs]
    recvs2 = sends2 if in_place else [H.empty_dev(n, dtype) for _ in range(R)]
    vccl.vcclCommSetTuning(comms[0], algo=vccl.vcclAlgoRing, proto=plan["proto"], nchannels=plan["nchannels"],
                           nthreads=plan["nthreads"], chunkBytes=plan["chunkBytes"], direct=plan["direct"])
    try:
        H.call(vccl, comms, "allreduce", sends2, recvs2, n, dtype, op)
        t.cuda.synchronize()
        ref_plan = vccl.vcclCommGetLastPlan(comms[0])
    finally:
        vccl.vcclCommSetTuning(comms[0])
    assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess
    assert (ref_plan["nchannels"], ref_plan["chunkBytes"], ref_plan["proto"]) == \
        (plan["nchannels"], plan["chunkBytes"], plan["proto"])
    E = H.ELEM[dtype]
    want = folds.ring_allreduce(xs, op, dtype, plan["nchannels"], plan["chunkBytes"] // E)
    for r in range(R):
        ref = H.from_dev(recvs2[r], dtype)
        assert got[r].tobytes() == ref.tobytes(), (r, plan)
        assert got[r].tobytes() == want.tobytes(), (r, plan)
    if dtype == "int32":
        assert want.tobytes() == defs.allreduce(xs, op, dtype)[0].tobytes()
    return plan


def test_no_alloc_twice_then_smaller(vccl):
    R = 8
    comms = vccl.vcclCommInitAll(R)
    try:
        p1 = _run(vccl, comms, R, "float32", "sum", 3 * 1024 * 1024 + 17, 1)
        p2 = _run(vccl, comms, R, "bfloat16", "sum", 1000, 2)
        assert p1["nchannels"] >= p2["nchannels"]
        _run(vccl, comms, R, "int32", "max", 77777, 3, in_place=True)
    finally:
        for c in comms:
            vccl.vcclCommDestroy(c)


def test_no_alloc_other_rank_counts(vccl):
    """Other rank counts reuse the same array (the counters and LL slots of
    the connections a call uses are cleared by that call)."""
    for R, n in ((16, 1 << 20), (3, 4099), (2, 8)):
        comms = vccl.vcclCommInitAll(R)
        try:
            _run(vccl, comms, R, "float32", "sum", n, 10 + R)
            _run(vccl, comms, R, "int32", "sum", max(1, n // 3), 20 + R)
        finally:
            for c in comms:
                vccl.vcclCommDestroy(c)


def test_no_alloc_rejects_bad_arguments(vccl):
    t = H.torch()
    x = [t.zeros(8, device="cuda") for _ in range(17)]
    for sends, recvs, count, dt in ((x[:1], x[:1], 8, vccl.vcclFloat32), (x[:17], x[:17], 8, vccl.vcclFloat32),
                                    (x[:4], x[:4], 8, 7), (x[:4], x[:4], (1 << 40) + 1, vccl.vcclFloat32)):
        with pytest.raises(vccl.VcclError) as e:
            vccl.vcclAllReduceNoAlloc(sends, recvs, count, dt, vccl.vcclSum)
        assert e.value.code == vccl.vcclInvalidArgument
    with pytest.raises(vccl.VcclError) as e:
        vccl.vcclAllReduceNoAlloc(x[:4], [None] * 4, 8, vccl.vcclFloat32, vccl.vcclSum)
    assert e.value.code == vccl.vcclInvalidArgument
    # nothing is enqueued for an empty call
    assert vccl.vcclAllReduceNoAlloc(x[:4], x[:4], 0, vccl.vcclFloat32, vccl.vcclSum)["nchannels"] == 0


def test_no_alloc_graph_capture_replays(vccl):
    """The allocation-free AllReduce captured in a HIP graph: each replay
    clears the scratch state it uses with a kernel (no memset node), so every
    replay, with eager work and other allocation-free calls between replays,
    gives the eager result."""
    t = H.torch()
    for R, n, dtype in ((8, 1 << 20, "float32"), (4, 4099, "bfloat16"), (16, 8, "float32")):
        print(f"no-alloc graph capture: R={R} n={n} {dtype}", flush=True)
        xs = si.rank_inputs(si.WL_RING_AR_SWEEP, R, dtype, n, extra=40 + R)
        sends = [H.to_dev(x) for x in xs]
        recvs = [H.empty_dev(n, dtype) for _ in range(R)]
        code = vccl.DTYPE_NAMES[dtype]
        plan = vccl.vcclAllReduceNoAlloc(sends, recvs, n, code, vccl.vcclSum)
        t.cuda.synchronize()
        ref = [H.from_dev(r, dtype).copy() for r in recvs]
        want = folds.ring_allreduce(xs, "sum", dtype, plan["nchannels"], plan["chunkBytes"] // H.ELEM[dtype])
        assert ref[0].tobytes() == want.tobytes()
        graph = t.cuda.CUDAGraph()
        with t.cuda.graph(graph):
            vccl.vcclAllReduceNoAlloc(sends, recvs, n, code, vccl.vcclSum, stream=t.cuda.current_stream())
        other = [t.randn(999, device="cuda") for _ in range(R)]
        oout = [t.empty(999, device="cuda") for _ in range(R)]
        for rep in range(4):
            for r in recvs:
                r.fill_(0x5A)
            vccl.vcclAllReduceNoAlloc(other, oout, 999, vccl.vcclFloat32, vccl.vcclSum)
            t.cuda.synchronize()
            graph.replay()
            t.cuda.synchronize()
            for r in range(R):
                assert H.from_dev(recvs[r], dtype).tobytes() == ref[r].tobytes(), (R, n, rep, r)
        del graph
