"""Parity at the workloads' full sizes, in the plans the benchmark times:
every output element against the oracle's closed-form folds (which the CPU
tests pin to the step simulation), plus properties that hold at any size.

* the benchmark's headline launch: 8 ranks, fp32 N(0,1), 64 MiB per rank,
  tuner plan, twice in a row.
* 8 ranks, fp32 N(0,1), 256 MiB per rank (the largest size of the sweep),
  ring AllReduce under Simple (tuner plan and 1 channel), LL and LL128
  (16 channels): every element bit-exact, all ranks identical, fp64 error
  bound.
* 16 ranks, 64 MiB per rank, bf16 U(-1,1) sum and int32 U[-2^20, 2^20] max:
  tree AllReduce and ring AllReduce, ReduceScatter, AllGather, Broadcast
  (root 8) and Reduce (root 15), tuner plans.
* 128 MiB requests through the server beside small ones: the same bits alone
  and in the mix, and every element of the oracle's fold for the plan each
  request was served with."""
import time

import numpy as np
import pytest

import synthetic_inputs as si
from oracle import definitions as defs
from oracle import elementwise as ew
from oracle import folds
from tests import gpu_harness as H

pytestmark = pytest.mark.gpu



@pytest.fixture(scope="module")
def vccl():
    import paper_2507_04786_amd as v
    return v


def _within_bound(got, xs, dtype):
    """Every element within gamma_{R-1} * sum |x| of the fp64 sum."""
    err = np.abs(ew.to_float64(dtype, got) - defs.fp64_sum(xs, dtype))
    return bool((err <= defs.sum_error_bound(xs, dtype) * (1 + 1e-9) + 1e-30).all())


def test_headline_launch_64mib_tuner_plan(vccl):
    """The launch the benchmark times: 8 ranks, fp32 N(0,1) from the same
    generator, 64 MiB per rank, the tuner's plan, issued twice (the second
    launch continues the connections' step counters): every element
    bit-exact against the oracle's fold, all ranks identical, every element
    within the fp64 recursive-summation bound."""
    t = H.torch()
    R, n = 8, 16 * 1024 * 1024
    xs = si.rank_inputs(si.WL_RING_AR_SWEEP, R, "float32", n)
    comms = vccl.vcclCommInitAll(R)
    try:
        sends = [H.to_dev(x) for x in xs]
        recvs = [H.empty_dev(n, "float32") for _ in range(R)]
        for launch in range(2):
            H.call(vccl, comms, "allreduce", sends, recvs, n, "float32")
            t.cuda.synchronize()
            assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess
            plan = vccl.vcclCommGetLastPlan(comms[0])
            print(f"headline launch {launch}: plan {plan}", flush=True)
            want = folds.ring_allreduce(xs, "sum", "float32", plan["nchannels"], plan["chunkBytes"] // 4)
            g0 = recvs[0].cpu().numpy()
            assert np.array_equal(g0.view(np.uint32), want.view(np.uint32)), (launch, plan)
            for r in range(1, R):
                assert bool(t.equal(recvs[r], recvs[0])), (launch, r)
            assert _within_bound(g0, xs, "float32")
    finally:
        for c in comms:
            vccl.vcclCommDestroy(c)


@pytest.fixture(scope="module")
def inputs_256mib():
    return si.rank_inputs(si.WL_RING_AR_SWEEP, 8, "float32", 64 * 1024 * 1024, extra=256)


@pytest.mark.parametrize("proto,C", [("auto", 0), ("simple", 1), ("ll", 16), ("ll128", 16)])
def test_allreduce_256mib(vccl, inputs_256mib, proto, C):
    t = H.torch()
    xs = inputs_256mib
    R, n = len(xs), len(xs[0])
    comms = vccl.vcclCommInitAll(R)
    try:
        sends = [H.to_dev(x) for x in xs]
        recvs = [H.empty_dev(n, "float32") for _ in range(R)]
        if proto == "auto":
            H.untune(vccl, comms)
        else:
            H.tune(vccl, comms, "ring", proto, nchannels=C, chunk=0, direct=1)
        print(f"256 MiB AllReduce, {proto}, {C} channels", flush=True)
        H.call(vccl, comms, "allreduce", sends, recvs, n, "float32")
        t.cuda.synchronize()
        assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess
        plan = vccl.vcclCommGetLastPlan(comms[0])
        for r in range(1, R):
            assert bool(t.equal(recvs[r], recvs[0])), (proto, r)
        g0 = recvs[0].cpu().numpy()
        del sends, recvs
        want = folds.ring_allreduce(xs, "sum", "float32", plan["nchannels"], plan["chunkBytes"] // 4)
        assert np.array_equal(g0.view(np.uint32), want.view(np.uint32)), (proto, plan)
        assert _within_bound(g0, xs, "float32")
    finally:
        for c in comms:
            vccl.vcclCommDestroy(c)


_INPUTS16 = {}


def _inputs16(dtype):
    """One draw per rank of 64 MiB serves every 16-rank collective (AllGather
    sends a prefix); drawn once per dtype for the module."""
    if dtype not in _INPUTS16:
        kw = dict(lo=-2**20, hi=2**20) if dtype == "int32" else {}
        _INPUTS16.clear()
        _INPUTS16[dtype] = si.rank_inputs(si.WL_TREE_AND_CHAINS, 16, dtype, (64 << 20) // H.ELEM[dtype], extra=64, **kw)
    return _INPUTS16[dtype]


CASES16 = [(dt, op, coll, algo) for dt, op in (("bfloat16", "sum"), ("int32", "max"))
           for coll, algo in (("allreduce", "tree"), ("allreduce", "ring"), ("reducescatter", None),
                              ("allgather", None), ("broadcast", None), ("reduce", None))
           if not (op == "max" and coll in ("allgather", "broadcast"))]


@pytest.mark.parametrize("dtype,op,coll,algo", CASES16)
def test_sixteen_ranks_64mib(vccl, dtype, op, coll, algo):
    """Every collective at 16 ranks and 64 MiB per rank under the tuner's plan
    (the tree forced for AllReduce once): every output element of every rank
    checked -- floats against the oracle's fold for the plan that ran,
    int32 max against the brute-force definition as well, copies against
    the inputs."""
    t = H.torch()
    R = 16
    E = H.ELEM[dtype]
    size = 64 << 20
    full = _inputs16(dtype)
    n = size // E // (R if coll in ("allgather", "reducescatter") else 1)
    xs = [x[:H.send_len(coll, n, R)] for x in full]
    root = 8 if coll == "broadcast" else 15
    comms = vccl.vcclCommInitAll(R)
    try:
        sends = [H.to_dev(x) for x in xs]
        recvs = [H.empty_dev(H.recv_len(coll, n, R), dtype) for _ in range(R)]
        if algo == "tree":
            vccl.vcclCommSetTuning(comms[0], algo=vccl.vcclAlgoTree)
        print(f"16 ranks, 64 MiB: {coll} {algo} {dtype} {op}", flush=True)
        try:
            H.call(vccl, comms, coll, sends, recvs, n, dtype, op, root)
            t.cuda.synchronize()
            assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess
            plan = vccl.vcclCommGetLastPlan(comms[0])
        finally:
            vccl.vcclCommSetTuning(comms[0])
        if algo == "tree":
            assert plan["algo"] == vccl.vcclAlgoTree
        what = f"{coll} {algo} {dtype} {op} plan {plan}"
        if coll == "allreduce":
            for r in range(1, R):
                assert bool(t.equal(recvs[r], recvs[0])), (what, r)
            got = H.from_dev(recvs[0], dtype)
            del sends, recvs
            if plan["algo"] == vccl.vcclAlgoTree:
                want = folds.tree_allreduce(xs, op, dtype, plan["nchannels"])
            else:
                want = folds.ring_allreduce(xs, op, dtype, plan["nchannels"], plan["chunkBytes"] // E)
            assert got.tobytes() == want.tobytes(), what
            if op == "max":
                assert want.tobytes() == defs.allreduce(xs, "max", dtype)[0].tobytes()
            else:
                assert _within_bound(got, xs, dtype), what
        elif coll == "reducescatter":
            for r in range(R):
                got = H.from_dev(recvs[r], dtype)
                assert got.tobytes() == folds.ring_reducescatter(xs, op, dtype, r).tobytes(), (what, r)
        elif coll == "reduce":
            got = H.from_dev(recvs[root], dtype)
            del sends, recvs
            want = folds.ring_reduce(xs, op, dtype, root)
            assert got.tobytes() == want.tobytes(), what
            if op == "max":
                assert want.tobytes() == defs.allreduce(xs, "max", dtype)[0].tobytes()
            else:
                assert _within_bound(got, xs, dtype), what
        elif coll == "allgather":
            want = np.concatenate(xs).tobytes()
            for r in range(R):
                assert H.from_dev(recvs[r], dtype).tobytes() == want, (what, r)
        else:
            for r in range(R):
                assert bool(t.equal(recvs[r], sends[root])), (what, r)
            assert H.from_dev(recvs[0], dtype).tobytes() == xs[root].tobytes()
    finally:
        for c in comms:
            vccl.vcclCommDestroy(c)


def test_serving_128mib_requests_alone_and_mixed(vccl):
    """128 MiB requests beside a small one through the server, alone and all
    at once: the same bits both ways, and every element of every rank equal
    to the oracle's fold for the plan each request was served with (the
    definition for copies and ReduceScatter's order-free fold)."""
    t = H.torch()
    R = 8
    codes = {"allreduce": 0, "allgather": 3, "reducescatter": 4}
    specs = [("allreduce", "float32", (128 << 20) // 4), ("allgather", "bfloat16", (128 << 20) // 2 // R),
             ("reducescatter", "int32", (128 << 20) // 4 // R), ("allreduce", "bfloat16", 509)]
    reqs = []
    for k, (coll, dtype, n) in enumerate(specs):
        kw = dict(lo=-2**20, hi=2**20) if dtype == "int32" else {}
        xs = si.rank_inputs(si.WL_SERVING, R, dtype, H.send_len(coll, n, R), extra=900 + k, **kw)
        reqs.append((coll, dtype, n, xs, [H.to_dev(x) for x in xs],
                     [H.empty_dev(H.recv_len(coll, n, R), dtype) for _ in range(R)]))
    comms = vccl.vcclCommInitAll(R)
    t.cuda.synchronize()
    srv = vccl.vcclServeCreate(comms, 4 << 30, 32)
    plans = {}

    def run(which):
        ids = []
        for k in which:
            rid = vccl.vcclServeSubmit(srv, codes[reqs[k][0]], vccl.DTYPE_NAMES[reqs[k][1]], vccl.vcclSum, 0,
                                       reqs[k][2], reqs[k][4], reqs[k][5])
            p = vccl.vcclServeGetPlan(srv, rid)
            assert plans.setdefault(k, p) == p  # a request's plan does not depend on the load
            ids.append(rid)
        deadline = time.time() + 60
        pending = set(ids)
        while pending and time.time() < deadline:
            for rid in list(pending):
                done, status, _ = vccl.vcclServeTest(srv, rid)
                if done:
                    assert status == vccl.vcclSuccess
                    pending.discard(rid)
        assert not pending

    try:
        alone = []
        for k in range(len(reqs)):
            run([k])
            alone.append([r.clone() for r in reqs[k][5]])
            for r in reqs[k][5]:
                r.view(t.uint8).fill_(0x5A)
            t.cuda.current_stream().synchronize()
        run(list(range(len(reqs))))
    finally:
        vccl.vcclServeDestroy(srv)
    try:
        assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess
        for k, (coll, dtype, n, xs, _, recvs) in enumerate(reqs):
            plan = plans[k]
            what = (coll, dtype, n, plan)
            for r in range(R):
                assert bool(t.equal(recvs[r], alone[k][r])), (what, r)
            if coll == "allgather":
                want = [np.concatenate(xs)] * R
            elif coll == "reducescatter":
                want = [folds.ring_reducescatter(xs, "sum", dtype, r) for r in range(R)]
            elif plan["algo"] == vccl.vcclAlgoTree:
                want = [folds.tree_allreduce(xs, "sum", dtype, plan["nchannels"])] * R
            else:
                want = [folds.ring_allreduce(xs, "sum", dtype, plan["nchannels"],
                                             plan["chunkBytes"] // H.ELEM[dtype])] * R
            for r in range(R):
                assert H.from_dev(recvs[r], dtype).tobytes() == want[r].tobytes(), (what, r)
            if coll == "allreduce":
                assert _within_bound(want[0], xs, dtype)
    finally:
        for c in comms:
            vccl.vcclCommDestroy(c)
