"""Parity at the workloads' full sizes, in the plans the benchmark times:
sampled elements against the oracle's closed-form folds (which the CPU tests
pin to the step simulation), plus properties that hold at any size.

* the benchmark's headline launch: 8 ranks, fp32 N(0,1), 64 MiB per rank,
  tuner plan, twice in a row.
* 8 ranks, fp32 N(0,1), 256 MiB per rank (the largest size of the sweep),
  ring AllReduce under Simple (tuner plan and 1 channel), LL and LL128
  (16 channels): bit-exact samples, all ranks identical, fp64 error bound.
* 16 ranks, 64 MiB per rank, bf16 U(-1,1) sum and int32 U[-2^20, 2^20] max:
  tree AllReduce and ring AllReduce, ReduceScatter, AllGather, Broadcast
  (root 8) and Reduce (root 15), tuner plans.
* 128 MiB requests through the server beside small ones: the same bits alone
  and in the mix, and the oracle's on samples."""
import time

import numpy as np
import pytest

import synthetic_inputs as si
from oracle import definitions as defs
from oracle import elementwise as ew
from oracle import folds
from tests import gpu_harness as H

pytestmark = pytest.mark.gpu

NSAMP = 8192


@pytest.fixture(scope="module")
def vccl():
    import paper_2507_04786_amd as v
    return v


def _sample(rng, n, k=NSAMP):
    idx = np.unique(rng.integers(0, n, k))
    return np.unique(np.concatenate([idx, [0, n - 1]]))


def _dev_at(x, idx):
    t = H.torch()
    return x[t.from_numpy(idx).to(x.device)]


def test_headline_launch_64mib_tuner_plan(vccl):
    """The launch the benchmark times: 8 ranks, fp32 N(0,1) from the same
    generator, 64 MiB per rank, the tuner's plan, issued twice (the second
    launch continues the connections' step counters): sampled elements
    bit-exact against the oracle's fold, all ranks identical, every sample
    within the fp64 recursive-summation bound."""
    t = H.torch()
    R, n = 8, 16 * 1024 * 1024
    xs = si.rank_inputs(si.WL_RING_AR_SWEEP, R, "float32", n)
    comms = vccl.vcclCommInitAll(R)
    try:
        sends = [H.to_dev(x) for x in xs]
        recvs = [H.empty_dev(n, "float32") for _ in range(R)]
        idx = _sample(np.random.default_rng(11), n)
        for launch in range(2):
            H.call(vccl, comms, "allreduce", sends, recvs, n, "float32")
            t.cuda.synchronize()
            assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess
            plan = vccl.vcclCommGetLastPlan(comms[0])
            print(f"headline launch {launch}: plan {plan}", flush=True)
            want = folds.ring_allreduce(xs, "sum", "float32", plan["nchannels"], plan["chunkBytes"] // 4, idx=idx)
            g0 = _dev_at(recvs[0], idx).cpu().numpy()
            assert np.array_equal(g0.view(np.uint32), want.view(np.uint32)), (launch, plan)
            for r in range(1, R):
                assert bool(t.equal(recvs[r], recvs[0])), (launch, r)
            err = np.abs(g0.astype(np.float64) - defs.fp64_sum([x[idx] for x in xs], "float32"))
            assert (err <= defs.sum_error_bound([x[idx] for x in xs], "float32") * (1 + 1e-9)).all()
    finally:
        for c in comms:
            vccl.vcclCommDestroy(c)


def test_allreduce_256mib_all_protocols(vccl):
    t = H.torch()
    R, n = 8, 64 * 1024 * 1024
    xs = si.rank_inputs(si.WL_RING_AR_SWEEP, R, "float32", n, extra=256)
    comms = vccl.vcclCommInitAll(R)
    try:
        sends = [H.to_dev(x) for x in xs]
        recvs = [H.empty_dev(n, "float32") for _ in range(R)]
        idx = _sample(np.random.default_rng(5), n)
        for proto, C in (("auto", 0), ("simple", 1), ("ll", 16), ("ll128", 16)):
            if proto == "auto":
                H.untune(vccl, comms)
            else:
                H.tune(vccl, comms, "ring", proto, nchannels=C, chunk=0, direct=1)
            try:
                H.call(vccl, comms, "allreduce", sends, recvs, n, "float32")
                t.cuda.synchronize()
                assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess
                plan = vccl.vcclCommGetLastPlan(comms[0])
            finally:
                H.untune(vccl, comms)
            want = folds.ring_allreduce(xs, "sum", "float32", plan["nchannels"], plan["chunkBytes"] // 4, idx=idx)
            g0 = _dev_at(recvs[0], idx).cpu().numpy()
            assert np.array_equal(g0.view(np.uint32), want.view(np.uint32)), (proto, plan)
            for r in range(1, R):
                assert bool(t.equal(recvs[r], recvs[0])), (proto, r)
            err = np.abs(g0.astype(np.float64) - defs.fp64_sum([x[idx] for x in xs], "float32"))
            assert (err <= defs.sum_error_bound([x[idx] for x in xs], "float32") * (1 + 1e-9)).all()
    finally:
        for c in comms:
            vccl.vcclCommDestroy(c)


@pytest.mark.parametrize("dtype,op", [("bfloat16", "sum"), ("int32", "max")])
def test_sixteen_ranks_64mib_every_collective(vccl, dtype, op):
    t = H.torch()
    R = 16
    E = H.ELEM[dtype]
    size = 64 << 20
    comms = vccl.vcclCommInitAll(R)
    kw = dict(lo=-2**20, hi=2**20) if dtype == "int32" else {}
    rng = np.random.default_rng(11)
    # one draw per rank serves every collective (AllGather sends a prefix)
    full = si.rank_inputs(si.WL_TREE_AND_CHAINS, R, dtype, size // E, extra=64, **kw)
    try:
        for coll, algo in (("allreduce", "tree"), ("allreduce", "ring"), ("reducescatter", None),
                           ("allgather", None), ("broadcast", None), ("reduce", None)):
            if op == "max" and coll in ("allgather", "broadcast"):
                continue
            n = size // E // (R if coll in ("allgather", "reducescatter") else 1)
            xs = [x[:H.send_len(coll, n, R)] for x in full]
            root = 8 if coll == "broadcast" else 15
            sends = [H.to_dev(x) for x in xs]
            recvs = [H.empty_dev(H.recv_len(coll, n, R), dtype) for _ in range(R)]
            if algo == "tree":
                vccl.vcclCommSetTuning(comms[0], algo=vccl.vcclAlgoTree)
            try:
                H.call(vccl, comms, coll, sends, recvs, n, dtype, op, root)
                t.cuda.synchronize()
                assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess
                plan = vccl.vcclCommGetLastPlan(comms[0])
            finally:
                vccl.vcclCommSetTuning(comms[0])
            what = f"{coll} {algo} {dtype} {op} plan {plan}"
            rl = H.recv_len(coll, n, R)
            idx = _sample(rng, rl)
            if coll == "allreduce":
                if plan["algo"] == 1:
                    want = folds.tree_allreduce(xs, op, dtype, plan["nchannels"], idx=idx)
                else:
                    want = folds.ring_allreduce(xs, op, dtype, plan["nchannels"], plan["chunkBytes"] // E, idx=idx)
                for r in (0, 5, 15):
                    got = H.from_dev(_dev_at(recvs[r], idx), dtype)
                    assert got.tobytes() == want.tobytes(), (what, r)
                if op == "max":
                    brute = defs.allreduce([x[idx] for x in xs], "max", dtype)[0]
                    assert want.tobytes() == brute.tobytes()
            elif coll == "reducescatter":
                for r in (0, 7, 15):
                    got = H.from_dev(_dev_at(recvs[r], idx), dtype)
                    assert got.tobytes() == folds.ring_reducescatter(xs, op, dtype, r, idx=idx).tobytes(), (what, r)
            elif coll == "reduce":
                got = H.from_dev(_dev_at(recvs[root], idx), dtype)
                assert got.tobytes() == folds.ring_reduce(xs, op, dtype, root, idx=idx).tobytes(), what
            elif coll == "allgather":
                blocks = idx // n
                want = np.array([xs[b][i] for b, i in zip(blocks, idx % n)], dtype=xs[0].dtype)
                for r in (0, 9):
                    assert H.from_dev(_dev_at(recvs[r], idx), dtype).tobytes() == want.tobytes(), (what, r)
            else:
                for r in (0, 8, 15):
                    assert bool(t.equal(recvs[r], sends[root])), (what, r)
            del sends, recvs
    finally:
        for c in comms:
            vccl.vcclCommDestroy(c)


def test_serving_128mib_requests_alone_and_mixed(vccl):
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

    def run(which):
        ids = [vccl.vcclServeSubmit(srv, codes[reqs[k][0]], vccl.DTYPE_NAMES[reqs[k][1]], vccl.vcclSum, 0,
                                    reqs[k][2], reqs[k][4], reqs[k][5]) for k in which]
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
        rng = np.random.default_rng(3)
        for k, (coll, dtype, n, xs, _, recvs) in enumerate(reqs):
            for r in range(R):
                assert bool(t.equal(recvs[r], alone[k][r])), (coll, dtype, r)
            rl = H.recv_len(coll, n, R)
            idx = _sample(rng, rl, 4096)
            got = H.from_dev(_dev_at(recvs[1], idx), dtype)
            if coll == "allgather":
                want = np.array([xs[b][i] for b, i in zip(idx // n, idx % n)], dtype=xs[0].dtype)
            elif coll == "reducescatter":
                want = folds.ring_reducescatter(xs, "sum", dtype, 1, idx=idx)
            else:
                # float AllReduce: identical on every rank, within the fp64 bound
                for r in range(R):
                    assert bool(t.equal(recvs[r], recvs[0]))
                ref = defs.fp64_sum([x[idx] for x in xs], dtype)
                bound = defs.sum_error_bound([x[idx] for x in xs], dtype)
                assert (np.abs(ew.to_float64(dtype, got) - ref) <= bound * (1 + 1e-9) + 1e-30).all()
                continue
            assert got.tobytes() == want.tobytes(), (coll, dtype)
    finally:
        for c in comms:
            vccl.vcclCommDestroy(c)
