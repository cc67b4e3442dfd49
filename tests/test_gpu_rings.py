"""Per-channel ring orders (Section II-C: each channel has its own ring, set
up at initialisation) through the C ABI: every ring collective under every
protocol, against the oracle's schedule simulation on the same rings, bit for
bit; grouped and served launches keep the per-call bits."""
import numpy as np
import pytest

import synthetic_inputs as si
from oracle import folds
from oracle import simulate as sim
from tests import gpu_harness as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vccl():
    import paper_2507_04786_amd as v
    return v


def _rings(R, nrings, seed):
    rng = np.random.default_rng([0x5EED, 88, R, seed])
    return [[int(x) for x in rng.permutation(R)] for _ in range(nrings)]


_SETS = {}


@pytest.fixture(scope="module")
def ring_set(vccl):
    def get(R, nrings):
        key = (R, nrings)
        if key not in _SETS:
            rings = _rings(R, nrings, nrings)
            _SETS[key] = (vccl.vcclCommInitAll(R, rings=rings), rings)
        return _SETS[key]
    yield get
    for comms, _ in _SETS.values():
        for c in comms:
            vccl.vcclCommDestroy(c)
    _SETS.clear()


def _inputs(R, dtype, n, extra):
    if dtype == "int32":
        return si.rank_inputs(3, R, "int32", n, lo=-2**20, hi=2**20, extra=extra)
    return si.rank_inputs(3, R, dtype, n, extra=extra)


def _run(vccl, comms, coll, xs, count, dtype, root=0):
    R = len(comms)
    sends = [H.to_dev(x) for x in xs]
    recvs = [H.empty_dev(H.recv_len(coll, count, R), dtype) for _ in range(R)]
    H.call(vccl, comms, coll, sends, recvs, count, dtype, "sum", root)
    H.torch().cuda.synchronize()
    assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess
    return [H.from_dev(r, dtype) for r in recvs]


def _same(got, want, what):
    got, want = np.ascontiguousarray(got), np.ascontiguousarray(want)
    assert got.shape == want.shape, what
    bad = np.nonzero(got.view(np.uint8) != want.view(np.uint8))[0]
    assert bad.size == 0, f"{what}: {bad.size} bytes differ, first at byte {bad[:4].tolist()}"


def test_rings_are_reported(vccl, ring_set):
    comms, rings = ring_set(8, 3)
    assert vccl.vcclCommGetRings(comms[5]) == rings
    plain = vccl.vcclCommInitAll(4)
    try:
        assert vccl.vcclCommGetRings(plain[0]) == [[0, 1, 2, 3]]
    finally:
        for c in plain:
            vccl.vcclCommDestroy(c)


@pytest.mark.parametrize("proto", ["simple", "ll", "ll128"])
@pytest.mark.parametrize("R,nrings,C,n,chunk", [(4, 2, 3, 7001, 1024), (8, 3, 5, 4099, 512),
                                                (16, 4, 6, 2051, 2048), (5, 1, 2, 999, 256)])
def test_every_ring_collective_on_rings(vccl, ring_set, proto, R, nrings, C, n, chunk):
    comms, rings = ring_set(R, nrings)
    print(f"rings {proto} R={R} rings={nrings} C={C} n={n}", flush=True)
    for coll in ("allreduce", "reducescatter", "allgather", "broadcast", "reduce"):
        for dtype in (("float32", "int32") if coll != "allgather" else ("float32",)):
            xs = _inputs(R, dtype, H.send_len(coll, n, R), extra=R * 100 + C)
            roots = [R - 1, 1] if coll in ("broadcast", "reduce") else [0]
            for root in roots:
                H.tune(vccl, comms, "ring", proto, nchannels=C, chunk=chunk, direct=-1)
                try:
                    got = _run(vccl, comms, coll, xs, n, dtype, root)
                    plan = vccl.vcclCommGetLastPlan(comms[0])
                finally:
                    H.untune(vccl, comms)
                assert plan["nchannels"] == C
                want = sim.run(coll, xs, dtype=dtype, nchannels=C, chunk_bytes=plan["chunkBytes"], root=root,
                               rings=rings)
                for r in range(R):
                    if coll == "reduce" and r != root:
                        continue
                    _same(got[r], want[r], f"{coll} {proto} {dtype} R={R} rings={nrings} root={root} rank {r}")


@pytest.mark.parametrize("direct", [0, 1])
def test_direct_and_fifo_paths_on_rings(vccl, ring_set, direct):
    """Simple with and without the direct AllGather phase / direct sends."""
    R, C, n = 8, 4, 30011
    comms, rings = ring_set(R, 3)
    for coll in ("allreduce", "allgather", "broadcast"):
        xs = _inputs(R, "float32", H.send_len(coll, n, R), extra=7 + direct)
        H.tune(vccl, comms, "ring", "simple", nchannels=C, chunk=4096, direct=direct)
        try:
            got = _run(vccl, comms, coll, xs, n, "float32", root=3)
            plan = vccl.vcclCommGetLastPlan(comms[0])
        finally:
            H.untune(vccl, comms)
        assert plan["direct"] == direct
        want = sim.run(coll, xs, dtype="float32", nchannels=C, chunk_bytes=4096, root=3, rings=rings)
        for r in range(R):
            _same(got[r], want[r], f"{coll} direct={direct} rank {r}")


def test_grouped_equals_per_call_on_rings(vccl, ring_set):
    """A group places channels on whatever lanes are free; each channel keeps
    its ring, so the grouped bits equal the per-call bits and the oracle's."""
    R = 8
    comms, rings = ring_set(R, 2)
    specs = [("allreduce", "float32", 50001), ("reducescatter", "float32", 7003), ("allreduce", "bfloat16", 999),
             ("allgather", "float32", 3001), ("allreduce", "float32", 12)]
    ins = [_inputs(R, dt, H.send_len(cl, n, R), extra=k) for k, (cl, dt, n) in enumerate(specs)]
    per_call, plans = [], []
    for (cl, dt, n), xs in zip(specs, ins):
        per_call.append(_run(vccl, comms, cl, xs, n, dt))
        plans.append(vccl.vcclCommGetLastPlan(comms[0]))
    sends = [[H.to_dev(x) for x in xs] for xs in ins]
    recvs = [[H.empty_dev(H.recv_len(cl, n, R), dt) for _ in range(R)] for (cl, dt, n) in specs]
    vccl.vcclGroupStart()
    for (cl, dt, n), s, d in zip(specs, sends, recvs):
        H.call(vccl, comms, cl, s, d, n, dt)
    vccl.vcclGroupEnd()
    H.torch().cuda.synchronize()
    assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess
    for k, ((cl, dt, n), xs) in enumerate(zip(specs, ins)):
        for r in range(R):
            _same(H.from_dev(recvs[k][r], dt), per_call[k][r], f"group item {k} {cl} rank {r}")
        if cl == "allreduce" and dt != "int32" and plans[k]["algo"] == vccl.vcclAlgoRing:
            E = H.ELEM[dt]
            want = folds.ring_allreduce(xs, "sum", dt, plans[k]["nchannels"], plans[k]["chunkBytes"] // E,
                                        rings=rings)
            _same(per_call[k][0], want, f"item {k} vs the fold on its rings")


def test_served_requests_on_rings(vccl, ring_set):
    """A served float AllReduce keeps its per-call channels and so its rings."""
    R = 8
    comms, rings = ring_set(R, 3)
    n = 1 << 18
    xs = _inputs(R, "float32", n, extra=55)
    per = _run(vccl, comms, "allreduce", xs, n, "float32")
    sends = [H.to_dev(x) for x in xs]
    recvs = [H.empty_dev(n, "float32") for _ in range(R)]
    H.torch().cuda.synchronize()
    srv = vccl.vcclServeCreate(comms, 1 << 30, 16)
    try:
        rid = vccl.vcclServeSubmit(srv, 0, vccl.vcclFloat32, vccl.vcclSum, 0, n, sends, recvs)
        plan = vccl.vcclServeGetPlan(srv, rid)
        import time
        deadline = time.time() + 30
        while True:
            done, status, _ = vccl.vcclServeTest(srv, rid)
            if done:
                assert status == vccl.vcclSuccess
                break
            assert time.time() < deadline, "request did not complete"
    finally:
        vccl.vcclServeDestroy(srv)
    got = [H.from_dev(r, "float32") for r in recvs]
    for r in range(R):
        _same(got[r], per[r], f"served vs per-call rank {r}")
    if plan["algo"] == vccl.vcclAlgoRing:
        want = folds.ring_allreduce(xs, "sum", "float32", plan["nchannels"], plan["chunkBytes"] // 4, rings=rings)
        _same(got[0], want, "served vs the fold on its rings")


def test_served_reducescatter_and_reduce_keep_per_call_bits_on_rings(vccl, ring_set):
    """On a set with several ring orders a float sum ReduceScatter or Reduce
    folds each channel along its own ring, so the server keeps its per-call
    channel count (where one ring would let it take fewer lanes)."""
    import time
    R = 8
    comms, rings = ring_set(R, 3)
    cases = []
    for coll, n, root in (("reducescatter", 1 << 17, 0), ("reduce", 1 << 19, 5)):
        xs = _inputs(R, "float32", H.send_len(coll, n, R), extra=len(cases) + 90)
        per = _run(vccl, comms, coll, xs, n, "float32", root)
        cases.append((coll, n, root, xs, per, vccl.vcclCommGetLastPlan(comms[0])))
    srv = vccl.vcclServeCreate(comms, 1 << 30, 64)  # the set's lane limit: every per-call plan fits
    outs = []
    try:
        for coll, n, root, xs, per, plan in cases:
            sends = [H.to_dev(x) for x in xs]
            recvs = [H.empty_dev(H.recv_len(coll, n, R), "float32") for _ in range(R)]
            H.torch().cuda.synchronize()
            code = {"reducescatter": 4, "reduce": 2}[coll]
            rid = vccl.vcclServeSubmit(srv, code, vccl.vcclFloat32, vccl.vcclSum, root, n, sends, recvs)
            sp = vccl.vcclServeGetPlan(srv, rid)
            deadline = time.time() + 30
            while True:
                done, status, _ = vccl.vcclServeTest(srv, rid)
                if done:
                    assert status == vccl.vcclSuccess
                    break
                assert time.time() < deadline, "request did not complete"
            outs.append(([H.from_dev(r, "float32") for r in recvs], sp))
    finally:
        vccl.vcclServeDestroy(srv)
    for (coll, n, root, xs, per, plan), (got, sp) in zip(cases, outs):
        assert sp["nchannels"] == plan["nchannels"], (coll, sp, plan)
        for r in range(R):
            if coll == "reduce" and r != root:
                continue
            _same(got[r], per[r], f"served {coll} vs per-call rank {r}")


@pytest.mark.parametrize("proto", ["simple", "ll"])
def test_trees_and_transfers_ignore_ring_orders(vccl, ring_set, proto):
    """Ring orders shape ring collectives only: on a set with three of them a
    forced tree AllReduce (Section II-C, double binary tree) equals the
    oracle's tree simulation, and a grouped all-to-all of Send/Recv pairs
    equals its definition."""
    from oracle import definitions as defs
    R, C, n = 8, 3, 20011
    comms, rings = ring_set(R, 3)
    xs = _inputs(R, "float32", n, extra=321)
    H.tune(vccl, comms, "tree", proto, nchannels=C, chunk=4096)
    try:
        got = _run(vccl, comms, "allreduce", xs, n, "float32")
        plan = vccl.vcclCommGetLastPlan(comms[0])
    finally:
        H.untune(vccl, comms)
    assert plan["algo"] == vccl.vcclAlgoTree
    want = sim.run("allreduce", xs, dtype="float32", nchannels=C, chunk_bytes=plan["chunkBytes"], algo="tree")
    for r in range(R):
        _same(got[r], want[r], f"tree {proto} on rings rank {r}")
    m = 1001
    ys = si.rank_inputs(si.WL_P2P, R, "int32", R * m, lo=-2**20, hi=2**20, extra=17)
    sends = [H.to_dev(y) for y in ys]
    outs = [H.empty_dev(R * m, "int32") for _ in range(R)]
    H.torch().cuda.synchronize()
    vccl.vcclGroupStart()
    for a in range(R):
        for b in range(R):
            vccl.vcclSend(sends[a][b * m:(b + 1) * m], m, vccl.vcclInt32, b, comms[a])
            vccl.vcclRecv(outs[b][a * m:(a + 1) * m], m, vccl.vcclInt32, a, comms[b])
    vccl.vcclGroupEnd()
    H.torch().cuda.synchronize()
    assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess
    want = defs.alltoall(ys)
    for b in range(R):
        _same(H.from_dev(outs[b], "int32"), want[b], f"all-to-all on rings, rank {b}")
