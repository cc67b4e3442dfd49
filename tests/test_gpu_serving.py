"""Serving: continuous batching over a persistent kernel.  Requests admitted
while others run overlap on the device; each result is the same bits alone
and in the mix, and matches the oracle."""
import numpy as np
import pytest

import synthetic_inputs as si
from oracle import definitions as defs
from oracle import folds
from tests import gpu_harness as H

pytestmark = pytest.mark.gpu

R = 8
KINDS = [(0.6, "allreduce"), (0.2, "allgather"), (0.2, "reducescatter")]
CODES = {"allreduce": 0, "broadcast": 1, "reduce": 2, "allgather": 3, "reducescatter": 4}


@pytest.fixture(scope="module")
def vccl():
    import paper_2507_04786_amd as v
    return v


def _requests(seed, count, lo, hi):
    rng = si.rng_for(si.WL_SERVING, 0, seed)
    sizes = si.log_uniform_sizes(rng, count, lo, hi)
    reqs = []
    for i in range(count):
        u = rng.uniform()
        coll = "allreduce" if u < 0.6 else ("allgather" if u < 0.8 else "reducescatter")
        dtype = ["float32", "bfloat16", "int32"][int(rng.integers(0, 3))]
        E = H.ELEM[dtype]
        n = max(1, int(sizes[i]) // E // (R if coll != "allreduce" else 1))
        kw = dict(lo=-2**20, hi=2**20) if dtype == "int32" else {}
        xs = si.rank_inputs(si.WL_SERVING, R, dtype, H.send_len(coll, n, R), extra=seed * 10000 + i, **kw)
        reqs.append((coll, dtype, n, xs))
    return reqs


def _buffers(reqs):
    bufs = []
    for coll, dtype, n, xs in reqs:
        sends = [H.to_dev(x) for x in xs]
        recvs = [H.empty_dev(H.recv_len(coll, n, R), dtype) for _ in range(R)]
        bufs.append((sends, recvs))
    H.torch().cuda.synchronize()
    return bufs


def _submit(vccl, srv, req, buf, plans=None, k=None):
    """Submits one request; with `plans`, records the plan it was admitted
    with under key k and checks it equals any plan recorded before (a
    request's plan depends only on the request)."""
    coll, dtype, n, _ = req
    rid = vccl.vcclServeSubmit(srv, CODES[coll], vccl.DTYPE_NAMES[dtype], vccl.vcclSum, 0, n, buf[0], buf[1])
    if plans is not None:
        p = vccl.vcclServeGetPlan(srv, rid)
        assert plans.setdefault(k, p) == p, (k, plans[k], p)
    return rid


def _wait(vccl, srv, ids):
    import time
    pending = set(ids)
    deadline = time.time() + 60
    while pending and time.time() < deadline:
        for rid in list(pending):
            done, status, _ = vccl.vcclServeTest(srv, rid)
            if done:
                assert status == vccl.vcclSuccess
                pending.discard(rid)
    assert not pending, "requests did not complete"


def _snapshot(bufs, reqs):
    return [[H.from_dev(r, req[1]).copy() for r in buf[1]] for buf, req in zip(bufs, reqs)]


@pytest.mark.parametrize("lanes", [16, 64])
def test_alone_equals_mix_and_oracle(vccl, lanes):
    """lanes 64: the set's lane limit at 8 ranks, two workgroups per CU."""
    print(f"serving alone/mix lanes={lanes}", flush=True)
    comms = vccl.vcclCommInitAll(R)
    try:
        reqs = _requests(1, 40, 1024, 4 << 20)
        bufs = _buffers(reqs)
        srv = vccl.vcclServeCreate(comms, 4 << 30, lanes)
        try:
            alone = []
            plans = {}
            # no device-wide synchronisation while the persistent kernel runs
            # (it would wait for the kernel's idle exit): completion is
            # published with a system-scope release, so plain copies suffice
            for k, (req, buf) in enumerate(zip(reqs, bufs)):
                _wait(vccl, srv, [_submit(vccl, srv, req, buf, plans, k)])
                alone.append([H.from_dev(r, req[1]).copy() for r in buf[1]])
                for r in buf[1]:
                    r.view(H.torch().uint8).fill_(0x5A)
                H.torch().cuda.current_stream().synchronize()
            ids = [_submit(vccl, srv, req, buf, plans, k) for k, (req, buf) in enumerate(zip(reqs, bufs))]
            _wait(vccl, srv, ids)
            mix = _snapshot(bufs, reqs)
        finally:
            vccl.vcclServeDestroy(srv)
        assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess
        for k, (coll, dtype, n, xs) in enumerate(reqs):
            for r in range(R):
                assert np.array_equal(alone[k][r].view(np.uint8), mix[k][r].view(np.uint8)), (k, coll, dtype, n, r)
            plan = plans[k]
            if coll == "allgather":
                want = defs.allgather(xs)
            elif dtype == "int32":
                want = (defs.allreduce if coll == "allreduce" else defs.reducescatter)(xs, "sum", "int32")
            elif coll == "reducescatter":
                want = [folds.ring_reducescatter(xs, "sum", dtype, r) for r in range(R)]
            elif plan["algo"] == vccl.vcclAlgoTree:
                # float AllReduce: the oracle's fold for the plan it was served with
                want = [folds.tree_allreduce(xs, "sum", dtype, plan["nchannels"])] * R
            else:
                want = [folds.ring_allreduce(xs, "sum", dtype, plan["nchannels"],
                                             plan["chunkBytes"] // H.ELEM[dtype])] * R
            for r in range(R):
                assert np.array_equal(mix[k][r].view(np.uint8), want[r].view(np.uint8)), (k, coll, dtype, r, plan)
            if coll == "allreduce" and dtype != "int32":
                err = np.abs(H_to64(dtype, mix[k][0]) - defs.fp64_sum(xs, dtype))
                assert (err <= defs.sum_error_bound(xs, dtype) * (1 + 1e-9) + 1e-30).all()
        # after the server the per-call path works again on the same lanes
        x = [H.to_dev(np.full(8, r, np.int32)) for r in range(R)]
        for r in range(R):
            vccl.vcclAllReduce(x[r], x[r], 8, vccl.vcclInt32, vccl.vcclSum, comms[r])
        H.torch().cuda.synchronize()
        assert int(x[0][0].item()) == 28
    finally:
        for c in comms:
            vccl.vcclCommDestroy(c)


def H_to64(dtype, a):
    from oracle import elementwise as ew
    return ew.to_float64(dtype, a)


def test_poisson_replay_reports_latencies(vccl):
    comms = vccl.vcclCommInitAll(R)
    try:
        reqs = _requests(2, 200, 1024, 1 << 20)
        bufs = _buffers(reqs)
        srv = vccl.vcclServeCreate(comms, 4 << 30, 16)
        try:
            with pytest.raises(vccl.VcclError) as e:  # the lanes belong to the server
                t = H.torch().zeros(4, device="cuda")
                for r in range(R):
                    vccl.vcclAllReduce(t, t, 4, vccl.vcclFloat32, vccl.vcclSum, comms[r])
            assert e.value.code == vccl.vcclInvalidUsage
            arr = si.poisson_arrivals(si.rng_for(si.WL_SERVING, 1), len(reqs), 20000.0)
            objs = [vccl.make_request(CODES[c], vccl.DTYPE_NAMES[d], vccl.vcclSum, 0, n, b[0], b[1])
                    for (c, d, n, _), b in zip(reqs, bufs)]
            lat, st = vccl.vcclServeReplay(srv, objs, (arr * 1e9).astype(np.int64))
        finally:
            vccl.vcclServeDestroy(srv)
        assert all(s == vccl.vcclSuccess for s in st)
        assert all(x > 0 for x in lat)
        assert np.percentile(lat, 99) < 1e9
    finally:
        for c in comms:
            vccl.vcclCommDestroy(c)


def test_dead_rank_fails_requests_in_bounded_time(vccl):
    """A rank whose workgroups never show up (test hook) with a 20 ms wait
    limit: the request completes with RemoteError, later submissions fail at
    once, the whole persistent grid leaves, and the server is destroyed."""
    import time
    t = H.torch()
    R = 4
    comms = vccl.vcclCommInitAll(R)
    try:
        vccl.vcclCommSetTimeout(comms[0], 20000)
        vccl.vcclCommDebugSetDeadRanks(comms[0], 1 << 2)
        xs = [t.ones(4096, device="cuda") for _ in range(R)]
        t.cuda.synchronize()
        srv = vccl.vcclServeCreate(comms, 1 << 30, 4)
        try:
            t0 = time.time()
            rid = vccl.vcclServeSubmit(srv, 0, vccl.vcclFloat32, vccl.vcclSum, 0, 4096, xs, xs)
            status = None
            while time.time() - t0 < 30:
                done, status, _ = vccl.vcclServeTest(srv, rid)
                if done:
                    break
            assert status == vccl.vcclRemoteError
            assert time.time() - t0 < 30
            rid = vccl.vcclServeSubmit(srv, 0, vccl.vcclFloat32, vccl.vcclSum, 0, 4096, xs, xs)
            done, status, _ = vccl.vcclServeTest(srv, rid)
            assert done and status == vccl.vcclRemoteError
        finally:
            t0 = time.time()
            vccl.vcclServeDestroy(srv)
            assert time.time() - t0 < 10
        assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclRemoteError
    finally:
        for c in comms:
            vccl.vcclCommDestroy(c)


def test_every_collective_in_place_max_and_errors(vccl):
    """Broadcast and Reduce (roots at both ends), max, and in-place requests
    through the server give the per-call bits; int32 results equal their
    definitions.  Submissions the server can never run fail at once with
    InvalidArgument: a zero count, more bytes than the budget."""
    t = H.torch()
    Rs = 4
    comms = vccl.vcclCommInitAll(Rs)
    try:
        specs = [("broadcast", "bfloat16", "sum", 30011, 0), ("broadcast", "int32", "sum", 4099, Rs - 1),
                 ("reduce", "int32", "max", 70001, 3), ("reduce", "float32", "sum", 5000, 0),
                 ("allreduce", "bfloat16", "max", 12345, 0), ("allreduce", "int32", "sum", 65537, 0),
                 ("reducescatter", "int32", "max", 3001, 0), ("allgather", "float32", "sum", 777, 0)]
        data = []
        for k, (coll, dtype, op, n, root) in enumerate(specs):
            kw = dict(lo=-2**20, hi=2**20) if dtype == "int32" else {}
            xs = si.rank_inputs(si.WL_SERVING, Rs, dtype, H.send_len(coll, n, Rs), extra=777000 + k, **kw)
            data.append(xs)

        def run(served, in_place):
            outs = []
            srv = vccl.vcclServeCreate(comms, 1 << 30, 8) if served else None
            try:
                for (coll, dtype, op, n, root), xs in zip(specs, data):
                    sends = [H.to_dev(x) for x in xs]
                    if in_place and coll == "allreduce":
                        recvs = sends
                    else:
                        recvs = [H.empty_dev(H.recv_len(coll, n, Rs), dtype) for _ in range(Rs)]
                    t.cuda.synchronize()
                    if served:
                        rid = vccl.vcclServeSubmit(srv, CODES[coll], vccl.DTYPE_NAMES[dtype], vccl.OP_NAMES[op],
                                                   root, n, sends, recvs)
                        _wait(vccl, srv, [rid])
                    else:
                        H.call(vccl, comms, coll, sends, recvs, n, dtype, op, root)
                    t.cuda.current_stream().synchronize()
                    outs.append([H.from_dev(r, dtype).copy() for r in recvs])
                if served:
                    # requests the server can never run fail at submission,
                    # before any device work; the buffers hold the full count
                    # either way (in place, 4 x 2 GiB), so a wrong admission
                    # could not touch memory outside them
                    big = [t.zeros(1 << 29, dtype=t.int32, device="cuda") for _ in range(Rs)]
                    t.cuda.synchronize()
                    for cnt in (0, 1 << 29):  # zero count; 8 GiB in flight against a 1 GiB budget
                        with pytest.raises(vccl.VcclError) as e:
                            vccl.vcclServeSubmit(srv, CODES["allreduce"], vccl.vcclInt32, vccl.vcclSum, 0, cnt,
                                                 big, big)
                        assert e.value.code == vccl.vcclInvalidArgument, cnt
                    del big
            finally:
                if served:
                    vccl.vcclServeDestroy(srv)
            return outs

        for in_place in (False, True):
            per_call = run(False, in_place)
            served = run(True, in_place)
            for k, (coll, dtype, op, n, root) in enumerate(specs):
                ranks = [root] if coll == "reduce" else range(Rs)
                for r in ranks:
                    assert np.array_equal(served[k][r].view(np.uint8), per_call[k][r].view(np.uint8)), \
                        (k, coll, dtype, op, in_place, r)
                if dtype == "int32":
                    xs = data[k]
                    if coll == "broadcast":
                        want = [xs[root]] * Rs
                    elif coll == "reduce":
                        want = {root: defs.allreduce(xs, op, "int32")[0]}
                    elif coll == "allreduce":
                        want = defs.allreduce(xs, op, "int32")
                    else:
                        want = defs.reducescatter(xs, op, "int32")
                    for r in ranks:
                        assert np.array_equal(served[k][r], want[r]), (k, coll, op, r)
        assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess
    finally:
        for c in comms:
            vccl.vcclCommDestroy(c)


def test_requests_across_idle_exits(vccl):
    """The persistent kernel leaves after 1 ms without work and is relaunched
    when work arrives.  Bursts of 1-4 requests (1-4 lanes each) separated by
    0-3 ms pauses post work while leaders are leaving, so entries land on
    lanes whose leader has already closed them as well as on lanes still
    open.  Every request must complete with the definition's result; the
    500 ms wait limit turns a lane left without its workgroups into a quick
    RemoteError rather than a long wait."""
    import os
    import time
    Rs = 4
    old = os.environ.get("VCCL_SERVE_IDLE_US")
    os.environ["VCCL_SERVE_IDLE_US"] = "1000"
    comms = vccl.vcclCommInitAll(Rs)
    try:
        vccl.vcclCommSetTimeout(comms[0], 500000)
        rng = np.random.default_rng(2024)
        pool = []
        for k in range(4):
            n = int(rng.integers(256, 64 * 1024))
            xs = si.rank_inputs(si.WL_SERVING, Rs, "int32", n, lo=-2**20, hi=2**20, extra=555000 + k)
            pool.append((n, xs, [H.to_dev(x) for x in xs], [H.empty_dev(n, "int32") for _ in range(Rs)],
                         defs.allreduce(xs, "sum", "int32")[0]))
        H.torch().cuda.synchronize()
        srv = vccl.vcclServeCreate(comms, 1 << 30, 8)
        try:
            for burst in range(60):
                ks = rng.permutation(4)[:int(rng.integers(1, 5))]
                ids = [vccl.vcclServeSubmit(srv, 0, vccl.vcclInt32, vccl.vcclSum, 0, pool[k][0], pool[k][2],
                                            pool[k][3]) for k in ks]
                _wait(vccl, srv, ids)
                for k in ks:
                    n, xs, _, recvs, want = pool[k]
                    for r in range(Rs):
                        assert np.array_equal(H.from_dev(recvs[r], "int32"), want), (burst, k, r)
                        recvs[r].view(H.torch().uint8).fill_(0x5A)
                H.torch().cuda.current_stream().synchronize()
                time.sleep(float(rng.uniform(0, 3e-3)))
        finally:
            vccl.vcclServeDestroy(srv)
        assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess
    finally:
        if old is None:
            del os.environ["VCCL_SERVE_IDLE_US"]
        else:
            os.environ["VCCL_SERVE_IDLE_US"] = old
        for c in comms:
            vccl.vcclCommDestroy(c)
