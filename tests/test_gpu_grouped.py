"""Grouped calls (Section II-A, group calls run as one launch): 64 mixed
collectives of 8 ranks in one GroupStart/GroupEnd, one persistent launch over
a work list, bit-identical to one launch per call and to the oracle."""
import numpy as np
import pytest

import synthetic_inputs as si
from oracle import definitions as defs
from oracle import folds
from tests import gpu_harness as H

pytestmark = pytest.mark.gpu

DT = ["float32", "bfloat16", "int32"]
COLLS = ["allreduce", "allgather", "reducescatter"]


@pytest.fixture(scope="module")
def vccl():
    import paper_2507_04786_amd as v
    return v


@pytest.fixture(scope="module")
def comms(vccl):
    cs = vccl.vcclCommInitAll(8)
    yield cs
    for c in cs:
        vccl.vcclCommDestroy(c)


def _batch(seed, count, lo, hi, R=8):
    """count collectives: kind uniform over AR/AG/RS, size log-uniform in
    [lo, hi] bytes (nccl-tests size = larger per-rank buffer), dtype uniform."""
    rng = si.rng_for(si.WL_GROUPED, 0, seed)
    sizes = si.log_uniform_sizes(rng, count, lo, hi)
    out = []
    for i in range(count):
        coll = COLLS[int(rng.integers(0, 3))]
        dtype = DT[int(rng.integers(0, 3))]
        E = H.ELEM[dtype]
        n = max(1, int(sizes[i]) // E // (R if coll in ("allgather", "reducescatter") else 1))
        if dtype == "int32":
            xs = si.rank_inputs(si.WL_GROUPED, R, "int32", H.send_len(coll, n, R), lo=-2**20, hi=2**20,
                                extra=seed * 1000 + i)
        else:
            xs = si.rank_inputs(si.WL_GROUPED, R, dtype, H.send_len(coll, n, R), extra=seed * 1000 + i)
        out.append((coll, dtype, n, xs))
    return out


def _expected(coll, dtype, n, xs, plan_ch, plan_chunk):
    R = len(xs)
    if coll == "allgather":
        return defs.allgather(xs)
    if coll == "reducescatter":
        if dtype == "int32":
            return defs.reducescatter(xs, "sum", "int32")
        return [folds.ring_reducescatter(xs, "sum", dtype, r) for r in range(R)]
    if dtype == "int32":
        return defs.allreduce(xs, "sum", "int32")
    return None  # float AllReduce: compared against the per-call launch (same plan, same bits)


def _issue(vccl, comms, batch, grouped):
    t = H.torch()
    R = len(comms)
    recvs = []
    sends = []
    for coll, dtype, n, xs in batch:
        sends.append([H.to_dev(x) for x in xs])
        recvs.append([H.empty_dev(H.recv_len(coll, n, R), dtype) for _ in range(R)])
    t.cuda.synchronize()
    if grouped:
        vccl.vcclGroupStart()
    for k, (coll, dtype, n, xs) in enumerate(batch):
        H.call(vccl, comms, coll, sends[k], recvs[k], n, dtype)
    if grouped:
        vccl.vcclGroupEnd()
    t.cuda.synchronize()
    assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess
    return [[H.from_dev(r, b[1]) for r in rs] for rs, b in zip(recvs, batch)]


def test_grouped_64_equals_per_call_and_oracle(vccl, comms):
    batch = _batch(1, 64, 4 * 1024, 4 * 1024 * 1024)
    per_call = _issue(vccl, comms, batch, grouped=False)
    grouped = _issue(vccl, comms, batch, grouped=True)
    info = vccl.vcclCommGetLastPlan(comms[0])
    assert info["ncolls"] == 64 and info["nitems"] >= 64
    for k, (coll, dtype, n, xs) in enumerate(batch):
        for r in range(8):
            a, b = grouped[k][r], per_call[k][r]
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), (k, coll, dtype, n, r)
        want = _expected(coll, dtype, n, xs, None, None)
        if want is not None:
            for r in range(8):
                assert np.array_equal(grouped[k][r].view(np.uint8), want[r].view(np.uint8)), (k, coll, dtype, r)


def test_grouped_float_allreduce_matches_fold(vccl, comms):
    """Each AllReduce of a group follows its own plan's fold order."""
    R = 8
    batch = [("allreduce", "float32", n, si.rank_inputs(si.WL_GROUPED, R, "float32", n, extra=n))
             for n in (1000, 70001, 300000)]
    out = _issue(vccl, comms, batch, grouped=True)
    for k, (coll, dtype, n, xs) in enumerate(batch):
        # the same collective alone reveals its plan (channels, chunk)
        alone = _issue(vccl, comms, [batch[k]], grouped=False)
        info = vccl.vcclCommGetLastPlan(comms[0])
        if info["algo"] == 0:
            want = folds.ring_allreduce(xs, "sum", "float32", info["nchannels"], info["chunkBytes"] // 4)
        else:
            want = folds.tree_allreduce(xs, "sum", "float32", info["nchannels"])
        for r in range(R):
            assert np.array_equal(out[k][r].view(np.uint32), alone[0][r].view(np.uint32))
            assert np.array_equal(out[k][r].view(np.uint32), want.view(np.uint32)), (n, r)


def test_incomplete_group_is_rejected(vccl, comms):
    t = H.torch()
    x = t.zeros(16, device="cuda")
    vccl.vcclGroupStart()
    for r in range(7):  # rank 7 never calls
        vccl.vcclAllReduce(x, x, 16, vccl.vcclFloat32, vccl.vcclSum, comms[r])
    with pytest.raises(vccl.VcclError) as e:
        vccl.vcclGroupEnd()
    assert e.value.code == vccl.vcclInvalidUsage
    # the set still works afterwards
    xs = [np.full(16, r, np.float32) for r in range(8)]
    got = _issue(vccl, comms, [("allreduce", "float32", 16, xs)], grouped=False)
    assert np.all(got[0][0] == 28.0)


def test_device_timestamps_of_a_group(vccl, comms):
    batch = _batch(2, 8, 4096, 65536)
    _issue(vccl, comms, batch, grouped=True)
    st = vccl.vcclCommGetLastTimestamps(comms[0], 8)
    assert len(st) == 8 and all(s > 0 for s in st)
