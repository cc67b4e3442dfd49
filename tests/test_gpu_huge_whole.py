"""Buffers past 4 GiB per rank, every output element checked: offsets,
channel partitions (Section V-C) and steps must stay 64-bit from the planner
to the last store (tests/test_gpu_huge.py samples four-rank int32 cases).
Two ranks keep the host side small and give every collective a result that
holds at any size: an fp32 AllReduce, ReduceScatter or Reduce of two ranks
is one IEEE addition per element (either order gives the same bits), so the
whole output equals the element-wise sum, and the copies equal their
sources.  For the AllReduce the oracle's fold for the reported plan is also
compared on sampled elements: random ones, both sides of every channel
boundary, the elements around the 2 GiB and 4 GiB byte offsets, and the
last ones."""
import numpy as np
import pytest

import synthetic_inputs as si
from oracle import folds
from oracle import partition as pt
from tests import gpu_harness as H

pytestmark = pytest.mark.gpu

R = 2
N_AR = (1 << 30) + 4099      # fp32 elements per rank: 4 GiB + 16 KiB


@pytest.fixture(scope="module")
def vccl():
    import paper_2507_04786_amd as v
    return v


def _sample(n, nch, align, seed):
    rng = np.random.default_rng([0x5EED, 4096, seed])
    per = pt.round_up(pt.ceil_div(n, nch), align)
    pts = [rng.integers(0, n, size=1 << 20)]
    for c in range(1, nch + 1):
        b = min(n, c * per)
        pts.append(np.arange(max(0, b - 2), min(n, b + 2)))
    for byte in (1 << 31, 1 << 32):
        e = byte // 4
        pts.append(np.arange(max(0, e - 3), min(n, e + 3)))
    pts.append(np.arange(n - 8, n))
    return np.unique(np.concatenate(pts))


def test_allreduce_past_4gib(vccl):
    t = H.torch()
    print(f"huge AllReduce: {R} ranks, fp32, {N_AR} elements per rank", flush=True)
    xs = si.rank_inputs(si.WL_RING_AR_SWEEP, R, "float32", N_AR, extra=4096)
    comms = vccl.vcclCommInitAll(R)
    try:
        sends = [H.to_dev(x) for x in xs]
        recvs = [H.empty_dev(N_AR, "float32") for _ in range(R)]
        H.call(vccl, comms, "allreduce", sends, recvs, N_AR, "float32")
        t.cuda.synchronize()
        assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess
        plan = vccl.vcclCommGetLastPlan(comms[0])
        print(f"plan {plan}", flush=True)
        # every element: one fp32 addition, and both ranks hold the same bits
        assert bool(t.equal(recvs[0], sends[0] + sends[1]))
        assert bool(t.equal(recvs[1], recvs[0]))
        # the oracle's fold for this plan on sampled elements
        idx = _sample(N_AR, plan["nchannels"], pt.align_units("allreduce", 4), 1)
        want = folds.ring_allreduce(xs, "sum", "float32", plan["nchannels"], plan["chunkBytes"] // 4, idx=idx)
        got = recvs[0][t.from_numpy(idx).to("cuda")].cpu().numpy()
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    finally:
        for c in comms:
            vccl.vcclCommDestroy(c)
        del xs
        t.cuda.empty_cache()


def test_copies_past_4gib(vccl):
    """AllGather into 4 GiB + 8 KiB per rank, then Broadcast of 4 GiB +
    16 KiB from rank 1: bitwise copies of their sources."""
    t = H.torch()
    comms = vccl.vcclCommInitAll(R)
    try:
        n = (1 << 29) + 1025                       # fp32 elements sent per rank
        print(f"huge AllGather: {R} ranks, {n} fp32 elements per rank", flush=True)
        xs = si.rank_inputs(si.WL_TREE_AND_CHAINS, R, "float32", n, extra=4096)
        sends = [H.to_dev(x) for x in xs]
        del xs
        recvs = [H.empty_dev(R * n, "float32") for _ in range(R)]
        H.call(vccl, comms, "allgather", sends, recvs, n, "float32")
        t.cuda.synchronize()
        assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess
        print(f"plan {vccl.vcclCommGetLastPlan(comms[0])}", flush=True)
        for r in range(R):
            for q in range(R):
                assert bool(t.equal(recvs[r][q * n:(q + 1) * n], sends[q])), (r, q)
        del sends, recvs
        t.cuda.empty_cache()

        m = (1 << 30) + 4097                       # fp32 elements broadcast
        print(f"huge Broadcast: {R} ranks, {m} fp32 elements, root 1", flush=True)
        xs = si.rank_inputs(si.WL_TREE_AND_CHAINS, R, "float32", m, extra=4097)
        sends = [H.to_dev(x) for x in xs]
        del xs
        recvs = [H.empty_dev(m, "float32") for _ in range(R)]
        H.call(vccl, comms, "broadcast", sends, recvs, m, "float32", root=1)
        t.cuda.synchronize()
        assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess
        print(f"plan {vccl.vcclCommGetLastPlan(comms[0])}", flush=True)
        for r in range(R):
            assert bool(t.equal(recvs[r], sends[1])), r
        del sends, recvs
    finally:
        for c in comms:
            vccl.vcclCommDestroy(c)
        t.cuda.empty_cache()


def test_reductions_past_4gib(vccl):
    """ReduceScatter from 4 GiB + 8 KiB per rank, then Reduce of 4 GiB +
    16 KiB to rank 0: each output element is one fp32 addition of the two
    ranks' elements."""
    t = H.torch()
    comms = vccl.vcclCommInitAll(R)
    try:
        n = (1 << 29) + 1029                       # fp32 elements received per rank
        print(f"huge ReduceScatter: {R} ranks, {R * n} fp32 elements sent per rank", flush=True)
        xs = si.rank_inputs(si.WL_TREE_AND_CHAINS, R, "float32", R * n, extra=4098)
        sends = [H.to_dev(x) for x in xs]
        del xs
        recvs = [H.empty_dev(n, "float32") for _ in range(R)]
        H.call(vccl, comms, "reducescatter", sends, recvs, n, "float32")
        t.cuda.synchronize()
        assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess
        print(f"plan {vccl.vcclCommGetLastPlan(comms[0])}", flush=True)
        for r in range(R):
            assert bool(t.equal(recvs[r], sends[0][r * n:(r + 1) * n] + sends[1][r * n:(r + 1) * n])), r
        del sends, recvs
        t.cuda.empty_cache()

        m = (1 << 30) + 4101                       # fp32 elements reduced
        print(f"huge Reduce: {R} ranks, {m} fp32 elements, root 0", flush=True)
        xs = si.rank_inputs(si.WL_TREE_AND_CHAINS, R, "float32", m, extra=4099)
        sends = [H.to_dev(x) for x in xs]
        del xs
        recvs = [H.empty_dev(m, "float32") for _ in range(R)]
        H.call(vccl, comms, "reduce", sends, recvs, m, "float32", root=0)
        t.cuda.synchronize()
        assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess
        print(f"plan {vccl.vcclCommGetLastPlan(comms[0])}", flush=True)
        assert bool(t.equal(recvs[0], sends[0] + sends[1]))
        del sends, recvs
    finally:
        for c in comms:
            vccl.vcclCommDestroy(c)
        t.cuda.empty_cache()
