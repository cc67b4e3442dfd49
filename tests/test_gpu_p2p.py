"""Send/Recv through the C ABI (Section II-A point-to-point and group calls;
Section IV-A P2P_DIRECT): every transfer is a bitwise copy, a grouped
all-to-all matches the oracle's definition, bytes around the receive buffer
stay untouched, and matching errors are reported."""
import numpy as np
import pytest

import synthetic_inputs as si
from oracle import definitions as defs
from tests import gpu_harness as H

pytestmark = pytest.mark.gpu

GUARD = 64  # bytes checked on each side of a receive buffer


@pytest.fixture(scope="module")
def vccl():
    import paper_2507_04786_amd as v
    return v


def _code(vccl, dtype):
    return vccl.DTYPE_NAMES[dtype]


def _guarded(t, n, dtype, fill=0xA5):
    """A receive buffer of n elements with GUARD bytes on both sides."""
    E = H.ELEM[dtype]
    raw = t.full((n * E + 2 * GUARD,), fill, dtype=t.uint8, device="cuda")
    return raw, raw[GUARD:GUARD + n * E]


def _check_guards(raw, fill=0xA5):
    h = raw.cpu().numpy()
    assert (h[:GUARD] == fill).all() and (h[-GUARD:] == fill).all(), "bytes outside the receive buffer changed"


def test_pairs_outside_a_group(vccl):
    t = H.torch()
    R = 4
    comms = vccl.vcclCommInitAll(R)
    try:
        cases = [(1, "int32"), (17, "bfloat16"), (1001, "float32"), (70001, "bfloat16"), (600001, "float32")]
        k = 0
        for a in range(R):
            for b in range(R):
                n, dtype = cases[k % len(cases)]
                k += 1
                x = si.rank_inputs(si.WL_P2P, 1, dtype, n, extra=a * 16 + b)[0]
                src = H.to_dev(x)
                raw, dst = _guarded(t, n, dtype)
                t.cuda.synchronize()
                vccl.vcclSend(src, n, _code(vccl, dtype), b, comms[a])
                vccl.vcclRecv(dst, n, _code(vccl, dtype), a, comms[b])
                t.cuda.synchronize()
                assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess
                got = dst.cpu().numpy()
                want = defs.sendrecv(x)
                assert got.tobytes() == want.tobytes(), (a, b, n, dtype)
                _check_guards(raw)
                plan = vccl.vcclCommGetLastPlan(comms[0])
                assert plan["proto"] == 0 and plan["direct"] == 1
    finally:
        for c in comms:
            vccl.vcclCommDestroy(c)


@pytest.mark.parametrize("dtype,n", [("bfloat16", 1000), ("float32", 4099), ("int32", 65543), ("float32", 1)])
def test_grouped_alltoall(vccl, dtype, n):
    t = H.torch()
    R = 8
    comms = vccl.vcclCommInitAll(R)
    try:
        kw = dict(lo=-2**20, hi=2**20) if dtype == "int32" else {}
        xs = si.rank_inputs(si.WL_P2P, R, dtype, R * n, extra=n, **kw)
        sends = [H.to_dev(x) for x in xs]
        E = H.ELEM[dtype]
        outs = [_guarded(t, R * n, dtype) for _ in range(R)]
        t.cuda.synchronize()
        code = _code(vccl, dtype)
        vccl.vcclGroupStart()
        for a in range(R):
            for b in range(R):
                vccl.vcclSend(sends[a][b * n:(b + 1) * n], n, code, b, comms[a])
                vccl.vcclRecv(outs[b][1][a * n * E:(a + 1) * n * E], n, code, a, comms[b])
        vccl.vcclGroupEnd()
        t.cuda.synchronize()
        assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess
        plan = vccl.vcclCommGetLastPlan(comms[0])
        assert plan["ncolls"] == R * R
        want = defs.alltoall(xs)
        for b in range(R):
            got = outs[b][1].cpu().numpy()
            assert got.tobytes() == want[b].tobytes(), (dtype, n, b)
            _check_guards(outs[b][0])
    finally:
        for c in comms:
            vccl.vcclCommDestroy(c)


def test_group_mixes_collectives_and_transfers(vccl):
    t = H.torch()
    R = 4
    comms = vccl.vcclCommInitAll(R)
    try:
        n = 5003
        xs = si.rank_inputs(si.WL_P2P, R, "int32", n, lo=-2**20, hi=2**20, extra=99)
        ar_in = [H.to_dev(x) for x in xs]
        ar_out = [H.empty_dev(n, "int32") for _ in range(R)]
        ring = [H.empty_dev(n, "int32") for _ in range(R)]
        t.cuda.synchronize()
        vccl.vcclGroupStart()
        for r in range(R):
            vccl.vcclAllReduce(ar_in[r], ar_out[r], n, vccl.vcclInt32, vccl.vcclSum, comms[r])
        for r in range(R):  # every rank passes its input to its successor
            vccl.vcclSend(ar_in[r], n, vccl.vcclInt32, (r + 1) % R, comms[r])
            vccl.vcclRecv(ring[(r + 1) % R], n, vccl.vcclInt32, r, comms[(r + 1) % R])
        vccl.vcclGroupEnd()
        t.cuda.synchronize()
        assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess
        want = defs.allreduce(xs, "sum", "int32")
        for r in range(R):
            assert np.array_equal(H.from_dev(ar_out[r], "int32"), want[r])
            assert np.array_equal(H.from_dev(ring[r], "int32"), xs[(r - 1) % R])
    finally:
        for c in comms:
            vccl.vcclCommDestroy(c)


def test_matching_errors(vccl):
    t = H.torch()
    R = 2
    comms = vccl.vcclCommInitAll(R)
    try:
        x = t.zeros(64, device="cuda")
        y = t.zeros(64, device="cuda")
        with pytest.raises(vccl.VcclError) as e:
            vccl.vcclSend(x, 8, vccl.vcclFloat32, 2, comms[0])  # no rank 2
        assert e.value.code == vccl.vcclInvalidArgument
        with pytest.raises(vccl.VcclError) as e:
            vccl.vcclSend(x[1:].view(t.uint8)[1:], 4, vccl.vcclFloat32, 1, comms[0])  # misaligned
        assert e.value.code == vccl.vcclInvalidArgument
        vccl.vcclSend(x, 8, vccl.vcclFloat32, 1, comms[0])
        with pytest.raises(vccl.VcclError) as e:
            vccl.vcclRecv(y, 12, vccl.vcclFloat32, 0, comms[1])  # count differs
        assert e.value.code == vccl.vcclInvalidUsage
        vccl.vcclGroupStart()
        vccl.vcclSend(x, 8, vccl.vcclFloat32, 1, comms[0])  # never received
        with pytest.raises(vccl.VcclError) as e:
            vccl.vcclGroupEnd()
        assert e.value.code == vccl.vcclInvalidUsage
        # the set still works afterwards
        x.fill_(3.0)
        vccl.vcclSend(x, 64, vccl.vcclFloat32, 1, comms[0])
        vccl.vcclRecv(y, 64, vccl.vcclFloat32, 0, comms[1])
        t.cuda.synchronize()
        assert bool((y == 3.0).all())
        assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess
    finally:
        for c in comms:
            vccl.vcclCommDestroy(c)
