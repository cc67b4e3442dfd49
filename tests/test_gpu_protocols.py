"""The device's FIFO lines decoded by the oracle's line formats (Section III:
LL = 4 B data + 4 B flag per 8 B unit, LL128 = 120 B data + 8 B flag per
128 B line), and the LL128 tear probe (Section III-C: 128-byte stores must not
be split; the protocol is kept only where none tears)."""
import numpy as np
import pytest

import synthetic_inputs as si
from oracle import protocol as pr
from oracle import simulate as sim
from tests import gpu_harness as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vccl():
    import paper_2507_04786_amd as v
    return v


@pytest.mark.parametrize("proto", ["ll", "ll128"])
def test_fifo_lines_follow_the_paper_format(vccl, proto):
    """2 ranks, 1 channel, 100 fp32: rank 0 sends x0[52:100] at connection
    step 0 and the reduced segment [0:52) at step 1; the receiver's FIFO slots
    hold them in the line format with flags 1 and 2."""
    t = H.torch()
    comms = vccl.vcclCommInitAll(2)  # fresh set: connection steps start at 0
    try:
        xs = si.rank_inputs(7, 2, "float32", 100)
        H.tune(vccl, comms, "ring", proto, nchannels=1, chunk=0)
        sends = [H.to_dev(x) for x in xs]
        recvs = [H.empty_dev(100, "float32") for _ in range(2)]
        H.call(vccl, comms, "allreduce", sends, recvs, 100, "float32")
        t.cuda.synchronize()
        out = sim.run("allreduce", xs, dtype="float32", nchannels=1,
                      chunk_bytes=16384 if proto == "ll" else 576000)[0]
        code = vccl.PROTO_NAMES[proto]
        slot = pr.SLOT_BYTES[proto]
        for step, payload in ((0, xs[0][52:100]), (1, out[0:52])):
            nbytes = payload.nbytes
            if proto == "ll":
                nunits = -(-nbytes // 4)
                nunits += nunits % 2  # units travel in pairs
                raw = vccl.vcclCommDebugReadFifo(comms[0], 0, 1, code, step * slot, nunits * 8)
                data, ok = pr.ll_decode(np.frombuffer(raw, dtype="<u8"), step, nbytes)
            else:
                nlines = -(-nbytes // 120)
                raw = vccl.vcclCommDebugReadFifo(comms[0], 0, 1, code, step * slot, nlines * 128)
                data, ok = pr.ll128_decode(np.frombuffer(raw, dtype=np.uint8), step, nbytes)
            assert ok, f"{proto} step {step}: flags are not {step + 1}"
            assert data.tobytes() == payload.tobytes(), f"{proto} step {step}: payload differs"
    finally:
        for c in comms:
            vccl.vcclCommDestroy(c)


def test_ll128_lines_never_tear(vccl):
    # device-scope stores: 4 pairs put writer and reader on different XCDs,
    # 8 pairs on the same XCD; XCD-scope plain stores: pairs share an XCD
    for scope, pairs in ((0, 4), (0, 8), (1, 8), (1, 16)):
        torn, checked, res = vccl.vcclProbeLL128Tear(pairs, 2048, 100, scope)
        assert res == vccl.vcclSuccess, (scope, pairs)
        assert checked == pairs * 2048 * 100
        assert torn == 0, (scope, pairs)
