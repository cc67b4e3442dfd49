"""The algorithmic bytes behind every roofline fraction in bench.py, pinned by
counting them step by step.

Each collective is written out as the primitive sequence every rank runs
(Section V-E step tables: send, recvReduceSend, recvReduceCopySend,
recvCopySend, recv, copySend, recvReduceCopy, and the direct variants of
Section IV-A), and every step is charged what it loads and stores: a read of
the rank's input, a write of its output, a read or write of a FIFO slot at
f bytes per payload byte (1 Simple, 2 LL, 16/15 LL128), or a direct read or
write of a receive buffer.  The sums must equal bench.py's closed forms for
every collective, protocol and rank count."""
from fractions import Fraction

import pytest

import bench

F = {0: Fraction(1), 1: Fraction(2), 2: Fraction(16, 15)}

# per step: (input reads, output writes, FIFO reads, FIFO writes, direct reads, direct writes)
STEP = {
    "send": (1, 0, 0, 1, 0, 0),
    "recvReduceSend": (1, 0, 1, 1, 0, 0),
    "recvReduceCopySend": (1, 1, 1, 1, 0, 0),
    "recvReduceCopySend_direct": (1, 1, 1, 0, 0, 1),  # final value also written into the peer's buffer
    "recvCopySend": (0, 1, 1, 1, 0, 0),
    "directRecvCopySend": (0, 0, 0, 0, 1, 1),         # data already in my buffer: forward it
    "recv": (0, 1, 1, 0, 0, 0),
    "directRecv": (0, 0, 0, 0, 0, 0),                  # the peer wrote my buffer
    "recvReduceCopy": (1, 1, 1, 0, 0, 0),
    "copySend": (1, 1, 0, 1, 0, 0),
    "copySend_direct": (1, 1, 0, 0, 0, 1),
    "send_direct_only": (1, 0, 0, 0, 0, 1),            # root of a direct Broadcast: its local copy moved
    "copy_root_local": (1, 1, 0, 0, 0, 0),             # last rank of a direct Broadcast: root send -> root recv
}


def cost(step, f):
    i, o, fr, fw, dr, dw = STEP[step]
    return i + o + f * (fr + fw) + dr + dw


def ring_allreduce(R, direct):
    steps = ["send"] + ["recvReduceSend"] * (R - 2)
    if direct:
        steps += ["recvReduceCopySend_direct"] + ["directRecvCopySend"] * (R - 2) + ["directRecv"]
    else:
        steps += ["recvReduceCopySend"] + ["recvCopySend"] * (R - 2) + ["recv"]
    return [steps] * R  # every rank, each step on one segment of S / R


def ring_reducescatter(R):
    return [["send"] + ["recvReduceSend"] * (R - 2) + ["recvReduceCopy"]] * R  # steps on blocks of b


def ring_allgather(R, direct):
    if direct:
        return [["copySend_direct"] + ["directRecvCopySend"] * (R - 2) + ["directRecv"]] * R
    return [["copySend"] + ["recvCopySend"] * (R - 2) + ["recv"]] * R


def ring_broadcast(R, direct):
    """The step table's chain: root copySend, middle recvCopySend, last recv."""
    if direct:
        return [["copySend_direct"]] + [["directRecvCopySend"]] * (R - 2) + [["directRecv"]]
    return [["copySend"]] + [["recvCopySend"]] * (R - 2) + [["recv"]]


def kernel_direct_broadcast(R):
    """What the kernel runs under direct Simple: the root only sends, and the
    last rank copies the root's input into the root's receive buffer."""
    return [["send_direct_only"]] + [["directRecvCopySend"]] * (R - 2) + [["copy_root_local"]]


def ring_reduce(R):
    return [["send"]] + [["recvReduceSend"]] * (R - 2) + [["recvReduceCopy"]]


def total(per_rank, f, unit):
    return sum(cost(s, f) for steps in per_rank for s in steps) * unit


@pytest.mark.parametrize("R", range(2, 17))
@pytest.mark.parametrize("proto", [0, 1, 2])
def test_allreduce_bytes(R, proto):
    S = 1 << 20
    f = F[proto]
    for direct in ([0, 1] if proto == 0 else [0]):
        plan = {"proto": proto, "direct": direct, "algo": 0}
        want = total(ring_allreduce(R, direct), f, Fraction(S, R))
        assert bench.alg_bytes_per_launch(plan, R, S) == pytest.approx(float(want), rel=1e-12), (R, proto, direct)
        assert bench.coll_alg_bytes("allreduce", plan, R, S) == pytest.approx(float(want), rel=1e-12)


@pytest.mark.parametrize("R", range(2, 17))
@pytest.mark.parametrize("proto", [0, 1, 2])
def test_chain_and_block_collective_bytes(R, proto):
    S = R << 20  # the larger per-rank buffer; blocks of S / R
    f = F[proto]
    for direct in ([0, 1] if proto == 0 else [0]):
        plan = {"proto": proto, "direct": direct, "algo": 0}
        b = Fraction(S, R)
        cases = {
            "reducescatter": total(ring_reducescatter(R), f, b),
            "allgather": total(ring_allgather(R, direct), f, b),
            "broadcast": total(ring_broadcast(R, direct), f, S),
            "reduce": total(ring_reduce(R), f, S),
        }
        for coll, want in cases.items():
            got = bench.coll_alg_bytes(coll, plan, R, S)
            assert got == pytest.approx(float(want), rel=1e-12), (coll, R, proto, direct)


@pytest.mark.parametrize("R", range(2, 17))
def test_moved_root_copy_reads_the_root_input_once_more(R):
    """The bench's Broadcast fraction is against the step table's (2R - 1) S;
    the kernel, whose last rank makes the root's local copy, moves exactly
    one S more (the root's input is read twice), so the fraction it reports
    is a lower bound of the bytes actually moved per second."""
    S = 1 << 20
    table = total(ring_broadcast(R, 1), Fraction(1), S)
    moved = total(kernel_direct_broadcast(R), Fraction(1), S)
    assert table == (2 * R - 1) * S and moved == table + S


def test_headline_bytes_value():
    """The figure the headline roofline divides by: 36 S at 8 ranks, 64 MiB."""
    plan = {"proto": 0, "direct": 1, "algo": 0}
    assert bench.alg_bytes_per_launch(plan, 8, 64 << 20) == 36 * (64 << 20) == 2415919104
