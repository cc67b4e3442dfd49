"""Seeded random groups (Section II-A: calls between GroupStart and GroupEnd
form one launch): each case issues a random batch of collectives and
Send/Recv pairs among a random number of ranks, with the tuner's plans,
once call by call and once as one group.  Every collective must give the
same bits both ways (a grouped collective keeps its plan), int32 sums must
equal the brute-force definition, and every Send/Recv pair must deliver the
sender's buffer unchanged.  This exercises the work list: placement of
items from many collectives on lanes, lane starts, argument tables and
mixed protocols and algorithms in one launch."""
import numpy as np
import pytest

import synthetic_inputs as si
from oracle import definitions as defs
from tests import gpu_harness as H

pytestmark = pytest.mark.gpu

NCASES = 24
COLLS = ("allreduce", "reducescatter", "allgather", "broadcast", "reduce")
DTYPES = ("int32", "float32", "bfloat16")


def cases(seed=4786, count=NCASES):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        R = int(rng.choice([2, 3, 4, 6, 8, 11, 16]))
        batch = []
        for k in range(int(rng.integers(1, 11))):
            coll = COLLS[int(rng.integers(len(COLLS)))]
            dtype = DTYPES[int(rng.integers(len(DTYPES)))]
            lg = rng.uniform(2, 21)  # counts from 4 to 2M elements, log-uniform
            n = max(1, int(2 ** lg) // (R if coll in ("allgather", "reducescatter") else 1))
            batch.append((coll, dtype, n, int(rng.integers(R))))
        npairs = int(rng.integers(0, 2 * R))
        pairs = [(int(rng.integers(R)), int(rng.integers(R)), int(rng.integers(1, 300000))) for _ in range(npairs)]
        out.append((i, R, batch, pairs))
    return out


def _inputs(i, k, R, coll, dtype, n):
    sn = H.send_len(coll, n, R)
    if dtype == "int32":
        return si.rank_inputs(si.WL_GROUPED, R, dtype, sn, lo=-2**20, hi=2**20, extra=9000 + 100 * i + k)
    return si.rank_inputs(si.WL_GROUPED, R, dtype, sn, extra=9000 + 100 * i + k)


def _issue(vccl, comms, batch, inputs, pairs, grouped):
    t = H.torch()
    R = len(comms)
    sends = [[H.to_dev(x) for x in xs] for xs in inputs]
    recvs = [[H.empty_dev(H.recv_len(c, n, R), d) for _ in range(R)] for (c, d, n, _), xs in zip(batch, inputs)]
    psend = [H.to_dev(np.arange(cnt, dtype=np.int32) * 7 + 1000 * a + b) for (a, b, cnt) in pairs]
    precv = [H.empty_dev(cnt, "int32") for (_, _, cnt) in pairs]
    t.cuda.synchronize()
    if grouped:
        vccl.vcclGroupStart()
    for (coll, dtype, n, root), s, r in zip(batch, sends, recvs):
        H.call(vccl, comms, coll, s, r, n, dtype, "sum", root)
    # outside a group a pair is issued as soon as its second side is posted
    for (a, b, cnt), s, r in zip(pairs, psend, precv):
        vccl.vcclSend(s, cnt, vccl.vcclInt32, b, comms[a])
        vccl.vcclRecv(r, cnt, vccl.vcclInt32, a, comms[b])
    if grouped:
        vccl.vcclGroupEnd()
    t.cuda.synchronize()
    assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess
    outs = [[H.from_dev(x, d) for x in rs] for rs, (_, d, _, _) in zip(recvs, batch)]
    pouts = [H.from_dev(x, "int32") for x in precv]
    return outs, pouts


@pytest.fixture(scope="module")
def vccl():
    import paper_2507_04786_amd as v
    return v


def test_random_groups_equal_per_call_and_definitions(vccl):
    comm_sets = {}
    try:
        # one communicator set alive at a time, cases grouped by rank count
        for (i, R, batch, pairs) in sorted(cases(), key=lambda c: (c[1], c[0])):
            print(f"case {i}: R={R} batch={batch} pairs={len(pairs)}", flush=True)
            if R not in comm_sets:
                for comms in comm_sets.values():
                    for c in comms:
                        vccl.vcclCommDestroy(c)
                comm_sets = {R: vccl.vcclCommInitAll(R)}
            comms = comm_sets[R]
            inputs = [_inputs(i, k, R, c, d, n) for k, (c, d, n, _) in enumerate(batch)]
            per_call, p1 = _issue(vccl, comms, batch, inputs, pairs, grouped=False)
            grouped, p2 = _issue(vccl, comms, batch, inputs, pairs, grouped=True)
            for k, (coll, dtype, n, root) in enumerate(batch):
                ranks = [root] if coll == "reduce" else range(R)
                for r in ranks:
                    assert np.array_equal(grouped[k][r].view(np.uint8), per_call[k][r].view(np.uint8)), \
                        f"case {i} item {k} {coll} {dtype} n={n} rank {r}"
                if dtype == "int32" and coll == "allreduce":
                    want = defs.allreduce(inputs[k], "sum", "int32")
                    for r in range(R):
                        assert np.array_equal(grouped[k][r], want[r]), f"case {i} item {k} int32 sum rank {r}"
                if coll == "allgather":
                    want = defs.allgather(inputs[k])
                    for r in range(R):
                        assert np.array_equal(grouped[k][r].view(np.uint8), want[r].view(np.uint8)), \
                            f"case {i} item {k} allgather rank {r}"
            for (a, b, cnt), x, y in zip(pairs, p1, p2):
                src = np.arange(cnt, dtype=np.int32) * 7 + 1000 * a + b
                assert np.array_equal(x, src) and np.array_equal(y, src), f"case {i} pair {a}->{b} count {cnt}"
    finally:
        for comms in comm_sets.values():
            for c in comms:
                vccl.vcclCommDestroy(c)
