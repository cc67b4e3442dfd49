"""Seeded random plans against the oracle's FIFO schedule simulation.

Each case draws a rank count, a collective, a dtype and op, a protocol, an
algorithm (the tree for AllReduce), a channel count, a chunk, a workgroup
size and a ragged count (Simple: direct copies into peer buffers on every
other case), runs it on the device with that tuning, and
compares every rank's output bit for bit with the oracle run on the plan the
library reports (channels and chunk after its clamps).  The combinations go
beyond the fixed matrices: odd rank counts with trees and chains, 64- and
1024-thread workgroups, tiny and slot-sized chunks, every channel count up
to the communicator's lane limit (64 for up to 4 ranks)."""
import numpy as np
import pytest

import synthetic_inputs as si
from oracle import simulate as sim
from tests import gpu_harness as H

pytestmark = pytest.mark.gpu

NCASES = 160
COLLS = ("allreduce", "reducescatter", "allgather", "broadcast", "reduce")
DTYPE_OPS = (("int32", "sum"), ("int32", "max"), ("float32", "sum"), ("float32", "max"),
             ("bfloat16", "sum"), ("bfloat16", "max"))
ELEM = {"int32": 4, "float32": 4, "bfloat16": 2}


def cases(seed=2507, count=NCASES):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        R = int(rng.choice([2, 3, 4, 5, 6, 7, 8, 9, 12, 15, 16]))
        coll = COLLS[int(rng.integers(len(COLLS)))]
        dtype, op = DTYPE_OPS[int(rng.integers(len(DTYPE_OPS)))]
        proto = ("simple", "ll", "ll128")[int(rng.integers(3))]
        algo = "tree" if coll == "allreduce" and rng.random() < 0.4 else "ring"
        C = int(rng.integers(1, 65))  # clamped to the lane limit when run
        T = int(rng.choice([64, 128, 256, 512, 1024]))
        chunk = int(rng.choice([0, 256, 1024, 4096, 16384, 65536, 131072, 262144]))
        E = ELEM[dtype]
        # keep the number of steps (and the simulator's time) bounded
        cap = max(64, (chunk or 131072) // E * C * 6)
        n = int(rng.integers(1, min(40000, cap) + 1))
        root = int(rng.integers(R))
        out.append((i, R, coll, dtype, op, proto, algo, C, T, chunk, n, root))
    return out


@pytest.fixture(scope="module")
def vccl():
    import paper_2507_04786_amd as v
    return v


def lane_limit(ncus, R):
    """The library's default: a workgroup per CU, in eights, 32 to 64 lanes."""
    return max(32, min(64, (ncus // R) // 8 * 8))


def test_random_plans_match_oracle(vccl):
    t = H.torch()
    ncus = t.cuda.get_device_properties(0).multi_processor_count
    comm_sets = {}
    try:
        # one communicator set alive at a time (a set's FIFOs take up to about
        # 32 GiB at 16 ranks once trees have run): cases grouped by rank count
        for (i, R, coll, dtype, op, proto, algo, C, T, chunk, n, root) in sorted(cases(), key=lambda c: (c[1], c[0])):
            C = min(C, lane_limit(ncus, R))
            print(f"case {i}: R={R} {coll} {dtype} {op} {proto} {algo} C={C} T={T} chunk={chunk} n={n} "
                  f"root={root} direct={int(proto == 'simple' and i % 2 == 0)}", flush=True)
            if R not in comm_sets:
                for comms in comm_sets.values():
                    for c in comms:
                        vccl.vcclCommDestroy(c)
                comm_sets = {R: vccl.vcclCommInitAll(R)}
            comms = comm_sets[R]
            sn = H.send_len(coll, n, R)
            if dtype == "int32":
                xs = si.rank_inputs(si.WL_TREE_AND_CHAINS, R, dtype, sn, lo=-2**20, hi=2**20, extra=1000 + i)
            else:
                xs = si.rank_inputs(si.WL_TREE_AND_CHAINS, R, dtype, sn, extra=1000 + i)
            sends = [H.to_dev(x) for x in xs]
            recvs = [H.empty_dev(H.recv_len(coll, n, R), dtype) for _ in range(R)]
            # direct copies (Simple) on every other case: the results do not
            # depend on them, the paths they take do
            direct = int(proto == "simple" and i % 2 == 0)
            H.tune(vccl, comms, algo, proto, nchannels=C, chunk=chunk, nthreads=T, direct=direct)
            try:
                H.call(vccl, comms, coll, sends, recvs, n, dtype, op, root)
                t.cuda.synchronize()
                assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess, f"case {i}"
                plan = vccl.vcclCommGetLastPlan(comms[0])
                assert plan["direct"] == direct, f"case {i}: direct {direct} requested, plan {plan}"
            finally:
                H.untune(vccl, comms)
            got = [H.from_dev(r, dtype) for r in recvs]
            want = sim.run(coll, xs, op=op, dtype=dtype, nchannels=plan["nchannels"],
                           chunk_bytes=plan["chunkBytes"], root=root,
                           algo="tree" if plan["algo"] == 1 else "ring")
            for r in range(R):
                if coll == "reduce" and r != root:
                    continue
                assert np.array_equal(got[r].view(np.uint8), want[r].view(np.uint8)), \
                    f"case {i} plan {plan} rank {r}"
    finally:
        for comms in comm_sets.values():
            for c in comms:
                vccl.vcclCommDestroy(c)
