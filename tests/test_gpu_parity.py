"""Parity of the HIP path with the CPU oracle, element by element, through the
C ABI.  Integer work and every reduction is compared bit for bit: the
schedule fixes the association order of float sums, and the oracle follows
the same schedule.  Sizes span several channels, loops and a ragged tail."""
import numpy as np
import pytest

import synthetic_inputs as si
from oracle import definitions as defs
from oracle import folds
from oracle import simulate as sim
from tests import gpu_harness as H

pytestmark = pytest.mark.gpu

PROTOS = ["simple", "ll", "ll128"]


@pytest.fixture(scope="module")
def vccl():
    import paper_2507_04786_amd as v
    return v


_CLIQUES = {}


@pytest.fixture(scope="module")
def comms_for(vccl):
    def get(R, scope="auto"):
        key = (R, scope)
        if key not in _CLIQUES:
            _CLIQUES[key] = H.init_comms(vccl, R, scope)
        return _CLIQUES[key]
    yield get
    for cs in _CLIQUES.values():
        for c in cs:
            vccl.vcclCommDestroy(c)
    _CLIQUES.clear()


def _inputs(R, dtype, n, wl=2, extra=0):
    if dtype == "int32":
        return si.rank_inputs(wl, R, "int32", n, lo=-2**20, hi=2**20, extra=extra)
    return si.rank_inputs(wl, R, dtype, n, extra=extra)


def _run(vccl, comms, coll, xs, count, dtype, op="sum", root=0):
    R = len(comms)
    t = H.torch()
    sends = [H.to_dev(x) for x in xs]
    recvs = [H.empty_dev(H.recv_len(coll, count, R), dtype) for _ in range(R)]
    H.call(vccl, comms, coll, sends, recvs, count, dtype, op, root)
    t.cuda.synchronize()
    assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess
    return [H.from_dev(r, dtype) for r in recvs]


def _assert_bits(got, want, what):
    got = np.ascontiguousarray(got)
    want = np.ascontiguousarray(want)
    assert got.shape == want.shape, (what, got.shape, want.shape)
    if not np.array_equal(got.view(np.uint8), want.view(np.uint8)):
        gv = got.view(np.uint8).reshape(len(got), -1)
        wv = want.view(np.uint8).reshape(len(want), -1)
        bad = np.nonzero((gv != wv).any(axis=1))[0]
        raise AssertionError(f"{what}: {len(bad)} of {len(got)} elements differ; first {bad[:8].tolist()} "
                             f"got {got[bad[:4]].tolist()} want {want[bad[:4]].tolist()}")


def test_ring_allreduce_4_ranks_int32_config(vccl, comms_for):
    """Ring AllReduce sum, 4 ranks, int32 U[-1000, 1000], 65,536 elements per
    rank, Simple, 1 channel, 8 KiB chunk, 8 slots."""
    R, n = 4, 65536
    comms = comms_for(R)
    xs = si.rank_inputs(si.WL_RING_AR_SMALL, R, "int32", n, lo=-1000, hi=1000)
    H.tune(vccl, comms, "ring", "simple", nchannels=1, chunk=8192)
    try:
        got = _run(vccl, comms, "allreduce", xs, n, "int32")
        info = vccl.vcclCommGetLastPlan(comms[0])
    finally:
        H.untune(vccl, comms)
    assert info["proto"] == 0 and info["nchannels"] == 1 and info["chunkBytes"] == 8192
    want = sim.run("allreduce", xs, dtype="int32", nchannels=1, chunk_bytes=8192)
    brute = defs.allreduce(xs, "sum", "int32")
    for r in range(R):
        _assert_bits(got[r], want[r], f"rank {r}")
        _assert_bits(got[r], brute[r], f"rank {r} brute force")


RING_CASES = [
    # R, n, channels, chunk bytes
    (2, 1, 1, 256), (2, 1000, 2, 256), (3, 4099, 3, 512), (4, 70001, 4, 4096),
    (8, 65543, 5, 2048), (16, 33333, 2, 1024), (8, 0, 1, 1024),
]


@pytest.mark.parametrize("proto", PROTOS)
@pytest.mark.parametrize("dtype,op", [("int32", "sum"), ("float32", "sum"), ("bfloat16", "sum"),
                                      ("float32", "max"), ("bfloat16", "max"), ("int32", "max")])
def test_ring_allreduce_matrix(vccl, comms_for, proto, dtype, op):
    for (R, n, C, chunk) in RING_CASES:
        comms = comms_for(R)
        xs = _inputs(R, dtype, n, extra=R * 7 + C)
        H.tune(vccl, comms, "ring", proto, nchannels=C, chunk=chunk)
        try:
            got = _run(vccl, comms, "allreduce", xs, n, dtype, op)
        finally:
            H.untune(vccl, comms)
        want = sim.run("allreduce", xs, op=op, dtype=dtype, nchannels=C, chunk_bytes=chunk)
        for r in range(R):
            _assert_bits(got[r], want[r], f"{proto} {dtype} {op} R={R} n={n} C={C} rank {r}")


@pytest.mark.parametrize("proto", PROTOS)
@pytest.mark.parametrize("coll", ["reducescatter", "allgather", "broadcast", "reduce"])
@pytest.mark.parametrize("dtype,op", [("int32", "sum"), ("bfloat16", "sum"), ("float32", "sum"), ("bfloat16", "max")])
def test_ring_collectives_matrix(vccl, comms_for, proto, coll, dtype, op):
    for (R, n, C, chunk) in [(2, 3, 1, 256), (4, 1001, 2, 512), (16, 2050, 3, 1024), (5, 40000, 4, 4096)]:
        comms = comms_for(R)
        sn = H.send_len(coll, n, R)
        xs = _inputs(R, dtype, sn, wl=3, extra=R + n)
        roots = sorted({0, R // 2, R - 1}) if coll in ("broadcast", "reduce") else [0]
        for root in roots:
            H.tune(vccl, comms, "ring", proto, nchannels=C, chunk=chunk)
            try:
                got = _run(vccl, comms, coll, xs, n, dtype, op, root)
            finally:
                H.untune(vccl, comms)
            want = sim.run(coll, xs, op=op, dtype=dtype, nchannels=C, chunk_bytes=chunk, root=root)
            for r in range(R):
                if coll == "reduce" and r != root:
                    continue
                _assert_bits(got[r], want[r], f"{coll} {proto} {dtype} {op} R={R} n={n} C={C} root={root} rank {r}")


@pytest.mark.parametrize("proto", PROTOS)
@pytest.mark.parametrize("dtype,op", [("int32", "sum"), ("bfloat16", "sum"), ("float32", "sum"), ("int32", "max")])
def test_tree_allreduce_matrix(vccl, comms_for, proto, dtype, op):
    for (R, n, C, chunk) in [(2, 5, 1, 256), (4, 3001, 2, 512), (7, 9000, 3, 1024), (16, 70001, 4, 4096),
                             (16, 100, 2, 256)]:
        comms = comms_for(R)
        xs = _inputs(R, dtype, n, wl=3, extra=n)
        H.tune(vccl, comms, "tree", proto, nchannels=C, chunk=chunk)
        try:
            got = _run(vccl, comms, "allreduce", xs, n, dtype, op)
        finally:
            H.untune(vccl, comms)
        want = sim.run("allreduce", xs, op=op, dtype=dtype, nchannels=C, chunk_bytes=chunk, algo="tree")
        for r in range(R):
            _assert_bits(got[r], want[r], f"tree {proto} {dtype} {op} R={R} n={n} C={C} rank {r}")


@pytest.mark.parametrize("R", [4, 8, 16])
def test_default_plans_match_oracle(vccl, comms_for, R):
    """Whatever the measured tuner picks (ring or tree, any protocol, up to 32
    channels, tabulated chunks and workgroup sizes) at sizes across the
    8 B .. 4 MiB range, with ragged counts: every collective against the
    oracle's folds for the plan it reports."""
    comms = comms_for(R)
    for lg in (3, 6, 10, 13, 16, 17, 18, 20, 21, 22):
        for coll, dtype in (("allreduce", "float32"), ("allreduce", "bfloat16"), ("reducescatter", "float32"),
                            ("allgather", "float32"), ("broadcast", "bfloat16"), ("reduce", "float32")):
            E = H.ELEM[dtype]
            per = (1 << lg) // E // (R if coll in ("allgather", "reducescatter") else 1)
            n = max(1, per - 3)
            xs = _inputs(R, dtype, H.send_len(coll, n, R), wl=2, extra=lg * 100 + R)
            root = R // 2 if coll in ("broadcast", "reduce") else 0
            got = _run(vccl, comms, coll, xs, n, dtype, "sum", root)
            plan = vccl.vcclCommGetLastPlan(comms[0])
            what = f"default plan {plan} {coll} {dtype} R={R} n={n}"
            if coll == "allreduce":
                if plan["algo"] == 1:
                    want = folds.tree_allreduce(xs, "sum", dtype, plan["nchannels"])
                else:
                    want = folds.ring_allreduce(xs, "sum", dtype, plan["nchannels"], plan["chunkBytes"] // E)
                for r in range(R):
                    _assert_bits(got[r], want, f"{what} rank {r}")
            elif coll == "reducescatter":
                for r in range(R):
                    _assert_bits(got[r], folds.ring_reducescatter(xs, "sum", dtype, r), f"{what} rank {r}")
            elif coll == "reduce":
                _assert_bits(got[root], folds.ring_reduce(xs, "sum", dtype, root), what)
            elif coll == "allgather":
                want = defs.allgather(xs)
                for r in range(R):
                    _assert_bits(got[r], want[r], f"{what} rank {r}")
            else:
                for r in range(R):
                    _assert_bits(got[r], xs[root], f"{what} rank {r}")


@pytest.mark.parametrize("split", [True, False])
def test_tree_halves_and_fused_channels(vccl, comms_for, split):
    """A Simple tree launched alone runs each channel as concurrent up and
    down halves on two lanes (VCCL_TREE_SPLIT=0: one fused workgroup per rank
    and channel); both give the oracle's bits for every dtype and op."""
    import os
    old = os.environ.get("VCCL_TREE_SPLIT")
    os.environ["VCCL_TREE_SPLIT"] = "1" if split else "0"
    try:
        for R in (4, 8, 16):
            comms = vccl.vcclCommInitAll(R)
            try:
                for dtype, op, n, C, chunk in (("float32", "sum", 100003, 3, 4096), ("bfloat16", "sum", 50001, 8, 2048),
                                               ("int32", "max", 70001, 16, 1024)):
                    xs = _inputs(R, dtype, n, wl=3, extra=R + C)
                    H.tune(vccl, comms, "tree", "simple", nchannels=C, chunk=chunk)
                    try:
                        got = _run(vccl, comms, "allreduce", xs, n, dtype, op)
                        info = vccl.vcclCommGetLastPlan(comms[0])
                    finally:
                        H.untune(vccl, comms)
                    lanes = 8 * ((C + 7) // 8) + C if split else C
                    assert info["nlanes"] == lanes, (R, C, info)
                    want = folds.tree_allreduce(xs, op, dtype, C)
                    for r in range(R):
                        _assert_bits(got[r], want, f"tree split={split} {dtype} {op} R={R} C={C} rank {r}")
            finally:
                for c in comms:
                    vccl.vcclCommDestroy(c)
    finally:
        if old is None:
            del os.environ["VCCL_TREE_SPLIT"]
        else:
            os.environ["VCCL_TREE_SPLIT"] = old


def test_wide_split_tree_runs_from_the_work_list(vccl):
    """With the lane limit raised to 64 (VCCL_MAX_CHANNELS), a split tree of
    more than 16 channels takes more lanes (8 ceil(C / 8) + C) than the launch
    descriptor holds and runs from the device work list: 24 and 32 channels
    at 8 and 16 ranks, every rank against the oracle's tree fold."""
    import os
    old = os.environ.get("VCCL_MAX_CHANNELS")
    os.environ["VCCL_MAX_CHANNELS"] = "64"
    try:
        for R in (8, 16):
            comms = vccl.vcclCommInitAll(R)
            try:
                for dtype, op, n, C, chunk in (("bfloat16", "sum", 300007, 32, 4096),
                                               ("float32", "sum", 200003, 24, 4096),
                                               ("int32", "max", 150001, 32, 2048)):
                    print(f"wide split tree R={R} {dtype} {op} C={C}", flush=True)
                    xs = _inputs(R, dtype, n, wl=3, extra=R * 7 + C)
                    H.tune(vccl, comms, "tree", "simple", nchannels=C, chunk=chunk)
                    try:
                        got = _run(vccl, comms, "allreduce", xs, n, dtype, op)
                        info = vccl.vcclCommGetLastPlan(comms[0])
                    finally:
                        H.untune(vccl, comms)
                    assert info["nchannels"] == C and info["nlanes"] == 8 * ((C + 7) // 8) + C, (R, C, info)
                    want = folds.tree_allreduce(xs, op, dtype, C)
                    for r in range(R):
                        _assert_bits(got[r], want, f"wide split tree {dtype} {op} R={R} C={C} rank {r}")
            finally:
                for c in comms:
                    vccl.vcclCommDestroy(c)
    finally:
        if old is None:
            del os.environ["VCCL_MAX_CHANNELS"]
        else:
            os.environ["VCCL_MAX_CHANNELS"] = old


@pytest.mark.parametrize("R,P", [(4, 2), (8, 2), (8, 4), (16, 4), (16, 8), (12, 3)])
def test_chain_tree_topology(vccl, R, P):
    """VCCL_TREE_RANKS_PER_NODE=P: chains within groups of P ranks, the double
    binary tree across them; every protocol, split and fused channels, sum and
    max, against the oracle's fold on the same topology."""
    import os
    old = os.environ.get("VCCL_TREE_RANKS_PER_NODE")
    os.environ["VCCL_TREE_RANKS_PER_NODE"] = str(P)
    try:
        comms = vccl.vcclCommInitAll(R)
    finally:
        if old is None:
            del os.environ["VCCL_TREE_RANKS_PER_NODE"]
        else:
            os.environ["VCCL_TREE_RANKS_PER_NODE"] = old
    try:
        for proto, dtype, op, n, C, chunk in (("simple", "float32", "sum", 40001, 4, 1024),
                                              ("ll", "bfloat16", "sum", 9001, 3, 0),
                                              ("ll128", "float32", "sum", 30001, 2, 0),
                                              ("simple", "int32", "max", 5001, 1, 512)):
            xs = _inputs(R, dtype, n, wl=3, extra=R * 10 + P)
            H.tune(vccl, comms, "tree", proto, nchannels=C, chunk=chunk)
            try:
                got = _run(vccl, comms, "allreduce", xs, n, dtype, op)
                info = vccl.vcclCommGetLastPlan(comms[0])
            finally:
                H.untune(vccl, comms)
            assert info["treeRanksPerNode"] == P and info["algo"] == 1
            want = folds.tree_allreduce(xs, op, dtype, C, ranks_per_node=P)
            for r in range(R):
                _assert_bits(got[r], want, f"chain tree R={R} P={P} {proto} {dtype} {op} rank {r}")
    finally:
        for c in comms:
            vccl.vcclCommDestroy(c)


@pytest.mark.parametrize("coll", ["allreduce", "allgather", "broadcast"])
def test_direct_variants_match(vccl, comms_for, coll):
    """P2P_DIRECT-style copies give the same bits as the FIFO path."""
    for (R, n, C, chunk) in [(2, 1000, 1, 512), (8, 65543, 4, 4096), (16, 20000, 3, 2048)]:
        comms = comms_for(R)
        xs = _inputs(R, "float32", n, extra=11)
        H.tune(vccl, comms, "ring", "simple", nchannels=C, chunk=chunk, direct=1)
        try:
            got = _run(vccl, comms, coll, xs, n, "float32", "sum", root=R - 1)
            assert vccl.vcclCommGetLastPlan(comms[0])["direct"] == 1
        finally:
            H.untune(vccl, comms)
        want = sim.run(coll, xs, dtype="float32", nchannels=C, chunk_bytes=chunk, root=R - 1)
        for r in range(R):
            _assert_bits(got[r], want[r], f"direct {coll} R={R} n={n} rank {r}")


def test_misaligned_and_subnormal_buffers(vccl, comms_for):
    """Element-aligned but not 16-byte-aligned buffers, subnormal inputs."""
    t = H.torch()
    R, n = 4, 1234
    comms = comms_for(R)
    xs = si.rank_inputs(5, R, "float32", n)
    xs[0][:10] = np.float32(1e-40)
    xs[1][:10] = np.float32(-3e-39)
    for proto in PROTOS:
        sends, recvs = [], []
        for x in xs:
            big = H.to_dev(np.concatenate([np.zeros(3, np.float32), x]))
            sends.append(big[3:])
            recvs.append(H.empty_dev(n + 1, "float32")[1:])
        H.tune(vccl, comms, "ring", proto, nchannels=2, chunk=1024)
        try:
            H.call(vccl, comms, "allreduce", sends, recvs, n, "float32")
            t.cuda.synchronize()
        finally:
            H.untune(vccl, comms)
        want = sim.run("allreduce", xs, dtype="float32", nchannels=2, chunk_bytes=1024)
        for r in range(R):
            _assert_bits(H.from_dev(recvs[r], "float32"), want[r], f"misaligned {proto} rank {r}")


@pytest.mark.parametrize("coll", ["allreduce", "allgather", "reducescatter", "broadcast"])
def test_in_place(vccl, comms_for, coll):
    t = H.torch()
    R, n = 8, 5000
    comms = comms_for(R)
    xs = _inputs(R, "int32", H.send_len(coll, n, R), extra=3)
    for proto in PROTOS:
        bufs, sends, recvs = [], [], []
        for r, x in enumerate(xs):
            if coll == "allgather":
                b = H.empty_dev(n * R, "int32")
                b[r * n:(r + 1) * n].copy_(H.to_dev(x))
                sends.append(b[r * n:(r + 1) * n])
                recvs.append(b)
            elif coll == "reducescatter":
                b = H.to_dev(x)
                sends.append(b)
                recvs.append(b[r * n:(r + 1) * n])
            else:
                b = H.to_dev(x)
                sends.append(b)
                recvs.append(b)
            bufs.append(b)
        H.tune(vccl, comms, "ring", proto, nchannels=3, chunk=2048)
        try:
            H.call(vccl, comms, coll, sends, recvs, n, "int32", "sum", root=2)
            t.cuda.synchronize()
        finally:
            H.untune(vccl, comms)
        want = sim.run(coll, xs, dtype="int32", nchannels=3, chunk_bytes=2048, root=2)
        for r in range(R):
            _assert_bits(H.from_dev(recvs[r], "int32"), want[r], f"in-place {coll} {proto} rank {r}")


def test_reduce_leaves_non_root_untouched(vccl, comms_for):
    t = H.torch()
    R, n = 4, 3000
    comms = comms_for(R)
    xs = _inputs(R, "float32", n)
    sends = [H.to_dev(x) for x in xs]
    recvs = [H.empty_dev(n, "float32", fill=0x77) for _ in range(R)]
    H.call(vccl, comms, "reduce", sends, recvs, n, "float32", "sum", root=1)
    t.cuda.synchronize()
    want = folds.ring_reduce(xs, "sum", "float32", 1)
    _assert_bits(H.from_dev(recvs[1], "float32"), want, "reduce root")
    for r in (0, 2, 3):
        assert (recvs[r].view(t.uint8) == 0x77).all().item()


def test_zero_counts_are_no_ops(vccl, comms_for):
    """A count of 0 is a legal call (null buffers allowed, as in the per-call
    API of Section II-A): it is matched across ranks like any other call,
    launches nothing and writes nothing; inside a group it leaves the
    group's other work intact (one collective in the launch)."""
    R = 4
    comms = comms_for(R)
    t = H.torch()
    for coll in ("allreduce", "reducescatter", "allgather", "broadcast", "reduce"):
        H.call(vccl, comms, coll, [None] * R, [None] * R, 0, "float32", "sum", 1)
    vccl.vcclSend(None, 0, vccl.vcclInt32, 1, comms[0])
    vccl.vcclRecv(None, 0, vccl.vcclInt32, 0, comms[1])
    t.cuda.synchronize()
    assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess
    n = 1000
    xs = _inputs(R, "int32", n, extra=71)
    sends = [H.to_dev(x) for x in xs]
    recvs = [H.empty_dev(n, "int32") for _ in range(R)]
    guard = [H.empty_dev(64, "int32") for _ in range(R)]
    vccl.vcclGroupStart()
    H.call(vccl, comms, "allgather", sends, guard, 0, "int32")
    H.call(vccl, comms, "allreduce", sends, recvs, n, "int32")
    H.call(vccl, comms, "broadcast", sends, guard, 0, "int32", root=2)
    vccl.vcclSend(sends[3], 0, vccl.vcclInt32, 2, comms[3])
    vccl.vcclRecv(guard[2], 0, vccl.vcclInt32, 3, comms[2])
    vccl.vcclGroupEnd()
    t.cuda.synchronize()
    assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess
    assert vccl.vcclCommGetLastPlan(comms[0])["ncolls"] == 1
    want = defs.allreduce(xs, "sum", "int32")
    for r in range(R):
        _assert_bits(H.from_dev(recvs[r], "int32"), want[r], f"allreduce beside zero counts, rank {r}")
        g = H.from_dev(guard[r], "int32").view(np.uint32)
        assert (g == 0x5A5A5A5A).all(), f"a zero-count call wrote rank {r}'s buffer"


def test_large_allreduce_sampled_and_bounded(vccl, comms_for):
    """8 ranks, fp32 N(0,1), 64 MiB per rank: sampled elements against the
    oracle's closed-form fold, every element against the fp64 sum within
    the recursive-summation bound, all ranks identical."""
    t = H.torch()
    R, n = 8, 16 * 1024 * 1024
    comms = comms_for(R)
    xs = si.rank_inputs(si.WL_RING_AR_SWEEP, R, "float32", n)
    sends = [H.to_dev(x) for x in xs]
    recvs = [H.empty_dev(n, "float32") for _ in range(R)]
    for proto in PROTOS:
        H.tune(vccl, comms, "ring", proto, nchannels=16, chunk=0)
        try:
            H.call(vccl, comms, "allreduce", sends, recvs, n, "float32")
            t.cuda.synchronize()
            info = vccl.vcclCommGetLastPlan(comms[0])
        finally:
            H.untune(vccl, comms)
        assert vccl.vcclCommGetAsyncError(comms[0]) == vccl.vcclSuccess
        out0 = H.from_dev(recvs[0], "float32")
        for r in range(1, R):
            assert t.equal(recvs[r], recvs[0]), f"rank {r} differs"
        rng = np.random.default_rng(99)
        idx = np.unique(np.concatenate([rng.integers(0, n, 20000), np.arange(64), np.arange(n - 64, n)]))
        want = folds.ring_allreduce(xs, "sum", "float32", info["nchannels"], info["chunkBytes"] // 4, idx=idx)
        _assert_bits(out0[idx], want, f"large {proto} sampled")
        err = np.abs(out0.astype(np.float64) - defs.fp64_sum(xs, "float32"))
        assert (err <= defs.sum_error_bound(xs, "float32") * (1 + 1e-9)).all()


@pytest.mark.parametrize("proto", PROTOS)
def test_device_scope_path(vccl, comms_for, proto):
    """VCCL_SCOPE=device: every store device-coherent (sc1), the path for
    lanes whose workgroups are not known to share an XCD."""
    for (R, n, C, chunk) in [(4, 70001, 4, 4096), (16, 3001, 3, 512), (8, 65543, 9, 2048)]:
        comms = comms_for(R, "device")
        for coll, algo in (("allreduce", "ring"), ("allreduce", "tree"), ("reducescatter", "ring"),
                           ("allgather", "ring")):
            xs = _inputs(R, "float32", H.send_len(coll, n, R), extra=5)
            H.tune(vccl, comms, algo, proto, nchannels=C, chunk=chunk)
            try:
                got = _run(vccl, comms, coll, xs, n, "float32")
                assert vccl.vcclCommGetLastPlan(comms[0])["scope"] == 0
            finally:
                H.untune(vccl, comms)
            want = sim.run(coll, xs, dtype="float32", nchannels=C, chunk_bytes=chunk, algo=algo)
            for r in range(R):
                _assert_bits(got[r], want[r], f"device scope {coll} {algo} {proto} R={R} rank {r}")


@pytest.mark.parametrize("proto", PROTOS)
def test_xcd_scope_is_the_default_and_reuses_slots_safely(vccl, comms_for, proto):
    """Default XCD scope (plain stores into the lane's L2, sc1 loads): tiny
    chunks make every FIFO slot and counter line be rewritten and re-read
    hundreds of times in one launch, in every algorithm."""
    R, n = 4, 60001
    comms = comms_for(R)
    for coll, algo in (("allreduce", "ring"), ("allreduce", "tree"), ("reducescatter", "ring"),
                       ("allgather", "ring"), ("broadcast", "ring"), ("reduce", "ring")):
        xs = _inputs(R, "int32", H.send_len(coll, n, R), extra=77)
        H.tune(vccl, comms, algo, proto, nchannels=1, chunk=256, direct=1)
        try:
            got = _run(vccl, comms, coll, xs, n, "int32", root=2)
            assert vccl.vcclCommGetLastPlan(comms[0])["scope"] == 1
        finally:
            H.untune(vccl, comms)
        want = sim.run(coll, xs, dtype="int32", nchannels=1, chunk_bytes=256, algo=algo, root=2)
        for r in range(R):
            if coll == "reduce" and r != 2:
                continue
            _assert_bits(got[r], want[r], f"xcd scope {coll} {algo} {proto} rank {r}")
