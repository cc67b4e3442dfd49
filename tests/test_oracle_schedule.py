"""Pins of the oracle's partition, topology and schedule simulation.

Each test checks the oracle against something other than itself: the
paper's step tables and Fig. 3 numbers (tests/golden/), brute-force
definitions (exact for int32 sum and max), closed-form fold orders derived
without the simulator, exact rational sums within the recursive-summation
error bound, and the double-binary-tree properties the paper states.
"""
import itertools
import os
import random

import numpy as np
import pytest

import synthetic_inputs as si
from oracle import definitions as defs
from oracle import elementwise as ew
from oracle import folds
from oracle import partition as pt
from oracle import simulate as sim
from oracle import topology as topo

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- partition

def _read_kv(name):
    out = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#")[0].strip()
        if line:
            k, v = line.split()
            out[k] = v
    return out


def test_fig3_partition_example():
    g = _read_kv("fig3_partition.txt")
    C, K, L = int(g["nchannels"]), int(g["chunkCount"]), int(g["loopCount"])
    R = L // K
    n = 16
    ch = pt.channel_ranges(n, C, 1)
    assert ch == [(0, 8), (8, 16)]
    for cs, ce in ch:
        loops = pt.ring_allreduce_loops(ce - cs, R, K, 1)
        assert len(loops) == 2
        for lp in loops:
            assert lp[-1][1] - lp[0][0] == L
            assert all(e - s == K for s, e in lp)


@pytest.mark.parametrize("n,C,align", [(0, 4, 4), (1, 1, 4), (100, 16, 4), (65536, 1, 4),
                                       (12345, 7, 8), (3, 16, 16), (1 << 20, 13, 4)])
def test_channel_ranges_cover_disjoint_aligned(n, C, align):
    ch = pt.channel_ranges(n, C, align)
    assert len(ch) == C
    pos = 0
    for s, e in ch:
        assert s == pos or (s == e == n)
        assert s % align == 0 or s == n
        pos = e
    assert pos == n


@pytest.mark.parametrize("n_c,R,K,A", [(0, 4, 8, 4), (5, 4, 8, 4), (64, 4, 4, 4), (65, 4, 4, 4),
                                        (1000, 8, 16, 4), (17, 16, 16, 8), (8192 * 3 + 7, 8, 2048, 4)])
def test_ring_allreduce_loops_cover(n_c, R, K, A):
    loops = pt.ring_allreduce_loops(n_c, R, K, A)
    pos = 0
    for lp in loops:
        assert len(lp) == R
        for s, e in lp:
            assert s == pos and e >= s
            pos = e
    assert pos == n_c
    if n_c % (R * K):
        base = lp[0][0]
        rem = n_c - base
        for s, e in lp:
            assert (s - base) % A == 0 or s == n_c
        assert lp[0][1] - lp[0][0] <= max(A, -(-rem // R) + A)


# ---------------------------------------------------------------- topology

@pytest.mark.parametrize("R", list(range(2, 33)))
def test_double_binary_tree_properties(R):
    A, B = topo.double_binary_tree(R)
    for t in (A, B):
        roots = [r for r in range(R) if t["parent"][r] < 0]
        assert roots == [t["root"]]
        assert len(t["children"][t["root"]]) == 1
        for r in range(R):
            assert len(t["children"][r]) <= 2
            for c in t["children"][r]:
                assert t["parent"][c] == r
            x, hops = r, 0
            while t["parent"][x] >= 0:
                x = t["parent"][x]
                hops += 1
                assert hops <= R
        depth = topo.tree_depth(t)
        assert depth <= int(np.ceil(np.log2(R))) + 1
    inner_a = {r for r in range(R) if A["children"][r]}
    inner_b = {r for r in range(R) if B["children"][r]}
    leaf_both = [r for r in range(R) if r not in inner_a and r not in inner_b]
    if R % 2 == 0:
        # the paper's properties: no rank is an inner node of both trees,
        # at most one rank is a leaf in both (here: none)
        assert not (inner_a & inner_b)
        assert len(leaf_both) <= 1
        assert [B["parent"][R - 1 - q] for q in range(R)] == \
            [(-1 if A["parent"][q] < 0 else R - 1 - A["parent"][q]) for q in range(R)]
    else:
        assert len(leaf_both) <= 1
        shifted = [(q + 1) % R for q in range(R)]
        assert [B["parent"][shifted[q]] for q in range(R)] == \
            [(-1 if A["parent"][q] < 0 else shifted[A["parent"][q]]) for q in range(R)]


def test_tree_depth_for_16_ranks_is_four():
    A, _ = topo.double_binary_tree(16)
    assert topo.tree_depth(A) == 4
    x, chain = 1, [1]
    while A["parent"][x] >= 0:
        x = A["parent"][x]
        chain.append(x)
    assert chain == [1, 2, 4, 8, 0]


# ---------------------------------------------------------------- step tables

def _golden_tables():
    tab = {}
    for line in open(os.path.join(GOLDEN, "step_tables.txt")):
        line = line.split("#")[0].strip()
        if not line:
            continue
        alg, rng, prims = line.split()
        tab.setdefault(alg, []).append((rng, prims.split(",")))
    return tab


def _bound(expr, k):
    # the tables write bounds as 0, k-2, 2k-3, ...: an optional factor of k plus a constant
    expr = expr.replace(" ", "")
    if "k" not in expr:
        return int(expr)
    coef, rest = expr.split("k")
    return (int(coef) if coef else 1) * k + (int(rest) if rest else 0)


def _expand(rng, k):
    if ".." in rng:
        a, b = rng.split("..")
        return list(range(_bound(a, k), _bound(b, k) + 1))
    return [_bound(rng, k)]


@pytest.mark.parametrize("k", list(range(2, 17)))
def test_ring_traces_follow_paper_tables(k):
    tab = _golden_tables()
    xs = si.rank_inputs(9, k, "int32", 40 * k)
    for alg, coll, xsx in (("ring_allreduce", "allreduce", xs),
                           ("ring_allgather", "allgather", xs),
                           ("ring_reducescatter", "reducescatter", xs)):
        expect = {}
        for rng, prims in tab[alg]:
            for t in _expand(rng, k):
                expect[t] = prims[0]
        nsteps = 2 * k - 1 if alg == "ring_allreduce" else k
        assert sorted(expect) == list(range(nsteps))
        trace = []
        sim.run(coll, xsx, dtype="int32", nchannels=2, chunk_bytes=32, trace=trace)
        assert trace
        per_rank_loop = {}
        for ent in trace:
            assert ent["prim"] == expect[ent["step"]], (alg, ent)
            per_rank_loop.setdefault((ent["rank"], ent["channel"], ent["loop"]), []).append(ent["step"])
        for steps in per_rank_loop.values():
            assert steps == list(range(nsteps))


@pytest.mark.parametrize("R", [2, 3, 5, 8, 16])
def test_chain_and_tree_roles_follow_paper_tables(R):
    tab = {alg: dict(rows) for alg, rows in _golden_tables().items()}
    xs = si.rank_inputs(9, R, "int32", 50 * R)
    for root in sorted({0, R // 2, R - 1}):
        tr = []
        sim.run("broadcast", xs, dtype="int32", chunk_bytes=64, root=root, trace=tr)
        for e in tr:
            role = "root" if e["rank"] == root else ("last" if e["rank"] == (root - 1) % R else "middle")
            assert [e["prim"]] == tab["ring_broadcast"][role]
        tr = []
        sim.run("reduce", xs, dtype="int32", chunk_bytes=64, root=root, trace=tr)
        for e in tr:
            role = "root" if e["rank"] == root else ("initiator" if e["rank"] == (root + 1) % R else "middle")
            assert [e["prim"]] == tab["ring_reduce"][role]
    trees = topo.double_binary_tree(R)
    tr = []
    sim.run("allreduce", xs, dtype="int32", nchannels=2, chunk_bytes=64, algo="tree", trace=tr)
    seq = {}
    for e in tr:
        seq.setdefault((e["channel"], e["rank"], e["loop"]), []).append(e["prim"])
    for (c, r, _), prims in seq.items():
        t = trees[c % 2]
        role = "root" if t["parent"][r] < 0 else ("middle" if t["children"][r] else "leaf")
        assert prims == tab["tree_allreduce"][role]


@pytest.mark.parametrize("R", [2, 3, 4, 8, 16])
def test_transfer_counts_per_loop(R):
    """AllReduce: 2R-1 calls and 2(R-1) sends and receives per rank per loop;
    ReduceScatter / AllGather: R calls and R-1 transfers."""
    xs = si.rank_inputs(9, R, "int32", 64 * R)
    for coll, calls in (("allreduce", 2 * R - 1), ("reducescatter", R), ("allgather", R)):
        tr = []
        sim.run(coll, xs, dtype="int32", nchannels=1, chunk_bytes=16, trace=tr)
        per = {}
        for e in tr:
            per.setdefault((e["rank"], e["loop"]), []).append(e["prim"])
        for prims in per.values():
            assert len(prims) == calls
            sends = sum(1 for p in prims if p.endswith("Send") or p == "send")
            recvs = sum(1 for p in prims if p.startswith("recv"))
            assert sends == calls - 1 and recvs == calls - 1


@pytest.mark.parametrize("R", [2, 4, 8, 16])
def test_link_bytes_give_the_bus_bandwidth_factors(R):
    """Bytes each rank puts on its outgoing link, over the message size S
    (nccl-tests convention: busBW = algBW x factor): ring AllReduce
    2(R-1)/R, ReduceScatter and AllGather (R-1)/R, Broadcast and Reduce 1
    for every rank but the last of the chain (which sends nothing)."""
    n = 64 * R  # elements per rank; divisible by R and the chunk
    xs = si.rank_inputs(9, R, "float32", n, extra=R)
    S = n * 4
    for coll, factor in (("allreduce", 2 * (R - 1) / R), ("reducescatter", (R - 1) / R),
                         ("allgather", (R - 1) / R), ("broadcast", 1.0), ("reduce", 1.0)):
        data = list(xs)
        if coll == "allgather":
            data = [x[: n // R] for x in xs]  # S = the gathered (larger) buffer
        tr = []
        sim.run(coll, data, dtype="float32", nchannels=2, chunk_bytes=32, root=1, trace=tr)
        sent = {}
        for e in tr:
            sent[e["rank"]] = sent.get(e["rank"], 0) + e["sent_bytes"]
        for r in range(R):
            if coll == "broadcast" and r == 0:    # root 1: the last of the chain is rank 0
                assert sent.get(r, 0) == 0
            elif coll == "reduce" and r == 1:     # the chain ends at the root
                assert sent.get(r, 0) == 0
            else:
                assert sent[r] == factor * S, (coll, R, r, sent[r], factor * S)


# ---------------------------------------------------------------- brute force

CASES = [(2, 1, 16), (3, 2, 32), (4, 1, 64), (5, 3, 48), (8, 4, 16), (16, 2, 128)]
SIZES = [0, 1, 3, 4, 17, 100, 1000, 4099]


@pytest.mark.parametrize("R,C,chunk", CASES)
@pytest.mark.parametrize("dtype,op", [("int32", "sum"), ("int32", "max"), ("float32", "max"), ("bfloat16", "max")])
def test_schedules_equal_definitions(R, C, chunk, dtype, op):
    rng = random.Random(R * 1000 + C)
    for n in SIZES:
        if dtype == "int32":
            xs = si.rank_inputs(3, R, "int32", n, lo=-2**20, hi=2**20, extra=n)
        else:
            xs = si.rank_inputs(3, R, dtype, n, dist="uniform", extra=n)
        want = defs.allreduce(xs, op, dtype)
        for algo in ("ring", "tree"):
            got = sim.run("allreduce", xs, op=op, dtype=dtype, nchannels=C, chunk_bytes=chunk, algo=algo)
            for g, w in zip(got, want):
                np.testing.assert_array_equal(g.view(np.uint8), w.view(np.uint8))
        big = np.concatenate
        xr = [big([x] * R) if n else x for x in xs]
        got = sim.run("reducescatter", xr, op=op, dtype=dtype, nchannels=C, chunk_bytes=chunk)
        for g, w in zip(got, defs.reducescatter(xr, op, dtype)):
            np.testing.assert_array_equal(g.view(np.uint8), w.view(np.uint8))
        root = rng.randrange(R)
        got = sim.run("reduce", xs, op=op, dtype=dtype, nchannels=C, chunk_bytes=chunk, root=root)
        np.testing.assert_array_equal(got[root].view(np.uint8), defs.reduce(xs, root, op, dtype)[root].view(np.uint8))
        got = sim.run("broadcast", xs, dtype=dtype, nchannels=C, chunk_bytes=chunk, root=root)
        for g, w in zip(got, defs.broadcast(xs, root)):
            np.testing.assert_array_equal(g.view(np.uint8), w.view(np.uint8))
        got = sim.run("allgather", xs, dtype=dtype, nchannels=C, chunk_bytes=chunk)
        for g, w in zip(got, defs.allgather(xs)):
            np.testing.assert_array_equal(g.view(np.uint8), w.view(np.uint8))


# ---------------------------------------------------------------- float folds

@pytest.mark.parametrize("dtype", ["float32", "bfloat16"])
@pytest.mark.parametrize("R,C,chunk", CASES)
def test_float_sums_follow_closed_form_folds(dtype, R, C, chunk):
    E = ew.ELEM_BYTES[dtype]
    for n in (1, 7, 100, 999, 3000):
        xs = si.rank_inputs(4, R, dtype, n, dist="normal" if dtype == "float32" else None, extra=n)
        ring = sim.run("allreduce", xs, dtype=dtype, nchannels=C, chunk_bytes=chunk)
        want = folds.ring_allreduce(xs, "sum", dtype, C, chunk // E)
        for g in ring:
            np.testing.assert_array_equal(g.view(np.uint8), want.view(np.uint8))
        tree = sim.run("allreduce", xs, dtype=dtype, nchannels=C, chunk_bytes=chunk, algo="tree", lag=7)
        want = folds.tree_allreduce(xs, "sum", dtype, C)
        for g in tree:
            np.testing.assert_array_equal(g.view(np.uint8), want.view(np.uint8))
        root = (n + R) % R
        red = sim.run("reduce", xs, dtype=dtype, nchannels=C, chunk_bytes=chunk, root=root)[root]
        np.testing.assert_array_equal(red.view(np.uint8), folds.ring_reduce(xs, "sum", dtype, root).view(np.uint8))
        xr = [np.concatenate([x] + [x[::-1]] * (R - 1)) for x in xs]
        rs = sim.run("reducescatter", xr, dtype=dtype, nchannels=C, chunk_bytes=chunk)
        for r in range(R):
            np.testing.assert_array_equal(rs[r].view(np.uint8),
                                          folds.ring_reducescatter(xr, "sum", dtype, r).view(np.uint8))


def test_two_ranks_reduce_to_plain_addition():
    rng = np.random.default_rng(5)
    a = rng.standard_normal(333).astype(np.float32)
    b = rng.standard_normal(333).astype(np.float32)
    for algo in ("ring", "tree"):
        out = sim.run("allreduce", [a, b], dtype="float32", nchannels=2, chunk_bytes=32, algo=algo)
        for o in out:
            np.testing.assert_array_equal(o, a + b)


@pytest.mark.parametrize("dtype", ["float32", "bfloat16"])
@pytest.mark.parametrize("R", [2, 3, 4, 5])
def test_tiny_float_sums_within_error_bound(dtype, R):
    n = 64
    xs = si.rank_inputs(6, R, dtype, n, dist="normal" if dtype == "float32" else None)
    bound = defs.sum_error_bound(xs, dtype)
    for algo in ("ring", "tree"):
        out = sim.run("allreduce", xs, dtype=dtype, nchannels=2, chunk_bytes=16, algo=algo)[0]
        got = ew.to_float64(dtype, out)
        for i in range(n):
            exact = defs.exact_sum([ew.to_float64(dtype, x[i:i + 1])[0] for x in xs])
            err = abs(float(exact - type(exact)(float(got[i]))))
            assert err <= bound[i] * (1 + 1e-12), (algo, i, err, bound[i])


@pytest.mark.parametrize("dtype", ["float32", "bfloat16"])
def test_integer_valued_floats_sum_exactly(dtype):
    R = 8
    bound = 2**24 // R if dtype == "float32" else 256 // R
    xs = [si.small_int_valued_float(dtype, 5000, si.rng_for(7, r), bound) for r in range(R)]
    exact = defs.fp64_sum(xs, dtype)
    for algo in ("ring", "tree"):
        out = sim.run("allreduce", xs, dtype=dtype, nchannels=3, chunk_bytes=256, algo=algo)
        for o in out:
            np.testing.assert_array_equal(ew.to_float64(dtype, o), exact)


# ---------------------------------------------------------------- deadlock

@pytest.mark.parametrize("R", [2, 4, 7, 8, 16])
@pytest.mark.parametrize("slots", [1, 2, 8])
def test_tree_lag_below_slots_never_deadlocks(R, slots):
    xs = si.rank_inputs(8, R, "int32", 64 * 40)
    for lag in range(slots):
        out = sim.run("allreduce", xs, dtype="int32", nchannels=2, chunk_bytes=16, algo="tree",
                      slots=slots, lag=lag)
        np.testing.assert_array_equal(out[0], defs.allreduce(xs, "sum", "int32")[0])


def test_simulator_detects_deadlock():
    # a tree whose ranks run far ahead of the slot budget must stall
    xs = si.rank_inputs(8, 8, "int32", 16 * 64)
    with pytest.raises(sim.Deadlock):
        sim.run("allreduce", xs, dtype="int32", nchannels=1, chunk_bytes=16, algo="tree", slots=1, lag=6)


def test_simulator_detects_dead_rank():
    xs = si.rank_inputs(8, 4, "int32", 64)
    programs = {}
    orig = sim._run

    def drop_rank(progs, *a, **k):
        progs = dict(progs)
        progs[2] = []
        return orig(progs, *a, **k)

    sim._run = drop_rank
    try:
        with pytest.raises((sim.Deadlock, AssertionError)):
            sim.run("allreduce", xs, dtype="int32", chunk_bytes=16)
    finally:
        sim._run = orig
    del programs


# ---------------------------------------------------------------- planted mistakes

def test_pins_catch_wrong_segment_index(monkeypatch):
    """A plausible slip (segment p - t instead of p - 1 - t) must fail a pin."""
    orig = sim.ring_allreduce

    def wrong(xs, op, dtype, nchannels, chunk, slots=8, trace=None, rings=None):
        R = len(xs)
        rot = [np.asarray(xs[(p + 1) % R]) for p in range(R)]
        return orig(rot, op, dtype, nchannels, chunk, slots, trace, rings)

    monkeypatch.setattr(sim, "ring_allreduce", wrong)
    xs = si.rank_inputs(4, 5, "float32", 500)
    got = sim.run("allreduce", xs, dtype="float32", nchannels=1, chunk_bytes=64)[0]
    want = folds.ring_allreduce(xs, "sum", "float32", 1, 16)
    assert not np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_pins_catch_swapped_tree_children(monkeypatch):
    orig = topo.double_binary_tree

    def swapped(R, ranks_per_node=1):
        trees = orig(R, ranks_per_node)
        for t in trees:
            t["children"] = [list(reversed(c)) for c in t["children"]]
        return trees

    xs = si.rank_inputs(4, 8, "float32", 3000)
    want = folds.tree_allreduce(xs, "sum", "float32", 2)
    monkeypatch.setattr(topo, "double_binary_tree", swapped)
    got = sim.run("allreduce", xs, dtype="float32", nchannels=2, chunk_bytes=64, algo="tree")[0]
    assert not np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_pins_catch_dropped_term(monkeypatch):
    orig = ew.combine
    calls = itertools.count()

    def drop_one(op, dtype, acc, local):
        return acc if next(calls) == 3 else orig(op, dtype, acc, local)

    xs = si.rank_inputs(3, 4, "int32", 256)
    want = defs.allreduce(xs, "sum", "int32")[0]
    monkeypatch.setattr(ew, "combine", drop_one)
    got = sim.run("allreduce", xs, dtype="int32", chunk_bytes=64)
    assert any(not np.array_equal(g, want) for g in got)
