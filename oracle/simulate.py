"""Step-by-step simulation of the ring and tree schedules.

Every rank runs, per loop iteration, exactly the primitive sequence of the
paper's step tables (Section V-E):

* Ring AllReduce (Table "Steps in one loop iteration of NCCL Ring
  AllReduce"): step 0 send; steps 1..k-2 recvReduceSend; step k-1
  recvReduceCopySend; steps k..2k-3 recvCopySend; step 2k-2 recv.
* Ring AllGather: step 0 copySend (send when in place); steps 1..k-2
  recvCopySend; step k-1 recv.
* Ring ReduceScatter: step 0 send; steps 1..k-2 recvReduceSend; step k-1
  recvReduceCopy; data moves from rank i to rank (i+1)%k.
* Tree AllReduce: root recvReduceCopySend; middle recvReduceSend then
  recvCopySend; leaf send then recv.
* Ring Broadcast: a chain from the root along the ring: root copySend (send
  in place), middle recvCopySend, last recv.
* Ring Reduce: a chain that ends at the root: initiator send, middle
  recvReduceSend, root recvReduceCopy.

Readings adopted where the paper is silent (the library follows the same):

* Ring segment index: at step ``t`` rank ``p`` works on segment
  ``(p - 1 - t) mod R`` (AllReduce, ReduceScatter) or block ``(p - t) mod R``
  (AllGather); so rank ``p`` ends the reduction phase owning segment ``p``.
* Broadcast chain: root, root+1, ..., root-1.  Reduce chain: root+1, ...,
  root-1, root (the "first GPU" is the root's successor).
* A channel may follow another ring order (``rings``, Section II-C; see
  ``topology.channel_ring``).  Every rule above then reads positions on the
  channel's ring for rank numbers: the rank at position ``q`` sends to the
  one at ``q + 1`` and works on segment ``(q - 1 - t) mod R``, the
  ReduceScatter and AllGather blocks are those of the ranks at positions
  ``(q - 1 - t)`` and ``(q - t)``, and the chains run along the ring from
  the root (Broadcast) or from the root's successor to the root (Reduce).
* A reduction step computes ``op(received, local)``; a tree node with two
  children computes ``op(op(local, first child), second child)``.
* Channel ``c`` of a tree AllReduce uses tree ``c mod 2`` of the double
  binary tree.
* Tree iterations may overlap: with ``lag = D`` a rank issues the upward
  step of chunk ``j`` before the downward step of chunk ``j - D``
  (``D = 0`` is the paper's order within one loop iteration).  Results do
  not depend on ``D``; the simulator checks that ``D <= slots - 1`` cannot
  deadlock.

Each connection (sender, receiver, kind) is an explicit FIFO with ``slots``
entries.  A primitive fires when every FIFO it receives from holds a message
and every FIFO it sends to has a free slot; a message carries a tag naming
the data it holds, and the receiver asserts that it is the one it expects.
If no rank can fire while work remains, the simulator raises ``Deadlock``.
"""
from __future__ import annotations

from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import elementwise as ew
from . import partition as pt
from . import topology as topo

DEFAULT_SLOTS = 8


class Deadlock(RuntimeError):
    pass


@dataclass
class Op:
    prim: str                      # primitive name as in the paper
    recv_from: list                # connection keys to receive from (in order)
    send_to: list                  # connection keys to send to
    src: tuple | None = None       # (array, start, end) local input
    dst: tuple | None = None       # (array, start, end) output
    reduce: bool = False
    tag: tuple = ()                # tag expected on receive / attached on send
    info: dict = field(default_factory=dict)


def _run(programs: dict, slots: int, op_name: str, dtype: str, trace: list | None):
    """Execute per-rank programs against bounded FIFOs until done or stuck."""
    fifos: dict = {}
    pcs = {r: 0 for r in programs}

    def fifo(key):
        q = fifos.get(key)
        if q is None:
            q = fifos[key] = deque()
        return q

    remaining = sum(len(p) for p in programs.values())
    while remaining:
        progressed = False
        for r, prog in programs.items():
            while pcs[r] < len(prog):
                op = prog[pcs[r]]
                if any(len(fifo(k)) == 0 for k in op.recv_from):
                    break
                if any(len(fifo(k)) >= slots for k in op.send_to):
                    break
                received = []
                for k in op.recv_from:
                    tag, data = fifo(k).popleft()
                    if tag != op.tag:
                        raise AssertionError(f"rank {r} {op.prim}: got {tag}, expected {op.tag}")
                    received.append(data)
                if op.src is not None:
                    arr, s, e = op.src
                    local = arr[s:e].copy()
                else:
                    local = None
                if op.reduce:
                    if len(received) == 1:
                        value = ew.combine(op_name, dtype, received[0], local)
                    else:
                        value = local
                        for v in received:
                            value = ew.combine(op_name, dtype, value, v)
                elif received:
                    value = received[0]
                else:
                    value = local
                if op.dst is not None:
                    arr, s, e = op.dst
                    arr[s:e] = value
                for k in op.send_to:
                    fifo(k).append((op.tag, value.copy()))
                if trace is not None:
                    ent = dict(rank=r, prim=op.prim, tag=op.tag, sent_bytes=int(value.nbytes) * len(op.send_to))
                    ent.update(op.info)
                    trace.append(ent)
                pcs[r] += 1
                remaining -= 1
                progressed = True
        if not progressed and remaining:
            stuck = {r: programs[r][pcs[r]].prim for r in programs if pcs[r] < len(programs[r])}
            raise Deadlock(f"no rank can progress; pending primitives: {stuck}")
    leftovers = {k: len(q) for k, q in fifos.items() if len(q)}
    if leftovers:
        raise AssertionError(f"messages left in FIFOs: {leftovers}")


def _ring_ar_prim(t: int, nranks: int) -> str:
    if t == 0:
        return "send"
    if t <= nranks - 2:
        return "recvReduceSend"
    if t == nranks - 1:
        return "recvReduceCopySend"
    if t <= 2 * nranks - 3:
        return "recvCopySend"
    return "recv"


def ring_allreduce(xs, op, dtype, nchannels, chunk, slots=DEFAULT_SLOTS, trace=None, rings=None):
    """Ring AllReduce of equal-length per-rank arrays; returns per-rank outputs."""
    R = len(xs)
    n = len(xs[0])
    E = ew.ELEM_BYTES[dtype]
    A = pt.align_units("allreduce", E)
    outs = [np.zeros_like(x) for x in xs]
    for c, (cs, ce) in enumerate(pt.channel_ranges(n, nchannels, A)):
        loops = pt.ring_allreduce_loops(ce - cs, R, chunk, A) if ce > cs else []
        order = topo.channel_ring(R, c, rings)
        programs = {}
        for p in range(R):
            prog = []
            q = order.index(p)
            nxt, prv = order[(q + 1) % R], order[(q - 1) % R]
            for l, segs in enumerate(loops):
                for t in range(2 * R - 1):
                    s = (q - 1 - t) % R
                    a, b = cs + segs[s][0], cs + segs[s][1]
                    prim = _ring_ar_prim(t, R)
                    recv = [("ring", prv, p)] if prim != "send" else []
                    send = [("ring", p, nxt)] if prim != "recv" else []
                    src = (xs[p], a, b) if t <= R - 1 else None
                    dst = (outs[p], a, b) if t >= R - 1 else None
                    reduce = 1 <= t <= R - 1
                    prog.append(Op(prim, recv, send, src, dst, reduce, (l, s),
                                   dict(channel=c, loop=l, step=t, start=a, end=b)))
            programs[p] = prog
        _run(programs, slots, op, dtype, trace)
    return outs


def ring_reducescatter(xs, op, dtype, nchannels, chunk, slots=DEFAULT_SLOTS, trace=None, rings=None):
    """xs[p] holds R blocks of n elements; rank p receives the reduced block p."""
    R = len(xs)
    n = len(xs[0]) // R
    E = ew.ELEM_BYTES[dtype]
    A = pt.align_units("reducescatter", E)
    outs = [np.zeros(n, dtype=xs[0].dtype) for _ in xs]
    for c, (cs, ce) in enumerate(pt.channel_ranges(n, nchannels, A)):
        chunks = pt.chunk_ranges(ce - cs, chunk) if ce > cs else []
        order = topo.channel_ring(R, c, rings)
        programs = {}
        for p in range(R):
            prog = []
            q = order.index(p)
            nxt, prv = order[(q + 1) % R], order[(q - 1) % R]
            for l, (a0, b0) in enumerate(chunks):
                a, b = cs + a0, cs + b0
                for t in range(R):
                    j = order[(q - 1 - t) % R]
                    if t == 0:
                        prim = "send"
                    elif t <= R - 2:
                        prim = "recvReduceSend"
                    else:
                        prim = "recvReduceCopy"
                    recv = [("ring", prv, p)] if t > 0 else []
                    send = [("ring", p, nxt)] if t < R - 1 else []
                    dst = (outs[p], a, b) if t == R - 1 else None
                    prog.append(Op(prim, recv, send, (xs[p], j * n + a, j * n + b), dst, t > 0, (l, j),
                                   dict(channel=c, loop=l, step=t, start=a, end=b, block=j)))
            programs[p] = prog
        _run(programs, slots, op, dtype, trace)
    return outs


def _as_bytes(x):
    return np.ascontiguousarray(x).view(np.uint8)


def ring_allgather(xs, dtype, nchannels, chunk_bytes, slots=DEFAULT_SLOTS, trace=None, rings=None):
    """xs[p] holds n elements; every rank receives the R blocks in rank order."""
    R = len(xs)
    xb = [_as_bytes(x) for x in xs]
    nb = len(xb[0])
    outs_b = [np.zeros(R * nb, dtype=np.uint8) for _ in xs]
    A = pt.align_units("allgather", ew.ELEM_BYTES[dtype])
    for c, (cs, ce) in enumerate(pt.channel_ranges(nb, nchannels, A)):
        chunks = pt.chunk_ranges(ce - cs, chunk_bytes) if ce > cs else []
        order = topo.channel_ring(R, c, rings)
        programs = {}
        for p in range(R):
            prog = []
            q = order.index(p)
            nxt, prv = order[(q + 1) % R], order[(q - 1) % R]
            for l, (a0, b0) in enumerate(chunks):
                a, b = cs + a0, cs + b0
                for t in range(R):
                    j = order[(q - t) % R]
                    if t == 0:
                        prim, recv, send, src = "copySend", [], [("ring", p, nxt)], (xb[p], a, b)
                    elif t <= R - 2:
                        prim, recv, send, src = "recvCopySend", [("ring", prv, p)], [("ring", p, nxt)], None
                    else:
                        prim, recv, send, src = "recv", [("ring", prv, p)], [], None
                    prog.append(Op(prim, recv, send, src, (outs_b[p], j * nb + a, j * nb + b), False, (l, j),
                                   dict(channel=c, loop=l, step=t, start=a, end=b, block=j)))
            programs[p] = prog
        _run(programs, slots, "sum", "int32", trace)
    return [o.view(xs[0].dtype) for o in outs_b]


def ring_broadcast(xs, root, dtype, nchannels, chunk_bytes, slots=DEFAULT_SLOTS, trace=None, rings=None):
    """Chain from the root along the ring; every rank receives xs[root]."""
    R = len(xs)
    xb = [_as_bytes(x) for x in xs]
    nb = len(xb[0])
    outs_b = [np.zeros(nb, dtype=np.uint8) for _ in xs]
    A = pt.align_units("broadcast", ew.ELEM_BYTES[dtype])
    for c, (cs, ce) in enumerate(pt.channel_ranges(nb, nchannels, A)):
        chunks = pt.chunk_ranges(ce - cs, chunk_bytes) if ce > cs else []
        order = topo.channel_ring(R, c, rings)
        programs = {}
        for p in range(R):
            q = order.index(p)
            pos = (q - order.index(root)) % R
            nxt, prv = order[(q + 1) % R], order[(q - 1) % R]
            prog = []
            for l, (a0, b0) in enumerate(chunks):
                a, b = cs + a0, cs + b0
                if pos == 0:
                    o = Op("copySend", [], [("ring", p, nxt)], (xb[p], a, b), (outs_b[p], a, b))
                elif pos < R - 1:
                    o = Op("recvCopySend", [("ring", prv, p)], [("ring", p, nxt)], None, (outs_b[p], a, b))
                else:
                    o = Op("recv", [("ring", prv, p)], [], None, (outs_b[p], a, b))
                o.tag = (l,)
                o.info = dict(channel=c, loop=l, pos=pos, start=a, end=b)
                prog.append(o)
            programs[p] = prog
        _run(programs, slots, "sum", "int32", trace)
    return [o.view(xs[0].dtype) for o in outs_b]


def ring_reduce(xs, root, op, dtype, nchannels, chunk, slots=DEFAULT_SLOTS, trace=None, rings=None):
    """Chain along the ring from the root's successor to the root; returns
    the root's output (others None)."""
    R = len(xs)
    n = len(xs[0])
    A = pt.align_units("reduce", ew.ELEM_BYTES[dtype])
    out = np.zeros_like(xs[root])
    for c, (cs, ce) in enumerate(pt.channel_ranges(n, nchannels, A)):
        chunks = pt.chunk_ranges(ce - cs, chunk) if ce > cs else []
        order = topo.channel_ring(R, c, rings)
        programs = {}
        for p in range(R):
            q = order.index(p)
            pos = (q - order.index(root) - 1) % R
            nxt, prv = order[(q + 1) % R], order[(q - 1) % R]
            prog = []
            for l, (a0, b0) in enumerate(chunks):
                a, b = cs + a0, cs + b0
                if pos == 0:
                    o = Op("send", [], [("ring", p, nxt)], (xs[p], a, b), None, False)
                elif pos < R - 1:
                    o = Op("recvReduceSend", [("ring", prv, p)], [("ring", p, nxt)], (xs[p], a, b), None, True)
                else:
                    o = Op("recvReduceCopy", [("ring", prv, p)], [], (xs[p], a, b), (out, a, b), True)
                o.tag = (l,)
                o.info = dict(channel=c, loop=l, pos=pos, start=a, end=b)
                prog.append(o)
            programs[p] = prog
        _run(programs, slots, op, dtype, trace)
    return [out if p == root else None for p in range(R)]


def tree_allreduce(xs, op, dtype, nchannels, chunk, slots=DEFAULT_SLOTS, lag=0, trace=None, ranks_per_node=1):
    """Double-binary-tree AllReduce; channel c uses tree c mod 2."""
    R = len(xs)
    n = len(xs[0])
    A = pt.align_units("allreduce", ew.ELEM_BYTES[dtype])
    trees = topo.double_binary_tree(R, ranks_per_node)
    outs = [np.zeros_like(x) for x in xs]
    if lag < 0:
        raise ValueError("lag must be >= 0")
    for c, (cs, ce) in enumerate(pt.channel_ranges(n, nchannels, A)):
        tr = trees[c % 2]
        tid = c % 2
        chunks = pt.chunk_ranges(ce - cs, chunk) if ce > cs else []
        nch = len(chunks)
        programs = {}
        for p in range(R):
            par, kids = tr["parent"][p], tr["children"][p]
            up_in = [("up", tid, k, p) for k in kids]
            down_out = [("down", tid, p, k) for k in kids]
            prog = []
            for j in range(nch + lag):
                if j < nch:
                    a, b = cs + chunks[j][0], cs + chunks[j][1]
                    info = dict(channel=c, loop=j, phase="up", start=a, end=b)
                    if par < 0:
                        prog.append(Op("recvReduceCopySend", up_in, down_out, (xs[p], a, b), (outs[p], a, b),
                                       True, (j,), info))
                    elif kids:
                        prog.append(Op("recvReduceSend", up_in, [("up", tid, p, par)], (xs[p], a, b), None,
                                       True, (j,), info))
                    else:
                        prog.append(Op("send", [], [("up", tid, p, par)], (xs[p], a, b), None, False, (j,), info))
                jd = j - lag
                if jd >= 0 and par >= 0:
                    a, b = cs + chunks[jd][0], cs + chunks[jd][1]
                    info = dict(channel=c, loop=jd, phase="down", start=a, end=b)
                    if kids:
                        prog.append(Op("recvCopySend", [("down", tid, par, p)], down_out, None, (outs[p], a, b),
                                       False, (jd,), info))
                    else:
                        prog.append(Op("recv", [("down", tid, par, p)], [], None, (outs[p], a, b),
                                       False, (jd,), info))
            programs[p] = prog
        _run(programs, slots, op, dtype, trace)
    return outs


def run(coll, xs, *, op="sum", dtype, nchannels=1, chunk_bytes, root=0, algo="ring",
        slots=DEFAULT_SLOTS, lag=0, trace=None, ranks_per_node=1, rings=None):
    """Dispatch by collective name; chunk_bytes is converted to partition units."""
    E = ew.ELEM_BYTES[dtype]
    ub = pt.unit_bytes(coll, E)
    if chunk_bytes % 16:
        raise ValueError("chunk_bytes must be a multiple of 16")
    K = chunk_bytes // ub
    if coll == "allreduce":
        if algo == "tree":
            return tree_allreduce(xs, op, dtype, nchannels, K, slots, lag, trace, ranks_per_node)
        return ring_allreduce(xs, op, dtype, nchannels, K, slots, trace, rings)
    if coll == "reducescatter":
        return ring_reducescatter(xs, op, dtype, nchannels, K, slots, trace, rings)
    if coll == "allgather":
        return ring_allgather(xs, dtype, nchannels, K, slots, trace, rings)
    if coll == "broadcast":
        return ring_broadcast(xs, root, dtype, nchannels, K, slots, trace, rings)
    if coll == "reduce":
        return ring_reduce(xs, root, op, dtype, nchannels, K, slots, trace, rings)
    raise ValueError(coll)
