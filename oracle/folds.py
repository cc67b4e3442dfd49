"""Closed-form association orders of the schedules' float reductions.

Derived from the step tables without running them, so they pin the
simulator (a wrong segment index, a dropped step or a swapped operand in the
simulator changes the order and the bits):

* Ring AllReduce: the data of segment ``s`` leaves rank ``s+1`` at step 0
  and gains one rank per step, so it is folded left to right over ranks
  ``s+1, s+2, ..., s+R`` (mod R); rank ``s`` adds the last term at step
  ``R-1``.  Every rank then receives those same bits.
* Ring ReduceScatter: block ``b`` is folded over ranks ``b+1, ..., b+R``,
  independent of channels and chunking.
* Ring Reduce: folded over ``root+1, root+2, ..., root``.
* Tree AllReduce: post-order on the channel's tree:
  ``f(v) = op(op(x_v, f(first child)), f(second child))``.
* With per-channel ring orders (``rings``; Section II-C) the ring folds run
  over ring positions: segment ``s`` of a channel is folded over the ranks
  at positions ``s+1, ..., s+R`` of that channel's ring, block ``b`` over
  the ranks that follow rank ``b`` on the ring, and a Reduce over the ranks
  that follow the root, ending at the root.

The segment of an element is computed arithmetically from the partition
reading (``partition`` module) rather than by walking loop lists.
"""
from __future__ import annotations

import numpy as np

from . import elementwise as ew
from . import partition as pt
from . import topology as topo


def _fold(terms, op, dtype):
    acc = terms[0]
    for t in terms[1:]:
        acc = ew.combine(op, dtype, acc, t)
    return acc


def ring_allreduce_segment_of(idx, n, nranks, nchannels, chunk, align):
    """Segment id (0..R-1) of each element index in ``idx``."""
    idx = np.asarray(idx, dtype=np.int64)
    per = pt.round_up(pt.ceil_div(n, nchannels), align) if n > 0 else 1
    c = idx // per
    cs = c * per
    ce = np.minimum(n, cs + per)
    rel = idx - cs
    n_c = ce - cs
    loop_count = nranks * chunk
    full = n_c // loop_count
    in_full = rel < full * loop_count
    seg_full = (rel % loop_count) // chunk
    rem = n_c - full * loop_count
    k2 = np.where(rem > 0, ((rem + nranks - 1) // nranks + align - 1) // align * align, 1)
    seg_last = (rel - full * loop_count) // k2
    return np.where(in_full, seg_full, seg_last)


def _channel_of(idx, n, nchannels, align):
    per = pt.round_up(pt.ceil_div(n, nchannels), align) if n > 0 else 1
    return np.asarray(idx, dtype=np.int64) // per


def _ring_orders(R, idx, n, nchannels, align, rings):
    """(channel ring order, mask of idx on channels with that order) pairs."""
    if rings is None:
        return [(list(range(R)), np.ones(len(idx), dtype=bool))]
    chan = _channel_of(idx, n, nchannels, align)
    return [(topo.channel_ring(R, k, rings), (chan % len(rings)) == k) for k in range(len(rings))]


def ring_allreduce(xs, op, dtype, nchannels, chunk, idx=None, rings=None):
    """Expected AllReduce output (identical on all ranks) at ``idx`` (default all)."""
    R = len(xs)
    n = len(xs[0])
    A = pt.align_units("allreduce", ew.ELEM_BYTES[dtype])
    if idx is None:
        idx = np.arange(n)
    idx = np.asarray(idx, dtype=np.int64)
    seg = ring_allreduce_segment_of(idx, n, R, nchannels, chunk, A)
    out = np.empty(len(idx), dtype=np.asarray(xs[0]).dtype)
    for ring, on in _ring_orders(R, idx, n, nchannels, A, rings):
        for s in range(R):
            m = on & (seg == s)
            if not m.any():
                continue
            order = [ring[(s + 1 + j) % R] for j in range(R)]
            out[m] = _fold([np.asarray(xs[q])[idx[m]] for q in order], op, dtype)
    return out


def ring_reducescatter(xs, op, dtype, rank, idx=None, nchannels=1, rings=None):
    """Expected ReduceScatter output of ``rank`` at ``idx`` (default all).
    ``nchannels`` matters only with ``rings``."""
    R = len(xs)
    n = len(xs[0]) // R
    A = pt.align_units("reducescatter", ew.ELEM_BYTES[dtype])
    if idx is None:
        idx = np.arange(n)
    idx = np.asarray(idx, dtype=np.int64)
    out = np.empty(len(idx), dtype=np.asarray(xs[0]).dtype)
    for ring, m in _ring_orders(R, idx, n, nchannels, A, rings):
        if not m.any():
            continue
        q0 = ring.index(rank)
        order = [ring[(q0 + 1 + j) % R] for j in range(R)]
        out[m] = _fold([np.asarray(xs[q])[rank * n + idx[m]] for q in order], op, dtype)
    return out


def ring_reduce(xs, op, dtype, root, idx=None, nchannels=1, rings=None):
    """Expected Reduce output at the root, at ``idx`` (default all).
    ``nchannels`` matters only with ``rings``."""
    R = len(xs)
    n = len(xs[0])
    A = pt.align_units("reduce", ew.ELEM_BYTES[dtype])
    if idx is None:
        idx = np.arange(n)
    idx = np.asarray(idx, dtype=np.int64)
    out = np.empty(len(idx), dtype=np.asarray(xs[0]).dtype)
    for ring, m in _ring_orders(R, idx, n, nchannels, A, rings):
        if not m.any():
            continue
        q0 = ring.index(root)
        order = [ring[(q0 + 1 + j) % R] for j in range(R)]
        out[m] = _fold([np.asarray(xs[q])[idx[m]] for q in order], op, dtype)
    return out


def tree_allreduce(xs, op, dtype, nchannels, idx=None, ranks_per_node=1):
    R = len(xs)
    n = len(xs[0])
    A = pt.align_units("allreduce", ew.ELEM_BYTES[dtype])
    trees = topo.double_binary_tree(R, ranks_per_node)
    if idx is None:
        idx = np.arange(n)
    idx = np.asarray(idx, dtype=np.int64)
    per = pt.round_up(pt.ceil_div(n, nchannels), A) if n > 0 else 1
    chan = idx // per
    out = np.empty(len(idx), dtype=np.asarray(xs[0]).dtype)

    def f(tree, v, sel):
        acc = np.asarray(xs[v])[sel]
        for k in tree["children"][v]:
            acc = ew.combine(op, dtype, acc, f(tree, k, sel))
        return acc

    for t in (0, 1):
        m = (chan % 2) == t
        if not m.any():
            continue
        tree = trees[t]
        out[m] = f(tree, tree["root"], idx[m])
    return out
