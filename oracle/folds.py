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


def ring_allreduce(xs, op, dtype, nchannels, chunk, idx=None):
    """Expected AllReduce output (identical on all ranks) at ``idx`` (default all)."""
    R = len(xs)
    n = len(xs[0])
    A = pt.align_units("allreduce", ew.ELEM_BYTES[dtype])
    if idx is None:
        idx = np.arange(n)
    idx = np.asarray(idx, dtype=np.int64)
    seg = ring_allreduce_segment_of(idx, n, R, nchannels, chunk, A)
    out = np.empty(len(idx), dtype=np.asarray(xs[0]).dtype)
    for s in range(R):
        m = seg == s
        if not m.any():
            continue
        order = [(s + 1 + j) % R for j in range(R)]
        out[m] = _fold([np.asarray(xs[q])[idx[m]] for q in order], op, dtype)
    return out


def ring_reducescatter(xs, op, dtype, rank, idx=None):
    """Expected ReduceScatter output of ``rank`` at ``idx`` (default all)."""
    R = len(xs)
    n = len(xs[0]) // R
    if idx is None:
        idx = np.arange(n)
    idx = np.asarray(idx, dtype=np.int64)
    order = [(rank + 1 + j) % R for j in range(R)]
    return _fold([np.asarray(xs[q])[rank * n + idx] for q in order], op, dtype)


def ring_reduce(xs, op, dtype, root, idx=None):
    R = len(xs)
    n = len(xs[0])
    if idx is None:
        idx = np.arange(n)
    idx = np.asarray(idx, dtype=np.int64)
    order = [(root + 1 + j) % R for j in range(R)]
    return _fold([np.asarray(xs[q])[idx] for q in order], op, dtype)


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
