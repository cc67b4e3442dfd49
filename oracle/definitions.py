"""Plain definitions of the five collectives (Section II-A lists them; their
meaning is the standard one) -- brute force, no schedule.

* AllReduce:     out_r[i] = (+)_q x_q[i]                for every rank r
* ReduceScatter: out_r[i] = (+)_q x_q[r*n + i]
* AllGather:     out_r[q*n + i] = x_q[i]
* Broadcast:     out_r = x_root
* Reduce:        out_root = (+)_q x_q
* Send/Recv:     recv_b = send_a (a copy); all-to-all through grouped
                 Send/Recv: out_b[a*n + i] = x_a[b*n + i]

For int32 sum (mod 2^32) and for max these are exact at every size, because
those operators are associative and commutative: they pin the schedules
completely.  For float sums the schedule fixes the rounding; ``fp64_sum``
gives the exact-as-possible reference and ``sum_error_bound`` the classical
bound for a recursive sum of m terms, gamma_{m-1} * sum|x| with
gamma_k = k*u / (1 - k*u) (Higham, Accuracy and Stability of Numerical
Algorithms, 2nd ed., Section 4.2).  For bf16 every hop rounds twice (fp32,
then bf16), so its unit roundoff is 2^-8 + 2^-24.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

from . import elementwise as ew


def _reduce_all(arrs, op, dtype):
    if dtype == "int32":
        wide = np.zeros(len(arrs[0]), dtype=np.int64)
        if op == "sum":
            for a in arrs:
                wide += a.astype(np.int64)
            return (wide & np.int64(0xFFFFFFFF)).astype(np.uint32).view(np.int32)
        return np.maximum.reduce([np.asarray(a, dtype=np.int32) for a in arrs])
    if op == "max":
        vals = [ew.to_float64(dtype, a) for a in arrs]
        best = vals[0].copy()
        best_src = np.zeros(len(best), dtype=np.int64)
        for q, v in enumerate(vals[1:], start=1):
            take = (v > best) | ((v == best) & np.signbit(best) & ~np.signbit(v))
            best = np.where(take, v, best)
            best_src = np.where(take, q, best_src)
        stacked = np.stack([np.asarray(a) for a in arrs])
        return stacked[best_src, np.arange(len(best))]
    raise ValueError("float sums have no schedule-free definition in the storage type; use fp64_sum")


def allreduce(xs, op, dtype):
    v = _reduce_all(xs, op, dtype)
    return [v.copy() for _ in xs]


def reducescatter(xs, op, dtype):
    R = len(xs)
    n = len(xs[0]) // R
    return [_reduce_all([x[r * n:(r + 1) * n] for x in xs], op, dtype) for r in range(R)]


def allgather(xs):
    full = np.concatenate([np.asarray(x) for x in xs])
    return [full.copy() for _ in xs]


def broadcast(xs, root):
    return [np.asarray(xs[root]).copy() for _ in xs]


def reduce(xs, root, op, dtype):
    v = _reduce_all(xs, op, dtype)
    return [v if r == root else None for r in range(len(xs))]


def sendrecv(x):
    """Point-to-point transfer (Section II-A, Send/Recv): the receiver's
    buffer ends up holding the sender's elements, bit for bit."""
    return np.array(x, copy=True)


def alltoall(xs):
    """Send/Recv between every ordered pair of ranks in one group (Section
    II-A, group calls): rank a sends block b of its buffer (n elements) to
    rank b, which stores it as block a.  out_b[a*n + i] = x_a[b*n + i]."""
    R = len(xs)
    n = len(xs[0]) // R
    return [np.concatenate([np.asarray(xs[a])[b * n:(b + 1) * n] for a in range(R)]) for b in range(R)]


def fp64_sum(arrs, dtype):
    """Element-wise sum of the exact input values, accumulated in fp64."""
    acc = np.zeros(len(arrs[0]), dtype=np.float64)
    for a in arrs:
        acc += ew.to_float64(dtype, a)
    return acc


def exact_sum(values):
    """Exact rational sum of a short list of floats (for tiny-input pins)."""
    total = Fraction(0)
    for v in values:
        total += Fraction(float(v))
    return total


def unit_roundoff(dtype):
    """Relative error of one reduction hop.  A bf16 hop rounds twice (the fp32
    sum to fp32, then that to bf16), so its factor is
    (1 + 2^-24)(1 + 2^-8) = 1 + 2^-8 + 2^-24 + 2^-32."""
    if dtype == "float32":
        return 2.0 ** -24
    if dtype == "bfloat16":
        return 2.0 ** -8 + 2.0 ** -24 + 2.0 ** -32
    raise ValueError(dtype)


def sum_error_bound(arrs, dtype):
    """gamma_{m-1} * sum_q |x_q| element-wise, m = number of terms."""
    m = len(arrs)
    u = unit_roundoff(dtype)
    k = m - 1
    gamma = k * u / (1.0 - k * u)
    absum = np.zeros(len(arrs[0]), dtype=np.float64)
    for a in arrs:
        absum += np.abs(ew.to_float64(dtype, a))
    return gamma * absum
