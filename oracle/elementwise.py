"""Element-wise reduction operators of the oracle.

The paper names the reduction ("an element-wise reduction with the
corresponding segment of its local data", Section V-E, Ring AllReduce) but
not its numerics.  Readings adopted here (each is part of the parity contract):

* int32 sum: two's-complement addition modulo 2^32.
* float32 sum: one IEEE-754 binary32 addition, round to nearest even, no
  fused operations, subnormals kept.  numpy's float32 ``+`` is exactly that.
* bfloat16 sum: every partial result travels between ranks as bf16, so each
  hop computes ``bf16_rne(f32(a) + f32(b))``: the fp32 sum rounded to nearest
  even in fp32, then rounded to nearest even in bf16.
* max (all types): ``a > b ? a : (b > a ? b : (signbit(a) ? b : a))``, i.e.
  ordinary max that prefers +0 over -0.  It is commutative and associative on
  NaN-free inputs, so its result does not depend on the schedule.

bf16 values are carried as ``numpy.uint16`` bit patterns.
"""
from __future__ import annotations

import numpy as np

ELEM_BYTES = {"int32": 4, "float32": 4, "bfloat16": 2}
OPS = ("sum", "max")


def bf16_to_f32(u16: np.ndarray) -> np.ndarray:
    """Exact widening: the bf16 pattern is the upper half of the fp32 pattern."""
    u16 = np.asarray(u16, dtype=np.uint16)
    return (u16.astype(np.uint32) << np.uint32(16)).view(np.float32)


def f32_to_bf16_rne(f: np.ndarray) -> np.ndarray:
    """Round fp32 to the nearest bf16, ties to even (NaN inputs unsupported).

    Written from the definition: keep the upper 16 bits, and round up when
    the discarded lower 16 bits exceed half an ulp, or equal half an ulp and
    the kept part is odd.  Overflow past the largest finite bf16 carries into
    the exponent and yields infinity, as round-to-nearest requires.
    """
    u = np.asarray(f, dtype=np.float32).view(np.uint32).astype(np.uint64)
    upper = u >> np.uint64(16)
    lower = u & np.uint64(0xFFFF)
    half = np.uint64(0x8000)
    round_up = (lower > half) | ((lower == half) & ((upper & np.uint64(1)) == np.uint64(1)))
    return (upper + round_up.astype(np.uint64)).astype(np.uint16)


def _float_max(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """max with +0 preferred over -0; a and b are float arrays of equal shape."""
    gt = a > b
    lt = b > a
    a_neg = np.signbit(a)
    pick_b = lt | (~gt & ~lt & a_neg)
    return np.where(pick_b, b, a)


def combine(op: str, dtype: str, acc: np.ndarray, local: np.ndarray) -> np.ndarray:
    """One reduction hop: ``acc (+) local`` element-wise, in the storage dtype."""
    if op not in OPS:
        raise ValueError(op)
    if dtype == "int32":
        a = np.asarray(acc, dtype=np.int32)
        b = np.asarray(local, dtype=np.int32)
        if op == "sum":
            wide = (a.astype(np.int64) + b.astype(np.int64)) & np.int64(0xFFFFFFFF)
            return wide.astype(np.uint32).view(np.int32)
        return np.maximum(a, b)
    if dtype == "float32":
        a = np.asarray(acc, dtype=np.float32)
        b = np.asarray(local, dtype=np.float32)
        if op == "sum":
            return a + b
        return _float_max(a, b)
    if dtype == "bfloat16":
        a = np.asarray(acc, dtype=np.uint16)
        b = np.asarray(local, dtype=np.uint16)
        fa, fb = bf16_to_f32(a), bf16_to_f32(b)
        if op == "sum":
            return f32_to_bf16_rne(fa + fb)
        # max returns one of its inputs, so the bf16 pattern is carried exactly
        gt = fa > fb
        lt = fb > fa
        pick_b = lt | (~gt & ~lt & np.signbit(fa))
        return np.where(pick_b, b, a).astype(np.uint16)
    raise ValueError(dtype)


def storage_dtype(dtype: str):
    return {"int32": np.int32, "float32": np.float32, "bfloat16": np.uint16}[dtype]


def to_float64(dtype: str, x: np.ndarray) -> np.ndarray:
    """Exact value of each element as fp64 (all three types widen exactly)."""
    if dtype == "bfloat16":
        return bf16_to_f32(x).astype(np.float64)
    return np.asarray(x).astype(np.float64)
