"""Seeded synthetic inputs for the virtual-rank collectives.

This module is shared by the CPU oracle, the tests and the benchmark.  It
holds no part of the collectives' arithmetic: it only draws per-rank input
arrays from seeded generators, with the value distributions and sizes of the
workloads the library is measured on (nccl-tests style size sweeps over ring
and tree collectives; the paper uses no dataset).

Seeding: ``numpy.random.default_rng([0x5EED, workload_id, rank])`` (PCG64), so
every rank of every workload has its own reproducible stream.

Element types and their storage:

* ``int32``    -> ``numpy.int32``, uniform integers in ``[lo, hi]``.
* ``float32``  -> ``numpy.float32``, standard normal N(0, 1) or uniform.
* ``bfloat16`` -> ``numpy.uint16`` holding the bf16 bit pattern.  Values are
  drawn as float32 U(-1, 1) and rounded to the nearest bf16 (ties to even),
  which yields bf16 values in [-1, 1].  The conversion belongs to the
  generator only (it shapes the input distribution); the collectives'
  own rounding is not done here.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 0x5EED

DTYPES = ("int32", "float32", "bfloat16")
ELEM_BYTES = {"int32": 4, "float32": 4, "bfloat16": 2}
STORAGE = {"int32": np.int32, "float32": np.float32, "bfloat16": np.uint16}

# Workload identifiers used in the seed tuple.
WL_RING_AR_SMALL = 1      # ring AllReduce, 4 ranks, int32 in [-1000, 1000]
WL_RING_AR_SWEEP = 2      # ring AllReduce, 8 ranks, fp32 N(0,1), 8 B .. 256 MiB
WL_TREE_AND_CHAINS = 3    # tree AllReduce + ring Bcast/Reduce/AG/RS, 16 ranks
WL_GROUPED = 4            # 64 grouped collectives, 8 ranks
WL_SERVING = 5            # Poisson request stream, 8 ranks
WL_P2P = 6                # Send/Recv pairs and grouped all-to-all


def rng_for(workload_id: int, rank: int, extra: int | None = None) -> np.random.Generator:
    key = [SEED_BASE, int(workload_id), int(rank)]
    if extra is not None:
        key.append(int(extra))
    return np.random.default_rng(key)


def draw(dtype: str, n: int, rng: np.random.Generator, dist: str | None = None,
         lo: int = -1000, hi: int = 1000) -> np.ndarray:
    """Draw ``n`` elements of ``dtype``.

    dist: for int32 ignored (uniform integers in [lo, hi]); for float32
    "normal" (default) or "uniform" (U(-1, 1)); for bfloat16 always U(-1, 1).
    """
    n = int(n)
    if dtype == "int32":
        return rng.integers(lo, hi + 1, size=n, dtype=np.int64).astype(np.int32)
    if dtype == "float32":
        if dist in (None, "normal"):
            return rng.standard_normal(n, dtype=np.float32)
        return rng.uniform(-1.0, 1.0, size=n).astype(np.float32)
    if dtype == "bfloat16":
        f = rng.uniform(-1.0, 1.0, size=n).astype(np.float32)
        return _bf16_nearest(f)
    raise ValueError(f"unknown dtype {dtype}")


def _bf16_nearest(f: np.ndarray) -> np.ndarray:
    """bf16 bit patterns of the finite float32 values f, rounded to nearest,
    ties to even: add just under half a bf16 ulp (plus one when the kept part
    is odd) and drop the low 16 bits."""
    u = np.asarray(f, dtype=np.float32).view(np.uint32).astype(np.uint64)
    odd = (u >> np.uint64(16)) & np.uint64(1)
    return ((u + np.uint64(0x7FFF) + odd) >> np.uint64(16)).astype(np.uint16)


def rank_inputs(workload_id: int, nranks: int, dtype: str, n: int,
                dist: str | None = None, lo: int = -1000, hi: int = 1000,
                extra: int | None = None) -> list[np.ndarray]:
    """One independent array of ``n`` elements per rank."""
    return [draw(dtype, n, rng_for(workload_id, r, extra), dist, lo, hi)
            for r in range(nranks)]


def small_int_valued_float(dtype: str, n: int, rng: np.random.Generator, bound: int) -> np.ndarray:
    """Integer-valued floats in [-bound, bound]: sums of a few of them are exact."""
    v = rng.integers(-bound, bound + 1, size=int(n)).astype(np.float32)
    if dtype == "float32":
        return v
    if dtype == "bfloat16":
        return (v.view(np.uint32) >> np.uint32(16)).astype(np.uint16)
    raise ValueError(dtype)


def log_uniform_sizes(rng: np.random.Generator, count: int, lo_bytes: int, hi_bytes: int) -> np.ndarray:
    """Sizes (bytes) drawn log-uniformly in [lo_bytes, hi_bytes]."""
    u = rng.uniform(np.log(lo_bytes), np.log(hi_bytes), size=int(count))
    return np.exp(u).astype(np.int64)


def poisson_arrivals(rng: np.random.Generator, count: int, rate_per_s: float) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process with the given rate."""
    gaps = rng.exponential(1.0 / float(rate_per_s), size=int(count))
    return np.cumsum(gaps)
