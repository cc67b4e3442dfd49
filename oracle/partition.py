"""Channel partition, outer loops and elementary-step chunks.

Follows Section V-C ("Iterative Execution of NCCL Collectives", Fig. 3 and
the channel-buffer table): the input is split into one contiguous region per
channel (``workOffset``, ``channelCount``); a channel region larger than the
channel buffer is processed in outer loop iterations; each elementary step
moves one chunk (``chunkCount`` elements, ``lastChunkCount`` for the last
one).  The unit of partitioning is one byte for AllGather and Broadcast and
one element of the data type for AllReduce, ReduceScatter and Reduce.

The paper prints no formulas.  Readings adopted (identical on the library
side, written independently there):

* Alignment: every channel start and every chunk size is a multiple of
  ``A = 16 / unit_bytes`` units, i.e. of 16 bytes.
* Channels: ``per = roundUp(ceil(n / C), A)``; channel ``c`` owns
  ``[c*per, min(n, (c+1)*per))``, possibly empty.
* Ring AllReduce: a loop iteration covers ``R`` segments of ``K`` units
  (``loopCount = R*K``).  A channel runs ``floor(n_c / (R*K))`` full loops;
  a remainder ``rem > 0`` forms one last loop whose segment size is
  ``K' = roundUp(ceil(rem / R), A)``, segment ``j`` being
  ``[min(rem, j*K'), min(rem, (j+1)*K'))`` -- possibly empty, and an empty
  segment still takes its step.
* Every other collective (ring ReduceScatter, AllGather, Broadcast, Reduce,
  tree AllReduce): the channel region is cut into chunks of ``K`` units,
  ``[j*K, min(n_c, (j+1)*K))``; one loop iteration per chunk.

Fig. 3's worked example (2 channels, chunkCount 2, loopCount 4) is the case
n = 16, C = 2, R = 2, K = 2, A = 1.
"""
from __future__ import annotations


def ceil_div(a: int, b: int) -> int:
    return -(-a // b)


def round_up(a: int, b: int) -> int:
    return ceil_div(a, b) * b


def unit_bytes(coll: str, elem_bytes: int) -> int:
    """Bytes per partition unit: bytes for AllGather/Broadcast, elements otherwise."""
    return 1 if coll in ("allgather", "broadcast") else elem_bytes


def align_units(coll: str, elem_bytes: int) -> int:
    return 16 // unit_bytes(coll, elem_bytes)


def channel_ranges(n: int, nchannels: int, align: int) -> list[tuple[int, int]]:
    """[start, end) of every channel's region, in units."""
    if nchannels < 1:
        raise ValueError("nchannels must be >= 1")
    per = round_up(ceil_div(n, nchannels), align) if n > 0 else 0
    out = []
    for c in range(nchannels):
        s = min(n, c * per)
        e = min(n, (c + 1) * per)
        out.append((s, e))
    return out


def ring_allreduce_loops(n_c: int, nranks: int, chunk: int, align: int) -> list[list[tuple[int, int]]]:
    """Per loop iteration, the R segments [start, end) relative to the channel start."""
    if chunk <= 0 or chunk % align:
        raise ValueError("chunk must be a positive multiple of the alignment")
    loops = []
    loop_count = nranks * chunk
    full = n_c // loop_count
    for l in range(full):
        base = l * loop_count
        loops.append([(base + j * chunk, base + (j + 1) * chunk) for j in range(nranks)])
    rem = n_c - full * loop_count
    if rem > 0:
        base = full * loop_count
        k2 = round_up(ceil_div(rem, nranks), align)
        loops.append([(base + min(rem, j * k2), base + min(rem, (j + 1) * k2)) for j in range(nranks)])
    return loops


def chunk_ranges(n_c: int, chunk: int) -> list[tuple[int, int]]:
    """Elementary-step chunks [start, end) of one channel region (relative)."""
    if chunk <= 0:
        raise ValueError("chunk must be positive")
    return [(s, min(n_c, s + chunk)) for s in range(0, n_c, chunk)]
