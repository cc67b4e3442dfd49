"""Helpers for the GPU tests: per-rank device buffers from seeded numpy inputs,
and one call per rank through the C ABI binding."""
from __future__ import annotations

import numpy as np

NP_STORAGE = {"int32": np.int32, "float32": np.float32, "bfloat16": np.uint16}
ELEM = {"int32": 4, "float32": 4, "bfloat16": 2}


def torch():
    import torch as t
    return t


def to_dev(arr: np.ndarray):
    t = torch()
    a = np.ascontiguousarray(arr)
    if a.dtype == np.uint16:
        a = a.view(np.int16)
    return t.from_numpy(a.copy()).to("cuda")


def from_dev(x, dtype: str) -> np.ndarray:
    a = x.cpu().numpy()
    if dtype == "bfloat16":
        return a.view(np.uint16)
    return a.view(NP_STORAGE[dtype])


def empty_dev(n: int, dtype: str, fill: int = 0x5A):
    """Device buffer of n elements filled with a byte pattern (to catch unwritten output)."""
    t = torch()
    tdt = {"int32": t.int32, "float32": t.float32, "bfloat16": t.int16}[dtype]
    buf = t.empty(max(n, 1), dtype=tdt, device="cuda")
    buf.view(t.uint8).fill_(fill)
    return buf[:n] if n else buf[:0]


def code(vccl, dtype: str) -> int:
    return vccl.DTYPE_NAMES[dtype]


def call(vccl, comms, coll: str, sends, recvs, count: int, dtype: str, op: str = "sum", root: int = 0,
         stream=None):
    dt = code(vccl, dtype)
    o = vccl.OP_NAMES[op]
    for r, comm in enumerate(comms):
        s, d = sends[r], recvs[r]
        if coll == "allreduce":
            vccl.vcclAllReduce(s, d, count, dt, o, comm, stream)
        elif coll == "reducescatter":
            vccl.vcclReduceScatter(s, d, count, dt, o, comm, stream)
        elif coll == "allgather":
            vccl.vcclAllGather(s, d, count, dt, comm, stream)
        elif coll == "broadcast":
            vccl.vcclBroadcast(s, d, count, dt, root, comm, stream)
        elif coll == "reduce":
            vccl.vcclReduce(s, d, count, dt, o, root, comm, stream)
        else:
            raise ValueError(coll)


def recv_len(coll: str, count: int, nranks: int) -> int:
    return count * nranks if coll == "allgather" else count


def send_len(coll: str, count: int, nranks: int) -> int:
    return count * nranks if coll == "reducescatter" else count


def tune(vccl, comms, algo="ring", proto="simple", nchannels=1, chunk=0, nthreads=0, direct=0):
    vccl.vcclCommSetTuning(comms[0], algo=vccl.ALGO_NAMES[algo], proto=vccl.PROTO_NAMES[proto],
                           nchannels=nchannels, nthreads=nthreads, chunkBytes=chunk, direct=direct)


def untune(vccl, comms):
    vccl.vcclCommSetTuning(comms[0])


def init_comms(vccl, R, scope="auto"):
    """Communicator set; scope "xcd" / "device" selects the store policy of
    the traffic between a lane's workgroups (VCCL_SCOPE), "auto" the library
    default (XCD scope)."""
    import os
    old = os.environ.get("VCCL_SCOPE")
    if scope in ("device", "xcd"):
        os.environ["VCCL_SCOPE"] = scope
    try:
        return vccl.vcclCommInitAll(R)
    finally:
        if scope in ("device", "xcd"):
            if old is None:
                del os.environ["VCCL_SCOPE"]
            else:
                os.environ["VCCL_SCOPE"] = old
