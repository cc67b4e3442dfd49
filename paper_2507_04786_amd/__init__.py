"""Python binding of the vccl C ABI (include/vccl.h): argument marshalling only.

Every function keeps the C name and argument order.  Buffers may be given as
torch tensors (their ``data_ptr()`` is passed), integers (device addresses)
or None (NULL); streams as ``torch.cuda.Stream``, an integer hipStream_t or
None (the null stream).  A result other than vcclSuccess raises VcclError
carrying the code; functions that return values through pointers in C return
them here.

The native library is paper_2507_04786_amd/lib/libvccl.so, built in-tree by
``python paper_2507_04786_amd/build.py`` (or ``__graft_entry__.build()``).  Importing this module without it
raises ImportError: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# VCCL_LIB may name another build of the same library (the race-detection
# build, lib/libvccl_jitter.so); the default is the in-tree libvccl.so
LIB_PATH = os.environ.get("VCCL_LIB") or os.path.join(_HERE, "lib", "libvccl.so")

# ---------------------------------------------------------------- constants (vccl.h)
vcclSuccess = 0
vcclUnhandledHipError = 1
vcclSystemError = 2
vcclInternalError = 3
vcclInvalidArgument = 4
vcclInvalidUsage = 5
vcclRemoteError = 6
vcclInProgress = 7

vcclInt32, vcclFloat32, vcclBfloat16 = 0, 1, 2
vcclSum, vcclMax = 0, 1
vcclAlgoAuto, vcclAlgoRing, vcclAlgoTree = -1, 0, 1
vcclProtoAuto, vcclProtoSimple, vcclProtoLL, vcclProtoLL128 = -1, 0, 1, 2
VCCL_MAX_RANKS = 16
VCCL_MAX_CHANNELS = 64

COLL_ALLREDUCE, COLL_BROADCAST, COLL_REDUCE, COLL_ALLGATHER, COLL_REDUCESCATTER = 0, 1, 2, 3, 4

DTYPE_NAMES = {"int32": vcclInt32, "float32": vcclFloat32, "bfloat16": vcclBfloat16}
PROTO_NAMES = {"simple": vcclProtoSimple, "ll": vcclProtoLL, "ll128": vcclProtoLL128}
ALGO_NAMES = {"ring": vcclAlgoRing, "tree": vcclAlgoTree}
OP_NAMES = {"sum": vcclSum, "max": vcclMax}


class VcclError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {vcclGetErrorString(code)} ({code})")


class vcclTuning_t(C.Structure):
    _fields_ = [("algo", C.c_int), ("proto", C.c_int), ("nchannels", C.c_int), ("nthreads", C.c_int),
                ("chunkBytes", C.c_size_t), ("direct", C.c_int)]


class vcclPlanInfo_t(C.Structure):
    _fields_ = [("algo", C.c_int), ("proto", C.c_int), ("nchannels", C.c_int), ("nthreads", C.c_int),
                ("direct", C.c_int), ("nlanes", C.c_int), ("nitems", C.c_int), ("ncolls", C.c_int),
                ("chunkBytes", C.c_size_t), ("grid", C.c_int), ("scope", C.c_int), ("treeRanksPerNode", C.c_int),
                ("ll128", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class vcclRequest_t(C.Structure):
    _fields_ = [("coll", C.c_int), ("datatype", C.c_int), ("op", C.c_int), ("root", C.c_int),
                ("count", C.c_size_t), ("send", C.c_void_p * VCCL_MAX_RANKS), ("recv", C.c_void_p * VCCL_MAX_RANKS)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"vccl native library not built: {LIB_PATH} is missing "
                          "(run python paper_2507_04786_amd/build.py)")
    try:
        # torch ships its own HIP runtime under the same soname; loading it
        # first lets the library bind to that one copy (a second runtime in
        # the process would keep torch from initialising the device)
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    P, I, U64, SZ, VP = C.c_void_p, C.c_int, C.c_uint64, C.c_size_t, C.c_void_p
    sig = {
        "vcclGetErrorString": (C.c_char_p, [I]),
        "vcclGetVersion": (I, [C.POINTER(I)]),
        "vcclCommInitAll": (I, [C.POINTER(P), I, C.POINTER(I)]),
        "vcclCommInitAllRings": (I, [C.POINTER(P), I, C.POINTER(I), I, C.POINTER(I)]),
        "vcclCommGetRings": (I, [P, C.POINTER(I), C.POINTER(I)]),
        "vcclCommDestroy": (I, [P]),
        "vcclCommAbort": (I, [P]),
        "vcclCommGetAsyncError": (I, [P, C.POINTER(I)]),
        "vcclCommCount": (I, [P, C.POINTER(I)]),
        "vcclCommUserRank": (I, [P, C.POINTER(I)]),
        "vcclAllReduce": (I, [VP, VP, SZ, I, I, P, VP]),
        "vcclBroadcast": (I, [VP, VP, SZ, I, I, P, VP]),
        "vcclReduce": (I, [VP, VP, SZ, I, I, I, P, VP]),
        "vcclAllGather": (I, [VP, VP, SZ, I, P, VP]),
        "vcclReduceScatter": (I, [VP, VP, SZ, I, I, P, VP]),
        "vcclSend": (I, [VP, SZ, I, I, P, VP]),
        "vcclRecv": (I, [VP, SZ, I, I, P, VP]),
        "vcclGroupStart": (I, []),
        "vcclGroupEnd": (I, []),
        "vcclCommSetTuning": (I, [P, C.POINTER(vcclTuning_t)]),
        "vcclCommGetLastPlan": (I, [P, C.POINTER(vcclPlanInfo_t)]),
        "vcclCommGetLastTimestamps": (I, [P, C.POINTER(U64), I, C.POINTER(I)]),
        "vcclCommSetTimeout": (I, [P, U64]),
        "vcclCommDebugSetDeadRanks": (I, [P, C.c_uint32]),
        "vcclCommDebugReadFifo": (I, [P, I, I, I, SZ, VP, SZ]),
        "vcclProbeLL128Tear": (I, [I, I, I, I, C.POINTER(U64), C.POINTER(U64)]),
        "vcclProbeXccIds": (I, [I, C.POINTER(I)]),
        "vcclServeCreate": (I, [C.POINTER(P), SZ, I, C.POINTER(P)]),
        "vcclServeSubmit": (I, [P, C.POINTER(vcclRequest_t), C.POINTER(U64)]),
        "vcclServeTest": (I, [P, U64, C.POINTER(I), C.POINTER(I), C.POINTER(U64)]),
        "vcclServeDestroy": (I, [P]),
        "vcclServeReplay": (I, [P, C.POINTER(vcclRequest_t), C.POINTER(U64), I, C.POINTER(U64), C.POINTER(I)]),
        "vcclServeDebugState": (I, [P, C.POINTER(U64), I]),
        "vcclServeGetPlan": (I, [P, U64, C.POINTER(vcclPlanInfo_t)]),
        "vcclCommDebugProfile": (I, [P, I]),
        "vcclCommGetTree": (I, [P, I, C.POINTER(I)]),
        "vcclCommDebugReadProfile": (I, [P, C.POINTER(U64), I, C.POINTER(I)]),
        "vcclAllReduceNoAlloc": (I, [C.POINTER(VP), C.POINTER(VP), I, SZ, I, I, VP, C.POINTER(vcclPlanInfo_t)]),
        "vcclReplayPerCall": (I, [C.POINTER(P), C.POINTER(vcclRequest_t), C.POINTER(U64), I, VP, C.POINTER(U64),
                                  C.POINTER(I)]),
        "vcclDebugPlanHost": (I, [I, I, SZ, I, I, I, C.POINTER(vcclTuning_t), C.POINTER(vcclPlanInfo_t)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()

# Handles created through this module and not yet destroyed.  At interpreter
# exit they are destroyed while the HIP runtime is still fully up (Python's
# exit handlers run before the C runtime's), so no device memory, pinned host
# memory or event of a communicator set is left to the runtime's own teardown.
_live: set = set()


def _destroy_live():
    for h in list(_live):
        _lib.vcclCommDestroy(C.c_void_p(h))
    _live.clear()


import atexit  # noqa: E402

atexit.register(_destroy_live)
EXPORTED = ("vcclGetErrorString vcclGetVersion vcclCommInitAll vcclCommDestroy vcclCommAbort "
            "vcclCommGetAsyncError vcclCommCount vcclCommUserRank vcclAllReduce vcclBroadcast vcclReduce "
            "vcclAllGather vcclReduceScatter vcclSend vcclRecv vcclGroupStart vcclGroupEnd vcclCommSetTuning "
            "vcclCommGetLastPlan "
            "vcclCommGetLastTimestamps vcclCommSetTimeout vcclCommDebugSetDeadRanks vcclCommDebugReadFifo "
            "vcclProbeLL128Tear vcclProbeXccIds vcclServeCreate vcclServeSubmit vcclServeTest "
            "vcclServeDestroy vcclServeReplay vcclServeDebugState vcclServeGetPlan vcclDebugPlanHost "
            "vcclReplayPerCall vcclAllReduceNoAlloc vcclCommDebugProfile vcclCommDebugReadProfile "
            "vcclCommGetTree vcclCommInitAllRings vcclCommGetRings").split()


def lib():
    return _lib


def _ptr(x):
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    return int(x)


def _stream(s):
    if s is None:
        return None
    if hasattr(s, "cuda_stream"):
        return s.cuda_stream
    return int(s)


def _check(res, where):
    if res != vcclSuccess:
        raise VcclError(res, where)


def vcclGetErrorString(code: int) -> str:
    return _lib.vcclGetErrorString(int(code)).decode()


def vcclGetVersion() -> int:
    v = C.c_int()
    _check(_lib.vcclGetVersion(C.byref(v)), "vcclGetVersion")
    return v.value


def vcclCommInitAll(nranks: int, devlist=None, rings=None) -> list:
    """rings: None (every channel on the identity ring) or a list of ring
    orders, each a permutation of range(nranks); channel c follows
    rings[c % len(rings)]."""
    arr = (C.c_void_p * nranks)()
    dl = None if devlist is None else (C.c_int * nranks)(*devlist)
    if rings is None:
        _check(_lib.vcclCommInitAll(arr, int(nranks), dl), "vcclCommInitAll")
    else:
        flat = [int(r) for row in rings for r in row]
        if len(flat) != len(rings) * nranks:
            raise ValueError("every ring order lists nranks ranks")
        _check(_lib.vcclCommInitAllRings(arr, int(nranks), dl, len(rings), (C.c_int * len(flat))(*flat)),
               "vcclCommInitAllRings")
    _live.update(arr[i] for i in range(nranks))
    return [C.c_void_p(arr[i]) for i in range(nranks)]


def vcclCommGetRings(comm) -> list:
    """The set's ring orders: a list of rows, row k the ranks of ring k in order."""
    n = vcclCommCount(comm)
    k = C.c_int()
    _check(_lib.vcclCommGetRings(comm, C.byref(k), None), "vcclCommGetRings")
    arr = (C.c_int * (k.value * n))()
    _check(_lib.vcclCommGetRings(comm, C.byref(k), arr), "vcclCommGetRings")
    return [list(arr[i * n:(i + 1) * n]) for i in range(k.value)]


def vcclCommDestroy(comm):
    _check(_lib.vcclCommDestroy(comm), "vcclCommDestroy")
    _live.discard(comm.value)


def vcclCommAbort(comm):
    _check(_lib.vcclCommAbort(comm), "vcclCommAbort")


def vcclCommGetAsyncError(comm) -> int:
    v = C.c_int()
    _check(_lib.vcclCommGetAsyncError(comm, C.byref(v)), "vcclCommGetAsyncError")
    return v.value


def vcclCommCount(comm) -> int:
    v = C.c_int()
    _check(_lib.vcclCommCount(comm, C.byref(v)), "vcclCommCount")
    return v.value


def vcclCommUserRank(comm) -> int:
    v = C.c_int()
    _check(_lib.vcclCommUserRank(comm, C.byref(v)), "vcclCommUserRank")
    return v.value


def vcclAllReduce(send, recv, count, datatype, op, comm, stream=None):
    _check(_lib.vcclAllReduce(_ptr(send), _ptr(recv), int(count), int(datatype), int(op), comm, _stream(stream)),
           "vcclAllReduce")


def vcclAllReduceNoAlloc(sends, recvs, count, datatype, op, stream=None) -> dict:
    """sends / recvs: one buffer per rank.  Returns the plan that ran."""
    R = len(sends)
    sa = (C.c_void_p * R)(*[_ptr(x) for x in sends])
    ra = (C.c_void_p * R)(*[_ptr(x) for x in recvs])
    info = vcclPlanInfo_t()
    _check(_lib.vcclAllReduceNoAlloc(sa, ra, R, int(count), int(datatype), int(op), _stream(stream),
                                     C.byref(info)), "vcclAllReduceNoAlloc")
    return info.as_dict()


def vcclBroadcast(send, recv, count, datatype, root, comm, stream=None):
    _check(_lib.vcclBroadcast(_ptr(send), _ptr(recv), int(count), int(datatype), int(root), comm, _stream(stream)),
           "vcclBroadcast")


def vcclReduce(send, recv, count, datatype, op, root, comm, stream=None):
    _check(_lib.vcclReduce(_ptr(send), _ptr(recv), int(count), int(datatype), int(op), int(root), comm,
                           _stream(stream)), "vcclReduce")


def vcclAllGather(send, recv, sendcount, datatype, comm, stream=None):
    _check(_lib.vcclAllGather(_ptr(send), _ptr(recv), int(sendcount), int(datatype), comm, _stream(stream)),
           "vcclAllGather")


def vcclReduceScatter(send, recv, recvcount, datatype, op, comm, stream=None):
    _check(_lib.vcclReduceScatter(_ptr(send), _ptr(recv), int(recvcount), int(datatype), int(op), comm,
                                  _stream(stream)), "vcclReduceScatter")


def vcclSend(send, count, datatype, peer, comm, stream=None):
    _check(_lib.vcclSend(_ptr(send), int(count), int(datatype), int(peer), comm, _stream(stream)), "vcclSend")


def vcclRecv(recv, count, datatype, peer, comm, stream=None):
    _check(_lib.vcclRecv(_ptr(recv), int(count), int(datatype), int(peer), comm, _stream(stream)), "vcclRecv")


def vcclGroupStart():
    _check(_lib.vcclGroupStart(), "vcclGroupStart")


def vcclGroupEnd():
    _check(_lib.vcclGroupEnd(), "vcclGroupEnd")


def vcclCommSetTuning(comm, algo=-1, proto=-1, nchannels=0, nthreads=0, chunkBytes=0, direct=-1):
    t = vcclTuning_t(int(algo), int(proto), int(nchannels), int(nthreads), int(chunkBytes), int(direct))
    _check(_lib.vcclCommSetTuning(comm, C.byref(t)), "vcclCommSetTuning")


def vcclCommGetLastPlan(comm) -> dict:
    info = vcclPlanInfo_t()
    _check(_lib.vcclCommGetLastPlan(comm, C.byref(info)), "vcclCommGetLastPlan")
    return info.as_dict()


def vcclCommGetLastTimestamps(comm, n: int) -> list:
    arr = (C.c_uint64 * n)()
    w = C.c_int()
    _check(_lib.vcclCommGetLastTimestamps(comm, arr, int(n), C.byref(w)), "vcclCommGetLastTimestamps")
    return [arr[i] for i in range(w.value)]


def vcclCommDebugProfile(comm, enable: bool = True):
    _check(_lib.vcclCommDebugProfile(comm, int(bool(enable))), "vcclCommDebugProfile")


def vcclCommDebugReadProfile(comm, entries: int) -> list:
    """Per (lane, rank) of the last launch: [start_ns, end_ns, wait_ns, items]."""
    arr = (C.c_uint64 * (4 * entries))()
    w = C.c_int()
    _check(_lib.vcclCommDebugReadProfile(comm, arr, int(entries), C.byref(w)), "vcclCommDebugReadProfile")
    return [list(arr[4 * k:4 * k + 4]) for k in range(w.value)]


def vcclCommGetTree(comm, tree: int) -> list:
    """Parent of every rank in the set's tree `tree` (0 or 1), -1 at the root."""
    n = vcclCommCount(comm)
    arr = (C.c_int * n)()
    _check(_lib.vcclCommGetTree(comm, int(tree), arr), "vcclCommGetTree")
    return list(arr)


def vcclCommSetTimeout(comm, timeout_us: int):
    _check(_lib.vcclCommSetTimeout(comm, int(timeout_us)), "vcclCommSetTimeout")


def vcclCommDebugSetDeadRanks(comm, mask: int):
    _check(_lib.vcclCommDebugSetDeadRanks(comm, int(mask)), "vcclCommDebugSetDeadRanks")


def vcclCommDebugReadFifo(comm, channel, rank, proto, offset, nbytes) -> bytes:
    buf = (C.c_uint8 * int(nbytes))()
    _check(_lib.vcclCommDebugReadFifo(comm, int(channel), int(rank), int(proto), int(offset), buf, int(nbytes)),
           "vcclCommDebugReadFifo")
    return bytes(buf)


def vcclProbeLL128Tear(pairs: int, lines: int, rounds: int, scope: int = 0):
    """scope 0: device-scope (sc1) stores; 1: XCD-scope plain stores (pairs a multiple of 8)."""
    torn, checked = C.c_uint64(), C.c_uint64()
    res = _lib.vcclProbeLL128Tear(int(pairs), int(lines), int(rounds), int(scope), C.byref(torn), C.byref(checked))
    if res not in (vcclSuccess, vcclRemoteError):
        raise VcclError(res, "vcclProbeLL128Tear")
    return torn.value, checked.value, res


def vcclProbeXccIds(n: int) -> list:
    arr = (C.c_int * n)()
    _check(_lib.vcclProbeXccIds(int(n), arr), "vcclProbeXccIds")
    return list(arr)


def vcclServeCreate(comms, budgetBytes: int, lanes: int):
    arr = (C.c_void_p * len(comms))(*[c.value for c in comms])
    out = C.c_void_p()
    _check(_lib.vcclServeCreate(arr, int(budgetBytes), int(lanes), C.byref(out)), "vcclServeCreate")
    return out


def make_request(coll, datatype, op, root, count, sends, recvs) -> vcclRequest_t:
    req = vcclRequest_t()
    req.coll, req.datatype, req.op, req.root, req.count = int(coll), int(datatype), int(op), int(root), int(count)
    for i, s in enumerate(sends):
        req.send[i] = _ptr(s)
    for i, r in enumerate(recvs):
        req.recv[i] = _ptr(r)
    return req


def vcclServeSubmit(server, coll, datatype, op, root, count, sends, recvs) -> int:
    req = make_request(coll, datatype, op, root, count, sends, recvs)
    rid = C.c_uint64()
    _check(_lib.vcclServeSubmit(server, C.byref(req), C.byref(rid)), "vcclServeSubmit")
    return rid.value


def vcclServeTest(server, rid: int):
    done, status, t = C.c_int(), C.c_int(), C.c_uint64()
    _check(_lib.vcclServeTest(server, int(rid), C.byref(done), C.byref(status), C.byref(t)), "vcclServeTest")
    return bool(done.value), status.value, t.value


def vcclServeReplay(server, requests, arrival_ns):
    """requests: list of vcclRequest_t; arrival_ns: offsets from the start.
    Returns (latency_ns list, status list)."""
    n = len(requests)
    arr = (vcclRequest_t * n)(*requests)
    at = (C.c_uint64 * n)(*[int(x) for x in arrival_ns])
    lat = (C.c_uint64 * n)()
    st = (C.c_int * n)()
    _check(_lib.vcclServeReplay(server, arr, at, n, lat, st), "vcclServeReplay")
    return list(lat), list(st)


VCCL_SERVE_DEBUG_WORDS = 7


def vcclServeDebugState(server, entries: int):
    """Per (lane, rank): [posted, seen, picked, done, polls, pickup_tick, finish_tick]."""
    w = VCCL_SERVE_DEBUG_WORDS
    arr = (C.c_uint64 * (w * entries))()
    _check(_lib.vcclServeDebugState(server, arr, int(entries)), "vcclServeDebugState")
    return [list(arr[w * k:w * k + w]) for k in range(entries)]


def vcclReplayPerCall(comms, requests, arrival_ns, stream=None):
    """The same request stream through one launch per request.
    Returns (latency_ns list, status list)."""
    n = len(requests)
    hs = (C.c_void_p * len(comms))(*[c.value for c in comms])
    arr = (vcclRequest_t * n)(*requests)
    at = (C.c_uint64 * n)(*[int(x) for x in arrival_ns])
    lat = (C.c_uint64 * n)()
    st = (C.c_int * n)()
    _check(_lib.vcclReplayPerCall(hs, arr, at, n, _stream(stream), lat, st), "vcclReplayPerCall")
    return list(lat), list(st)


def vcclServeGetPlan(server, rid: int) -> dict:
    info = vcclPlanInfo_t()
    _check(_lib.vcclServeGetPlan(server, int(rid), C.byref(info)), "vcclServeGetPlan")
    return info.as_dict()


def vcclDebugPlanHost(nranks, coll, count, datatype, ll128=1, single=1, tuning=None) -> dict:
    """tuning: None or a dict of vcclCommSetTuning's keyword arguments."""
    info = vcclPlanInfo_t()
    t = None
    if tuning is not None:
        d = dict(algo=-1, proto=-1, nchannels=0, nthreads=0, chunkBytes=0, direct=-1)
        d.update(tuning)
        t = C.byref(vcclTuning_t(int(d["algo"]), int(d["proto"]), int(d["nchannels"]), int(d["nthreads"]),
                                 int(d["chunkBytes"]), int(d["direct"])))
    _check(_lib.vcclDebugPlanHost(int(nranks), int(coll), int(count), int(datatype), int(ll128), int(single), t,
                                  C.byref(info)), "vcclDebugPlanHost")
    return info.as_dict()


def vcclServeDestroy(server):
    _check(_lib.vcclServeDestroy(server), "vcclServeDestroy")


def torch_dtype_code(dt) -> int:
    import torch
    return {torch.int32: vcclInt32, torch.float32: vcclFloat32, torch.bfloat16: vcclBfloat16}[dt]
