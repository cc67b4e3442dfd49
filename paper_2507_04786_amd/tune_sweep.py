"""Measure the plan space and write the tuner's table.

Runs every collective of ``--nranks`` virtual ranks at per-rank sizes
2^3 .. 2^28 bytes (``--min-log2`` / ``--max-log2``; nccl-tests convention:
the larger per-rank buffer) under
every (algorithm, protocol, channel count) the planner can choose, for
Simple from 1 MiB up every chunk of CHUNKS_SIMPLE (0: the planner's formula)
and workgroup size of THREADS_SIMPLE, for LL / LL128 from 64 KiB up every
workgroup size of THREADS_FLAG (0: the formula), times each point with HIP events on the launch stream, and
writes one JSON line per point.  ``--emit`` turns one or more such files into the C++ table the
planner reads (``csrc/tune_table.inc``), keyed by the chunk and workgroup
size each plan actually ran with: a request of 0 ("the tuner decides")
resolves to the table the library was built with, not to the formula.  One table serves collectives
launched alone and in groups: a different plan in a group would change the
order of a float reduction, and a collective's bits would then depend on its
grouping.  For every (ranks, collective, size bucket) it holds the fastest
measured plan, preferring fewer channels among plans
within 10 % of the best below 16 MiB (3 % from 16 MiB up): a lane left free
serves grouped or concurrent work, and a grouped launch runs every channel
of a collective as its own item, while a large collective's own time
dominates whatever it shares the device with.

Usage:
  python paper_2507_04786_amd/tune_sweep.py --nranks 8 --out sweep_r8.jsonl
  python paper_2507_04786_amd/tune_sweep.py --emit sweep_r4.jsonl sweep_r8.jsonl sweep_r16.jsonl
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
COLLS = ("allreduce", "reducescatter", "allgather", "broadcast", "reduce")
COLL_CODE = {"allreduce": 0, "broadcast": 1, "reduce": 2, "allgather": 3, "reducescatter": 4}
PROTOS = ("simple", "ll", "ll128")
CHANNELS = (1, 2, 4, 8, 16, 32, 64)  # 64 where the communicator's lane limit allows it
CHUNKS_SIMPLE = (0, 32 << 10, 64 << 10, 256 << 10)
CHUNK_MIN_LOG2 = 20
THREADS_FLAG = (0, 256, 1024)  # 0: the formula (512 from 256 KiB, else 256)
THREADS_SIMPLE = (0, 1024)  # Simple from CHUNK_MIN_LOG2 up; 0: the formula's 256
THREADS_MIN_LOG2 = 16
LOG2_MIN, LOG2_MAX = 3, 28
SLOW_MS = 4.0   # a plan slower than this at one size is not tried at larger sizes
TOLERANCE = 1.10  # plans this close to the fastest count as equal; the fewest channels wins
TOLERANCE_LARGE = 1.03  # the same from LARGE_LOG2 up
LARGE_LOG2 = 24


def sweep(args):
    sys.path.insert(0, os.path.dirname(HERE))
    import torch
    import paper_2507_04786_amd as vccl

    R = args.nranks
    torch.cuda.set_device(0)
    top = 1 << args.max_log2
    sends = [torch.empty(top // 4, dtype=torch.float32, device="cuda").normal_() for _ in range(R)]
    recvs = [torch.empty(top // 4, dtype=torch.float32, device="cuda") for _ in range(R)]
    stream = torch.cuda.current_stream()
    comms = vccl.vcclCommInitAll(R)
    out = open(args.out, "w")
    colls = args.colls.split(",") if args.colls else COLLS

    def issue(coll, n):
        for r in range(R):
            s, d = sends[r], recvs[r]
            if coll == "allreduce":
                vccl.vcclAllReduce(s, d, n, vccl.vcclFloat32, vccl.vcclSum, comms[r], stream)
            elif coll == "reducescatter":
                vccl.vcclReduceScatter(s, d, n, vccl.vcclFloat32, vccl.vcclSum, comms[r], stream)
            elif coll == "allgather":
                vccl.vcclAllGather(s, d, n, vccl.vcclFloat32, comms[r], stream)
            elif coll == "broadcast":
                vccl.vcclBroadcast(s, d, n, vccl.vcclFloat32, 0, comms[r], stream)
            else:
                vccl.vcclReduce(s, d, n, vccl.vcclFloat32, vccl.vcclSum, 0, comms[r], stream)

    try:
        for coll in colls:
            algos = ("ring", "tree") if coll == "allreduce" else ("ring",)
            slow = set()
            for lg in range(args.min_log2, args.max_log2 + 1):
                S = 1 << lg
                # count in elements of fp32; AG / RS: size is the larger buffer
                n = S // 4 // (R if coll in ("allgather", "reducescatter") else 1)
                if n < 1:
                    continue
                for algo in algos:
                    for proto in PROTOS:
                        chunks = CHUNKS_SIMPLE if (proto == "simple" and lg >= CHUNK_MIN_LOG2) else (0,)
                        if proto == "simple":
                            threads = THREADS_SIMPLE if lg >= CHUNK_MIN_LOG2 else (0,)
                        else:
                            threads = THREADS_FLAG if lg >= THREADS_MIN_LOG2 else (0,)
                        for C, ck, th in [(C, ck, th) for C in CHANNELS for ck in chunks for th in threads]:
                            key = (algo, proto, C, ck, th)
                            if key in slow:
                                continue
                            try:
                                vccl.vcclCommSetTuning(comms[0], algo=vccl.ALGO_NAMES[algo],
                                                       proto=vccl.PROTO_NAMES[proto], nchannels=C, chunkBytes=ck,
                                                       nthreads=th)
                            except vccl.VcclError:
                                continue  # more channels than this rank count's lane limit
                            issue(coll, n)
                            torch.cuda.synchronize()
                            plan = vccl.vcclCommGetLastPlan(comms[0])
                            t0 = time.perf_counter()
                            issue(coll, n)
                            torch.cuda.synchronize()
                            once = time.perf_counter() - t0
                            reps = max(3, min(20, int(0.004 / max(once, 1e-6))))
                            e0 = torch.cuda.Event(enable_timing=True)
                            e1 = torch.cuda.Event(enable_timing=True)
                            t0 = time.perf_counter()
                            e0.record(stream)
                            for _ in range(reps):
                                issue(coll, n)
                            e1.record(stream)
                            torch.cuda.synchronize()
                            wall = (time.perf_counter() - t0) / reps
                            ms = e0.elapsed_time(e1) / reps
                            err = vccl.vcclCommGetAsyncError(comms[0])
                            if err != vccl.vcclSuccess:
                                raise RuntimeError(f"device error at {coll} {S} {key}")
                            rec = dict(R=R, coll=coll, S=S, log2=lg, algo=algo, proto=proto, C=C, chunkReq=ck, Treq=th,
                                       Cplan=plan["nchannels"], chunk=plan["chunkBytes"],
                                       T=plan["nthreads"], direct=plan["direct"], scope=plan["scope"],
                                       ms=round(ms, 5),
                                       wall_ms=round(wall * 1e3, 5), reps=reps)
                            out.write(json.dumps(rec) + "\n")
                            if ms > SLOW_MS:
                                slow.add(key)
                out.flush()
                print(f"{coll} 2^{lg} done", flush=True)
    finally:
        vccl.vcclCommSetTuning(comms[0])
        for c in comms:
            vccl.vcclCommDestroy(c)
        out.close()


def _chunk_col(r):
    """The chunk the measured plan ran with, for the table's chunk column
    (Simple from CHUNK_MIN_LOG2 up, else 0 = the formula's).  A request of 0
    means "the tuner decides", which resolves to the table the library was
    built with, so the plan's own chunk is what was measured."""
    return r["chunk"] if r["proto"] == "simple" and r["log2"] >= CHUNK_MIN_LOG2 else 0


def _threads_col(r):
    """The workgroup size the measured plan ran with (LL / LL128 from
    THREADS_MIN_LOG2 up, Simple from CHUNK_MIN_LOG2 up, else 0), for the
    same reason."""
    lo = CHUNK_MIN_LOG2 if r["proto"] == "simple" else THREADS_MIN_LOG2
    return r["T"] if r["log2"] >= lo else 0


def _plan_key(r):
    return (r["algo"], r["proto"], r["Cplan"], _chunk_col(r), _threads_col(r))


def pick_best(rows):
    """Per (ranks, collective, size): every plan's time averaged over the
    sweep runs that measured it (one run's figure for a plan can be off by
    20 %), then the fastest, preferring fewer channels within tolerance."""
    best = {}
    for key in sorted({(r["R"], r["coll"], r["log2"]) for r in rows}):
        runs = {}
        for r in rows:
            if (r["R"], r["coll"], r["log2"]) == key:
                runs.setdefault(_plan_key(r), []).append(r)
        cands = [dict(rs[0], ms=sum(x["ms"] for x in rs) / len(rs)) for rs in runs.values()]
        tmin = min(r["ms"] for r in cands)
        tol = TOLERANCE_LARGE if key[2] >= LARGE_LOG2 else TOLERANCE
        near = [r for r in cands if r["ms"] <= tmin * tol]
        best[key] = min(near, key=lambda r: (r["Cplan"], r["ms"]))
    return best


def write_table(best, dest, paths, what):
    lines = ["// Generated by tune_sweep.py --emit from measured sweeps (fp32, sum, tuner-default",
             "// threads); one entry per (ranks, collective, log2 of the per-rank size), " + what + ".",
             "// Fields: nranks, coll, log2 bytes, algo (0 ring, 1 tree), proto (0 Simple, 1 LL,",
             "// 2 LL128), channels, chunk KiB (Simple from 1 MiB; 0: the planner's formula),",
             "// threads (LL / LL128 from 64 KiB, Simple from 1 MiB; used for a collective launched",
             "// alone; 0: the formula), measured microseconds.  Chunk and threads are those the",
             "// measured plan ran with.",
             f"// Sources: {', '.join(os.path.basename(p) for p in paths)}"]
    for (R, coll, lg), r in sorted(best.items(), key=lambda kv: (kv[0][0], COLL_CODE[kv[0][1]], kv[0][2])):
        lines.append("{%d, %d, %d, %d, %d, %d, %d, %d, %.1f}," % (
            R, COLL_CODE[coll], lg, 0 if r["algo"] == "ring" else 1, PROTOS.index(r["proto"]), r["Cplan"],
            _chunk_col(r) // 1024, _threads_col(r), r["ms"] * 1e3))
    open(dest, "w").write("\n".join(lines) + "\n")
    print(f"wrote {len(best)} entries to {dest}")


def emit(paths, dest):
    rows = []
    for p in paths:
        rows += [json.loads(line) for line in open(p) if line.strip()]
    write_table(pick_best(rows), dest, paths, "alone or in a group")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--nranks", type=int, default=8)
    ap.add_argument("--out", default="sweep.jsonl")
    ap.add_argument("--colls", default="")
    ap.add_argument("--min-log2", type=int, default=LOG2_MIN)
    ap.add_argument("--max-log2", type=int, default=LOG2_MAX)
    ap.add_argument("--emit", nargs="*")
    ap.add_argument("--dest", default=os.path.join(HERE, "csrc", "tune_table.inc"))
    args = ap.parse_args()
    if args.emit:
        emit(args.emit, args.dest)
    else:
        sweep(args)


if __name__ == "__main__":
    main()
