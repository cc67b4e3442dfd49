"""Benchmark: ring AllReduce of 8 virtual ranks on one MI355X.

Workload (the configuration the headline metric is quoted on): ring
AllReduce, sum, 8 virtual ranks, fp32 N(0,1) synthetic inputs, 64 MiB per
rank, plan chosen by the library's tuner.  One step = one AllReduce (the
eight per-rank calls, matched into one launch).  Prints ONE JSON line:

  value       busBW = algBW * 2(R-1)/R, algBW = bytes per rank / step time
  roofline    HBM-bound kernel: algorithmic bytes of one launch / its average
              duration (HIP events on the launch stream over the timed
              region) against the 8 TB/s HBM3E peak
  protocols   the same AllReduce forced to each protocol (busBW, HBM fraction)
  sizes       the AllReduce at 8 B .. 16 MiB per rank, tuner plan and each
              protocol forced: us per call (issued from Python), busBW, HBM
              fraction
  large_sizes the tuned AllReduce at 128 and 256 MiB per rank
  collectives_r16  every collective (and the tree AllReduce) at 16 ranks, bf16,
              64 MiB per rank: busBW and HBM fraction
  alltoall    grouped Send/Recv between all 8 x 8 rank pairs, 64 MiB per rank:
              the launch's device time and the host-inclusive time
  grouped     64 mixed collectives (AR/AG/RS, 4 KiB..16 MiB log-uniform, fp32 /
              bf16 / int32) in one GroupStart/GroupEnd launch against one
              launch per collective, and the same for a batch of sub-1 MiB
              collectives; bit equality of the two paths is checked
  serving     Poisson request streams (AR 60 % / AG 20 % / RS 20 %, 1 KiB..128 MiB
              log-uniform) replayed through the continuous-batching server at
              several arrival rates, and the same streams through one launch
              per request: p50 / p99 latency overall and per size bucket,
              offered vs achieved rate; a server of 32 lanes ('serving', one
              workgroup per CU) and of 64 ('serving_lanes64': a request of
              16 MiB or more holds half the lanes, so small requests run
              beside it)
  cpu_baseline the CPU oracle (numpy schedule simulation) on the same inputs
              and plan, timed on the host's cores, and the timed launch's
              result checked bit for bit on every element against the
              oracle's step simulation and its closed-form fold

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--size-mib 64]
                       [--no-cpu] [--no-protocols] [--no-grouped] [--no-serving]
                       [--no-collectives] [--serve-lanes 32,64]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "busBW GB/s & % HBM peak per protocol/size; p50/p99 latency of request stream"


def alg_bytes_per_launch(plan: dict, nranks: int, size: int) -> float:
    """Bytes the ring AllReduce schedule must load and store, FIFO and flag
    overhead included: [2R + 4f(R-1)] S, f = 1 / 2 / 16/15 for Simple / LL /
    LL128; (5R - 4) S when the AllGather phase writes straight into the peers'
    buffers (direct).  Tree AllReduce moves the same bytes as the ring."""
    R = nranks
    proto = plan["proto"]
    if proto == 0 and plan["direct"] and plan["algo"] == 0:
        return (5 * R - 4) * size
    f = {0: 1.0, 1: 2.0, 2: 16.0 / 15.0}[proto]
    return (2 * R + 4 * f * (R - 1)) * size


def progress(msg: str) -> None:
    """One line on stderr as each leg of the run ends (the JSON line stays
    alone on stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def kernel_source_digest() -> str:
    """Digest of what decides the launch's memory traffic: the kernel's
    sources (device code and the structures it shares with the host), the
    planner and the tuner's table (plan, chunk and store policy).  A recorded
    counter reading applies while it is unchanged."""
    import hashlib
    h = hashlib.sha256()
    for name in ("device.hip", "vccl_dev.h", "host_plan.cpp", "tune_table.inc"):
        with open(os.path.join(ROOT, "paper_2507_04786_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel_key: str):
    """HBM bytes per launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE,
    from profiles/<key>.traffic.json when it was taken on the current kernel."""
    path = os.path.join(ROOT, "profiles", kernel_key + ".traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        if rec.get("kernel_src_sha256_16") != kernel_source_digest():
            return None
        return float(rec["bytes_per_launch"])
    except Exception:
        return None


COLL_CODES = {"allreduce": 0, "broadcast": 1, "reduce": 2, "allgather": 3, "reducescatter": 4}
DTYPES = ("float32", "bfloat16", "int32")
ELEM = {"float32": 4, "bfloat16": 2, "int32": 4}


def _send_arenas(torch, si, workload, R, nbytes):
    """Per (dtype, rank): nbytes of seeded synthetic values on the device
    (fp32 N(0,1), bf16 U(-1,1), int32 U[-2^20, 2^20]), built by tiling a
    4 MiB draw.  Collectives read slices of these; they are never written."""
    import numpy as np
    out = {}
    tile = 4 << 20
    for dt in DTYPES:
        E = ELEM[dt]
        kw = dict(lo=-2 ** 20, hi=2 ** 20) if dt == "int32" else {}
        per = []
        for r in range(R):
            x = si.draw(dt, tile // E, si.rng_for(workload, r, 77), **kw)
            t = torch.from_numpy(np.ascontiguousarray(x).view(np.uint8)).cuda()
            per.append(t.repeat(max(1, nbytes // tile)))
        out[dt] = per
    return out


def _batch_specs(si, seed, count, lo, hi, R):
    rng = si.rng_for(si.WL_GROUPED, 0, seed)
    sizes = si.log_uniform_sizes(rng, count, lo, hi)
    specs = []
    for i in range(count):
        coll = ("allreduce", "allgather", "reducescatter")[int(rng.integers(0, 3))]
        dt = DTYPES[int(rng.integers(0, 3))]
        E = ELEM[dt]
        n = max(1, int(sizes[i]) // E // (R if coll != "allreduce" else 1))
        specs.append((coll, dt, n))
    return specs


def coll_alg_bytes(coll, plan, R, size):
    """Algorithmic bytes of one launch (FIFO traffic included; f = 1 / 2 /
    16/15 for Simple / LL / LL128).  size = the larger per-rank buffer.
    AllReduce as alg_bytes_per_launch; ReduceScatter / AllGather with block
    b = size / R: R [R + 1 + 2f(R-1)] b, or R (2R - 1) b for a direct
    AllGather; Broadcast / Reduce: [R + 1 + 2f(R-1)] size, or (2R - 1) size
    for a direct Broadcast (the step table's bytes; the kernel, whose last
    rank makes the root's local copy, reads the root's input once more)."""
    f = {0: 1.0, 1: 2.0, 2: 16.0 / 15.0}[plan["proto"]]
    direct = plan["proto"] == 0 and plan["direct"]
    if coll == "allreduce":
        return alg_bytes_per_launch(plan, R, size)
    if coll in ("reducescatter", "allgather"):
        b = size / R
        if coll == "allgather" and direct:
            return R * (2 * R - 1) * b
        return R * (R + 1 + 2 * f * (R - 1)) * b
    if coll == "broadcast" and direct:
        return (2 * R - 1) * size
    return (R + 1 + 2 * f * (R - 1)) * size


def collectives_leg(vccl, torch, si, R=16, size=64 << 20, steps=10):
    """Every collective at one size: 16 ranks, bf16 U(-1,1), sum (the tree /
    chain workload), tuner plans plus the tree forced for AllReduce."""
    arenas = _send_arenas(torch, si, si.WL_TREE_AND_CHAINS, R, size)["bfloat16"]
    recvs = [torch.empty(size, dtype=torch.uint8, device="cuda") for _ in range(R)]
    comms = vccl.vcclCommInitAll(R)
    stream = torch.cuda.current_stream()
    bf = vccl.vcclBfloat16
    bus = {"allreduce": 2 * (R - 1) / R, "reducescatter": (R - 1) / R, "allgather": (R - 1) / R,
           "broadcast": 1.0, "reduce": 1.0}
    out = {"nranks": R, "bytes_per_rank": size, "dtype": "bf16", "op": "sum"}
    try:
        for name, coll, algo in (("allreduce", "allreduce", -1), ("allreduce_tree", "allreduce", 1),
                                 ("reducescatter", "reducescatter", -1), ("allgather", "allgather", -1),
                                 ("broadcast", "broadcast", -1), ("reduce", "reduce", -1)):
            vccl.vcclCommSetTuning(comms[0], algo=algo)
            n = size // 2 // (R if coll in ("allgather", "reducescatter") else 1)

            def issue():
                for r in range(R):
                    s, d = arenas[r], recvs[r]
                    if coll == "allreduce":
                        vccl.vcclAllReduce(s, d, n, bf, vccl.vcclSum, comms[r], stream)
                    elif coll == "reducescatter":
                        vccl.vcclReduceScatter(s, d, n, bf, vccl.vcclSum, comms[r], stream)
                    elif coll == "allgather":
                        vccl.vcclAllGather(s, d, n, bf, comms[r], stream)
                    elif coll == "broadcast":
                        vccl.vcclBroadcast(s, d, n, bf, 0, comms[r], stream)
                    else:
                        vccl.vcclReduce(s, d, n, bf, vccl.vcclSum, 0, comms[r], stream)

            for _ in range(2):
                issue()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                issue()
            e1.record(stream)
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) / 1e3 / steps
            err = vccl.vcclCommGetAsyncError(comms[0])
            if err != vccl.vcclSuccess:
                raise RuntimeError(f"device error {vccl.vcclGetErrorString(err)} in {name}")
            plan = vccl.vcclCommGetLastPlan(comms[0])
            ab = coll_alg_bytes(coll, plan, R, size)
            out[name] = {"ms": round(t * 1e3, 4), "busbw_gbs": round(size / t / 1e9 * bus[coll], 2),
                         "hbm_frac": round(ab / t / 1e9 / HBM_PEAK_GBS, 4),
                         "algo": ["ring", "tree"][plan["algo"]], "proto": ["simple", "ll", "ll128"][plan["proto"]],
                         "nchannels": plan["nchannels"], "nthreads": plan["nthreads"],
                         "chunk_bytes": plan["chunkBytes"], "direct": plan["direct"]}
            if name in ("allreduce", "allreduce_tree"):
                out[name]["roles"] = role_profile(vccl, torch, comms, issue, plan)
    finally:
        vccl.vcclCommSetTuning(comms[0])
        for c in comms:
            vccl.vcclCommDestroy(c)
    return out


def role_profile(vccl, torch, comms, issue, plan):
    """One more launch of `issue` with per-workgroup profiling on: for every
    (lane, rank) its span and the part spent waiting for step counters.
    Grouped by role -- for a tree, the rank's place in its channel's tree
    (leaf, interior, root) and, for a split channel, the half (up / down);
    for a ring, one group -- with the median busy fraction (1 - wait / span)
    and the median span of each group."""
    import numpy as np
    R = len(comms)
    vccl.vcclCommDebugProfile(comms[0], True)
    try:
        issue()
        torch.cuda.synchronize()
        recs = vccl.vcclCommDebugReadProfile(comms[0], 64 * R)
    finally:
        vccl.vcclCommDebugProfile(comms[0], False)
    C = plan["nchannels"]
    split = plan["algo"] == 1 and plan["nlanes"] > C
    off = 8 * ((C + 7) // 8)
    parents = [vccl.vcclCommGetTree(comms[0], t) for t in (0, 1)] if plan["algo"] == 1 else None
    groups = {}
    for k, (t0, t1, wait, items) in enumerate(recs):
        if not items:
            continue
        lane, rank = divmod(k, R)
        if parents is None:
            key = "ring"
        else:
            ch = lane if lane < C else lane - off
            par = parents[ch % 2]
            nk = sum(1 for q in range(R) if par[q] == rank)
            role = "root" if par[rank] < 0 else ("leaf" if nk == 0 else "interior")
            key = (("up_" if lane < C else "down_") if split else "") + role
        span = max(1, t1 - t0)
        groups.setdefault(key, []).append((1.0 - wait / span, span))
    return {k: {"workgroups": len(v), "busy_frac_median": round(float(np.median([b for b, _ in v])), 3),
                "span_us_median": round(float(np.median([sp for _, sp in v])) / 1e3, 1)}
            for k, v in sorted(groups.items())}


def alltoall_leg(vccl, torch, si, R=8, size=64 << 20, steps=10):
    """All-to-all through grouped Send/Recv: R ranks, fp32, `size` bytes per
    rank (R blocks of size / R), one group of R * R transfers per step.
    Algorithmic bytes: every byte is read once and written once, 2 R size.
    `ms` is the launch on the device (staging copies and kernel);
    `host_inclusive_ms` adds the host's issue and planning of the group."""
    import numpy as np
    n = size // 4 // R
    xs = si.rank_inputs(si.WL_P2P, R, "float32", 1 << 20)
    sends = [torch.from_numpy(x).cuda().repeat(R * n // (1 << 20)) for x in xs]
    recvs = [torch.empty(R * n, dtype=torch.float32, device="cuda") for _ in range(R)]
    comms = vccl.vcclCommInitAll(R)
    stream = torch.cuda.current_stream()

    def issue(ev=None):
        vccl.vcclGroupStart()
        for a in range(R):
            for b in range(R):
                vccl.vcclSend(sends[a][b * n:(b + 1) * n], n, vccl.vcclFloat32, b, comms[a], stream)
                vccl.vcclRecv(recvs[b][a * n:(a + 1) * n], n, vccl.vcclFloat32, a, comms[b], stream)
        if ev:
            ev[0].record(stream)
        vccl.vcclGroupEnd()
        if ev:
            ev[1].record(stream)

    try:
        for _ in range(2):
            issue()
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        t0 = time.perf_counter()
        for k in range(steps):
            issue(evs[k])
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        # the launch's own duration on the device: each group's events
        # queued behind a spin kernel (about 1.5 ms) that keeps the device
        # busy while GroupEnd plans the 2 R^2 calls on the host, so they
        # bracket the staging copies and the kernel only
        dev = []
        spin = getattr(torch.cuda, "_sleep", None)  # without it the events include the host's planning
        for k in range(steps):
            vccl.vcclGroupStart()
            for a in range(R):
                for b in range(R):
                    vccl.vcclSend(sends[a][b * n:(b + 1) * n], n, vccl.vcclFloat32, b, comms[a], stream)
                    vccl.vcclRecv(recvs[b][a * n:(a + 1) * n], n, vccl.vcclFloat32, a, comms[b], stream)
            if spin is not None:
                spin(1_000_000)
            evs[k][0].record(stream)
            vccl.vcclGroupEnd()
            evs[k][1].record(stream)
            torch.cuda.synchronize()
            dev.append(evs[k][0].elapsed_time(evs[k][1]))
        t = float(np.median(dev)) / 1e3
        err = vccl.vcclCommGetAsyncError(comms[0])
        if err != vccl.vcclSuccess:
            raise RuntimeError(f"device error {vccl.vcclGetErrorString(err)} in all-to-all")
        plan = vccl.vcclCommGetLastPlan(comms[0])
        ok = all(bool(torch.equal(recvs[b][a * n:a * n + 4096], sends[a][b * n:b * n + 4096]))
                 for a in range(R) for b in range(R))
    finally:
        for c in comms:
            vccl.vcclCommDestroy(c)
    return {"nranks": R, "bytes_per_rank": size, "transfers": R * R, "ms": round(t * 1e3, 4),
            "host_inclusive_ms": round(wall * 1e3, 4), "device_timed": spin is not None,
            "busbw_gbs": round(size / t / 1e9 * (R - 1) / R, 2),
            "hbm_frac": round(2 * R * size / t / 1e9 / HBM_PEAK_GBS, 4),
            "lanes": plan["nlanes"], "items": plan["nitems"], "sampled_blocks_equal": ok}


def sizes_leg(vccl, torch, comms, sends, recvs, stream):
    """The same AllReduce at sizes from 8 B to 16 MiB per rank under the
    tuner's plan and under each protocol forced (ring): microseconds per call,
    issued from Python one call per rank (below about 1 MiB the host's issue
    time, about 13 us a call, dominates), busBW and the HBM fraction of the
    plan's algorithmic bytes."""
    R = len(comms)
    out = {}
    for S in (8, 64 << 10, 1 << 20, 16 << 20):
        n = S // 4
        row = {}
        for name, algo, proto in (("tuned", -1, -1), ("simple", vccl.vcclAlgoRing, vccl.vcclProtoSimple),
                                  ("ll", vccl.vcclAlgoRing, vccl.vcclProtoLL),
                                  ("ll128", vccl.vcclAlgoRing, vccl.vcclProtoLL128)):
            vccl.vcclCommSetTuning(comms[0], algo=algo, proto=proto)

            def issue():
                for r in range(R):
                    vccl.vcclAllReduce(sends[r], recvs[r], n, vccl.vcclFloat32, vccl.vcclSum, comms[r], stream)

            for _ in range(3):
                issue()
            torch.cuda.synchronize()
            reps = 50 if S <= (1 << 20) else 10
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                issue()
            e1.record(stream)
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) / reps / 1e3
            p = vccl.vcclCommGetLastPlan(comms[0])
            row[name] = {"us_per_call": round(t * 1e6, 2), "busbw_gbs": round(S / t / 1e9 * 2 * (R - 1) / R, 3),
                         "hbm_frac": round(alg_bytes_per_launch(p, R, S) / t / 1e9 / HBM_PEAK_GBS, 4),
                         "algo": ["ring", "tree"][p["algo"]], "proto": ["simple", "ll", "ll128"][p["proto"]],
                         "nchannels": p["nchannels"]}
        out[str(S)] = row
    vccl.vcclCommSetTuning(comms[0])
    return out


def large_leg(vccl, torch, comms, sends, stream, sizes_mib=(128, 256), reps=10):
    """The tuned AllReduce above the headline size: 128 and 256 MiB per rank,
    where the buffers of all ranks (2-4 GiB each way) no longer fit in the
    memory-side cache.  Inputs are the headline's N(0,1) buffers tiled on
    the device.  Kernel time from events on the launch stream, busBW and the
    HBM fraction of the plan's algorithmic bytes."""
    R = len(comms)
    out = {}
    for mib in sizes_mib:
        S = mib << 20
        n = S // 4
        big_s = [x.repeat((n + x.numel() - 1) // x.numel())[:n].contiguous() for x in sends]
        big_r = [torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(R)]

        def issue():
            for r in range(R):
                vccl.vcclAllReduce(big_s[r], big_r[r], n, vccl.vcclFloat32, vccl.vcclSum, comms[r], stream)

        for _ in range(2):
            issue()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            issue()
        e1.record(stream)
        torch.cuda.synchronize()
        err = vccl.vcclCommGetAsyncError(comms[0])
        if err != vccl.vcclSuccess:
            raise RuntimeError(f"device error {vccl.vcclGetErrorString(err)}")
        t = e0.elapsed_time(e1) / reps / 1e3
        p = vccl.vcclCommGetLastPlan(comms[0])
        out[str(S)] = {"ms": round(t * 1e3, 4), "busbw_gbs": round(S / t / 1e9 * 2 * (R - 1) / R, 2),
                       "hbm_frac": round(alg_bytes_per_launch(p, R, S) / t / 1e9 / HBM_PEAK_GBS, 4),
                       "proto": ["simple", "ll", "ll128"][p["proto"]], "nchannels": p["nchannels"],
                       "chunk_bytes": p["chunkBytes"]}
        del big_s, big_r
        torch.cuda.empty_cache()
    return out


def grouped_leg(vccl, torch, si, comms, stream, seeds=10, reps=3):
    """64 collectives issued in one group against 64 separate launches, over
    `seeds` seeded batches.  Per batch: the time from the first call's issue
    to the last kernel's end (events on the launch stream, the host's issue
    and planning included, as a caller sees it) and the same with the
    launches queued behind a spin kernel (device time only).  Per
    collective: its completion latency from the batch's start -- per-call,
    an event after each launch; grouped, the launch's end less the time by
    which the collective's own completion stamp (the device clock, latest
    over its ranks) precedes the last one.  p50 / p99 over the sub-1 MiB
    collectives of all batches, both paths, both timings.  The two paths'
    outputs are compared bit for bit on every batch."""
    import numpy as np
    R = len(comms)
    arenas = _send_arenas(torch, si, si.WL_GROUPED, R, 16 << 20)
    codes = {"float32": vccl.vcclFloat32, "bfloat16": vccl.vcclBfloat16, "int32": vccl.vcclInt32}
    spin = getattr(torch.cuda, "_sleep", None)
    result = {"seeds": seeds, "reps_per_seed": reps}
    for name, lo, hi in (("mixed_4KiB_16MiB", 4 << 10, 16 << 20), ("sub_1MiB", 4 << 10, 1 << 20)):
        tot = {(g, d): [] for g in (0, 1) for d in (0, 1)}
        lat = {(g, d): [] for g in (0, 1) for d in (0, 1)}
        same, nbytes, nsub, ncoll, lanes = True, 0, 0, 0, 0
        for seed in range(1, seeds + 1):
            specs = _batch_specs(si, seed, 64, lo, hi, R)
            sizes = [n * ELEM[dt] * (R if c != "allreduce" else 1) for c, dt, n in specs]
            small = np.array([x < (1 << 20) for x in sizes])
            nbytes += int(sum(sizes))
            nsub += int(small.sum())
            ncoll += len(specs)
            recvs = []
            for coll, dt, n in specs:
                rl = n * R if coll == "allgather" else n
                recvs.append([torch.empty(rl * ELEM[dt], dtype=torch.uint8, device="cuda") for _ in range(R)])

            def issue_one(k):
                coll, dt, n = specs[k]
                for r in range(R):
                    sb, d = arenas[dt][r], recvs[k][r]
                    if coll == "allreduce":
                        vccl.vcclAllReduce(sb, d, n, codes[dt], vccl.vcclSum, comms[r], stream)
                    elif coll == "allgather":
                        vccl.vcclAllGather(sb, d, n, codes[dt], comms[r], stream)
                    else:
                        vccl.vcclReduceScatter(sb, d, n, codes[dt], vccl.vcclSum, comms[r], stream)

            def batch(group, device_only):
                if device_only and spin is not None:
                    # about 3.3 ms: longer than the host takes to issue a per-call
                    # batch (512 calls and 64 launches, about 1.3 ms), so the
                    # launches queue up and run back to back
                    spin(8_000_000)
                e0 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                evs = []
                if group:
                    vccl.vcclGroupStart()
                    for k in range(len(specs)):
                        issue_one(k)
                    vccl.vcclGroupEnd()
                    e1 = torch.cuda.Event(enable_timing=True)
                    e1.record(stream)
                else:
                    for k in range(len(specs)):
                        issue_one(k)
                        ev = torch.cuda.Event(enable_timing=True)
                        ev.record(stream)
                        evs.append(ev)
                    e1 = evs[-1]
                torch.cuda.synchronize()
                total = e0.elapsed_time(e1)
                if group:
                    st = np.array(vccl.vcclCommGetLastTimestamps(comms[0], len(specs)), dtype=np.float64)
                    per = total - (st.max() - st) / 1e6
                else:
                    per = np.array([e0.elapsed_time(ev) for ev in evs])
                return total, per

            for group in (0, 1):
                batch(group, False)  # warm-up (and the output the other path is compared with)
                if group == 0:
                    snap = [[x.clone() for x in rr] for rr in recvs]
                    for rr in recvs:
                        for x in rr:
                            x.fill_(0x5A)
                for device_only in (0, 1):
                    if device_only and spin is None:
                        continue
                    for _ in range(reps):
                        t, per = batch(group, device_only)
                        tot[(group, device_only)].append(t)
                        lat[(group, device_only)].extend(per[small].tolist())
            lanes = max(lanes, vccl.vcclCommGetLastPlan(comms[0])["nlanes"])
            same = same and all(bool(torch.equal(a, b)) for ra, rb in zip(snap, recvs) for a, b in zip(ra, rb))
            err = vccl.vcclCommGetAsyncError(comms[0])
            if err != vccl.vcclSuccess:
                raise RuntimeError(f"device error {vccl.vcclGetErrorString(err)} in grouped leg")
            del recvs, snap

        def med(key):
            return round(float(np.median(tot[key])), 4) if tot[key] else None

        def pct(key):
            v = lat[key]
            if not v:
                return None
            return {"p50_us": round(float(np.percentile(v, 50)) * 1e3, 1),
                    "p99_us": round(float(np.percentile(v, 99)) * 1e3, 1), "n": len(v)}

        g, pc, gd, pcd = med((1, 0)), med((0, 0)), med((1, 1)), med((0, 1))
        result[name] = {"ncolls_per_batch": 64, "bytes_per_batch": int(nbytes / seeds),
                        "sub_1MiB_fraction": round(nsub / ncoll, 3),
                        "grouped_ms": g, "per_call_ms": pc, "speedup": round(pc / g, 3),
                        "grouped_device_ms": gd, "per_call_device_ms": pcd,
                        "device_speedup": round(pcd / gd, 3) if gd and pcd else None,
                        "sub_1MiB_latency": {"grouped": pct((1, 0)), "per_call": pct((0, 0)),
                                             "grouped_device": pct((1, 1)), "per_call_device": pct((0, 1))},
                        "lanes": lanes, "grouped_equals_per_call": same}
    return result


SIZE_BUCKETS = (("under_1MiB", 0, 1 << 20), ("1_to_16MiB", 1 << 20, 16 << 20), ("over_16MiB", 16 << 20, 1 << 62))


def _stream_requests(vccl, si, rng, total, R, base_s, base_r, arena, codes, layout):
    """A request stream of the serving workload: AR 60 % / AG 20 % / RS 20 %,
    1 KiB..128 MiB log-uniform, dtypes uniform, ragged counts.  layout
    "random": buffers at random 16-byte aligned offsets of shared arenas
    (they overlap: timing only); "packed": every request's receive buffers
    at their own offsets (results can be compared)."""
    sizes = si.log_uniform_sizes(rng, total, 1 << 10, 128 << 20)
    reqs, meta, off_r = [], [], 0
    for i in range(total):
        u = rng.uniform()
        coll = "allreduce" if u < 0.6 else ("allgather" if u < 0.8 else "reducescatter")
        dt = DTYPES[int(rng.integers(0, 3))]
        E = ELEM[dt]
        n = max(1, int(sizes[i]) // E // (R if coll != "allreduce" else 1))
        span_s = n * E * (R if coll == "reducescatter" else 1)
        span_r = n * E * (R if coll == "allgather" else 1)
        off_s = int(rng.integers(0, (arena - span_s) // 16 + 1)) * 16
        if layout == "random":
            o = int(rng.integers(0, (arena - span_r) // 16 + 1)) * 16
        else:
            o = off_r
            off_r += (span_r + 255) // 256 * 256
        reqs.append(vccl.make_request(COLL_CODES[coll], codes[dt], vccl.vcclSum, 0, n,
                                      [b + off_s for b in base_s[dt]], [b + o for b in base_r]))
        meta.append((coll, dt, n, int(sizes[i]), o, span_r))
    return reqs, meta, off_r


def _bucket_stats(lat_us, sizes):
    import numpy as np
    out = {}
    for name, lo, hi in SIZE_BUCKETS:
        m = (sizes >= lo) & (sizes < hi)
        if m.any():
            out[name] = {"n": int(m.sum()), "p50_us": round(float(np.percentile(lat_us[m], 50)), 1),
                         "p99_us": round(float(np.percentile(lat_us[m], 99)), 1)}
    return out


def serving_leg(vccl, torch, si, R, rates, nreq, nwarm, lanes=32, budget=4 << 30, check_requests=120):
    """Poisson request streams through the continuous-batching server and,
    for the same streams (same requests, same arrival times), through one
    launch per request (vcclReplayPerCall, native like the server's loop).
    Per rate: offered vs achieved rate and p50 / p99 latency, overall and per
    size bucket, for both paths.  Then a check stream with every request's
    receive buffers apart, served and per-call: the outputs compared bit for
    bit."""
    import numpy as np
    arena = 128 << 20
    arenas = _send_arenas(torch, si, si.WL_SERVING, R, arena)
    recv = [torch.empty(arena, dtype=torch.uint8, device="cuda") for _ in range(R)]
    base_s = {dt: [t.data_ptr() for t in arenas[dt]] for dt in DTYPES}
    base_r = [t.data_ptr() for t in recv]
    codes = {"float32": vccl.vcclFloat32, "bfloat16": vccl.vcclBfloat16, "int32": vccl.vcclInt32}
    comms = vccl.vcclCommInitAll(R)
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    out = {"lanes": lanes, "budget_bytes": budget, "requests_per_rate": nreq, "warmup_per_rate": nwarm,
           "rates": []}

    def summary(lat_ns, arr, sizes):
        lat = np.asarray(lat_ns[nwarm:], dtype=np.float64) / 1e3
        done = arr[nwarm:] + lat / 1e6
        span = float(done.max() - arr[nwarm])
        return {"achieved_per_s": round(nreq / span, 1), "p50_us": round(float(np.percentile(lat, 50)), 1),
                "p99_us": round(float(np.percentile(lat, 99)), 1), "by_size": _bucket_stats(lat, sizes[nwarm:])}

    try:
        for k, lam in enumerate(rates):
            rng = si.rng_for(si.WL_SERVING, 0, 100 + k)
            total = nreq + nwarm
            reqs, meta, _ = _stream_requests(vccl, si, rng, total, R, base_s, base_r, arena, codes, "random")
            sizes = np.array([m[3] for m in meta])
            arr = si.poisson_arrivals(rng, total, lam)
            at = (arr * 1e9).astype(np.int64)
            srv = vccl.vcclServeCreate(comms, budget, lanes)
            try:
                lat_s, st = vccl.vcclServeReplay(srv, reqs, at)
            finally:
                vccl.vcclServeDestroy(srv)
            if any(x != vccl.vcclSuccess for x in st):
                raise RuntimeError("serving: a request failed")
            lat_p, st = vccl.vcclReplayPerCall(comms, reqs, at, stream)
            if any(x != vccl.vcclSuccess for x in st):
                raise RuntimeError("per-call replay: a request failed")
            row = {"offered_per_s": lam, "mean_bytes": int(sizes.mean())}
            row.update(summary(lat_s, arr, sizes))
            row["per_call"] = summary(lat_p, arr, sizes)
            out["rates"].append(row)
        # bit check: a stream with every request's receive buffers apart
        rng = si.rng_for(si.WL_SERVING, 0, 99)
        del recv
        torch.cuda.empty_cache()
        probe, meta, need = _stream_requests(vccl, si, rng, check_requests, R, base_s, [0] * R, arena, codes,
                                             "packed")
        rbufs = [torch.empty(need, dtype=torch.uint8, device="cuda") for _ in range(R)]
        reqs = [vccl.make_request(q.coll, q.datatype, q.op, q.root, q.count, list(q.send),
                                  [rbufs[r].data_ptr() + m[4] for r in range(R)]) for q, m in zip(probe, meta)]
        arr = (si.poisson_arrivals(rng, check_requests, 5000.0) * 1e9).astype(np.int64)
        for t in rbufs:
            t.fill_(0x5A)
        torch.cuda.synchronize()
        srv = vccl.vcclServeCreate(comms, budget, lanes)
        try:
            _, st = vccl.vcclServeReplay(srv, reqs, arr)
        finally:
            vccl.vcclServeDestroy(srv)
        served = [t.clone() for t in rbufs]
        for t in rbufs:
            t.fill_(0x5A)
        torch.cuda.synchronize()
        _, st2 = vccl.vcclReplayPerCall(comms, reqs, arr, stream)
        torch.cuda.synchronize()
        equal = 0
        for m in meta:
            o, span = m[4], m[5]
            equal += all(bool(torch.equal(served[r][o:o + span], rbufs[r][o:o + span])) for r in range(R))
        out["served_equals_per_call"] = {"requests": check_requests, "equal": int(equal),
                                         "arrival_rate_per_s": 5000.0,
                                         "all_succeeded": all(x == vccl.vcclSuccess for x in st + st2)}
        del served, rbufs
    finally:
        for c in comms:
            vccl.vcclCommDestroy(c)
    return out


# The oracle's inputs for the CPU baseline, set before the worker processes
# fork (and before the GPU is initialised), so every worker holds them.
_CPU = {}


def _cpu_channel(task):
    """One channel of the ring AllReduce through the oracle's step simulation
    (channels are independent: the simulation of channel c's slice with one
    channel is the channel's part of the whole simulation)."""
    from oracle import simulate as sim
    c, a, b, chunk_bytes = task
    out = sim.run("allreduce", [x[a:b] for x in _CPU["xs"]], dtype="float32", nchannels=1, chunk_bytes=chunk_bytes)
    return c, out[0]


def cpu_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def cpu_baseline_leg(pool, nworkers, xs, plan, R, S, seconds, gpu_out):
    """The oracle timed on the host: the step simulation of the same ring
    AllReduce (inputs, plan) on one thread, then its channels spread over
    `nworkers` processes; the all-process result is checked element by
    element against the GPU's output, and so is the oracle's closed-form
    fold."""
    import numpy as np
    from oracle import folds
    from oracle import partition as pt
    from oracle import simulate as sim
    n = len(xs[0])
    C, chunk = plan["nchannels"], plan["chunkBytes"]
    exact_fold = bool(np.array_equal(gpu_out.view(np.uint32),
                                     folds.ring_allreduce(xs, "sum", "float32", C, chunk // 4).view(np.uint32)))
    reps1, t1, t0 = 0, 0.0, time.perf_counter()
    while reps1 < 1 or time.perf_counter() - t0 < seconds / 2:
        a = time.perf_counter()
        sim.run("allreduce", xs, dtype="float32", nchannels=C, chunk_bytes=chunk)
        t1 += time.perf_counter() - a
        reps1 += 1
    tasks = [(c, a, b, chunk) for c, (a, b) in enumerate(pt.channel_ranges(n, C, pt.align_units("allreduce", 4)))
             if b > a]
    repsN, tN, t0 = 0, 0.0, time.perf_counter()
    got = None
    while repsN < 1 or time.perf_counter() - t0 < seconds / 2:
        a = time.perf_counter()
        parts = dict(pool.map(_cpu_channel, tasks, chunksize=1))
        tN += time.perf_counter() - a
        repsN += 1
        got = parts
    out = np.concatenate([got[c] for c, _, _, _ in tasks])
    exact_sim = bool(np.array_equal(out.view(np.uint32), gpu_out.view(np.uint32)))
    bus = 2 * (R - 1) / R
    single = S / (t1 / reps1) / 1e9 * bus
    allc = S / (tN / repsN) / 1e9 * bus
    info = cpu_info()
    return {"value": round(allc, 4), "unit": "GB/s", "cores": nworkers, "kind": "oracle",
            "sample": f"the full workload ({R} ranks x {S >> 20} MiB fp32, the timed launch's plan: {C} channels, "
                      f"{chunk} B chunks) through the oracle's step simulation (numpy): {repsN} repetitions with "
                      f"its channels over {nworkers} processes ({tN:.1f} s), {reps1} on one thread ({t1:.1f} s)",
            "single_thread": {"value": round(single, 4), "unit": "GB/s", "cores": 1},
            **info,
            "gpu_result_bit_exact_all_elements": {"step_simulation": exact_sim, "closed_form_fold": exact_fold}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--size-mib", type=int, default=64)
    ap.add_argument("--nranks", type=int, default=8)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-protocols", action="store_true")
    ap.add_argument("--no-grouped", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-collectives", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=2000, help="measured requests per arrival rate")
    ap.add_argument("--serve-warmup", type=int, default=200, help="requests per rate before measurement")
    ap.add_argument("--serve-rates", default="1000,2000,5000,10000,20000,50000,100000")
    ap.add_argument("--serve-lanes", default="32,64",
                    help="lanes of the server; the first gives 'serving', each further one 'serving_lanes<L>'")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--profile-workload", default="headline", choices=("headline", "ll", "ll128", "tree16"),
                    help="with --profile-pass: the headline AllReduce, the same forced to LL or LL128, or the "
                         "16-rank bf16 64 MiB tree AllReduce")
    ap.add_argument("--profile-pass", action="store_true",
                    help="for rocprofv3 counter runs: 3 plain 1 GiB device copies (calibration), "
                         "then `steps` AllReduces of the workload; prints nothing else")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: vccl runs all its virtual ranks on one GPU; "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    import synthetic_inputs as si

    R = args.nranks
    n = args.size_mib * (1 << 20) // 4
    S = n * 4
    xs = si.rank_inputs(si.WL_RING_AR_SWEEP, R, "float32", n)
    # the CPU baseline's worker processes fork now, before the GPU is
    # initialised, each holding the inputs; at most 16 (the host share of one GPU)
    pool, nworkers = None, 0
    if not args.no_cpu and not args.profile_pass:
        import multiprocessing
        _CPU["xs"] = xs
        nworkers = max(1, min(16, cpu_info()["usable_cpus"] or 1))
        pool = multiprocessing.get_context("fork").Pool(nworkers)

    import torch

    import paper_2507_04786_amd as vccl

    torch.cuda.set_device(0)
    sends = [torch.from_numpy(x).cuda() for x in xs]
    recvs = [torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(R)]
    comms = vccl.vcclCommInitAll(R)
    stream = torch.cuda.current_stream()

    def step():
        for r in range(R):
            vccl.vcclAllReduce(sends[r], recvs[r], n, vccl.vcclFloat32, vccl.vcclSum, comms[r], stream)

    def measure(steps, warmup):
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        err = vccl.vcclCommGetAsyncError(comms[0])
        if err != vccl.vcclSuccess:
            raise RuntimeError(f"device error {vccl.vcclGetErrorString(err)}")
        return wall / steps, e0.elapsed_time(e1) / 1e3 / steps

    if args.profile_pass:
        # a plain copy kernel of known size: its FETCH_SIZE / WRITE_SIZE readings
        # scale the counters of the collective kernel to bytes
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        wl = args.profile_workload
        if wl in ("ll", "ll128"):
            vccl.vcclCommSetTuning(comms[0], algo=vccl.vcclAlgoRing, proto=vccl.PROTO_NAMES[wl])
        if wl == "tree16":
            for c in comms:
                vccl.vcclCommDestroy(c)
            R16, S16 = 16, 64 << 20
            xb = si.rank_inputs(si.WL_TREE_AND_CHAINS, R16, "bfloat16", S16 // 2)
            sends = [torch.from_numpy(x.view(np.int16)).cuda() for x in xb]
            recvs = [torch.empty(S16 // 2, dtype=torch.int16, device="cuda") for _ in range(R16)]
            comms = vccl.vcclCommInitAll(R16)
            vccl.vcclCommSetTuning(comms[0], algo=vccl.vcclAlgoTree)

            def step():
                for r in range(R16):
                    vccl.vcclAllReduce(sends[r], recvs[r], S16 // 2, vccl.vcclBfloat16, vccl.vcclSum, comms[r],
                                       stream)
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        plan = vccl.vcclCommGetLastPlan(comms[0])
        for c in comms:
            vccl.vcclCommDestroy(c)
        print(json.dumps({"profile_pass": True, "workload": wl, "plan": plan, "copy_bytes": 2 * (1 << 30)}))
        return

    # headline: tuner's plan
    wall_step, ev_step = measure(args.steps, args.warmup)
    plan = vccl.vcclCommGetLastPlan(comms[0])
    # Section V-F's statistic: each of `steps` launches after the warm-up
    # timed on its own (events on the launch stream), median / min / max
    per_launch = []
    for _ in range(args.steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        step()
        e1.record(stream)
        torch.cuda.synchronize()
        per_launch.append(e0.elapsed_time(e1))
    launch_stats = {"runs": len(per_launch), "median_ms": round(float(np.median(per_launch)), 4),
                    "min_ms": round(float(np.min(per_launch)), 4), "max_ms": round(float(np.max(per_launch)), 4),
                    "busbw_at_median_gbs": round(S / (float(np.median(per_launch)) / 1e3) / 1e9 * 2 * (R - 1) / R, 2)}
    algbw = S / wall_step / 1e9
    busbw = algbw * 2 * (R - 1) / R
    abytes = alg_bytes_per_launch(plan, R, S)
    achieved = abytes / ev_step / 1e9
    key = f"collKernel_ring_allreduce_r{R}_{args.size_mib}MiB_fp32"
    traffic = load_traffic(key)
    progress(f"headline done: {ev_step * 1e3:.4f} ms per launch")

    protos = {}
    sizes = None
    large = None
    if not args.no_protocols:
        for name, code in (("simple", vccl.vcclProtoSimple), ("ll", vccl.vcclProtoLL), ("ll128", vccl.vcclProtoLL128)):
            vccl.vcclCommSetTuning(comms[0], algo=vccl.vcclAlgoRing, proto=code)
            w, e = measure(max(3, args.steps // 2), 2)
            p = vccl.vcclCommGetLastPlan(comms[0])
            b = alg_bytes_per_launch(p, R, S)
            protos[name] = {"busbw_gbs": round(S / w / 1e9 * 2 * (R - 1) / R, 2),
                            "hbm_frac": round(b / e / 1e9 / HBM_PEAK_GBS, 4),
                            "ms": round(e * 1e3, 4), "nchannels": p["nchannels"], "chunk_bytes": p["chunkBytes"],
                            "direct": p["direct"]}
        vccl.vcclCommSetTuning(comms[0])
        progress("protocols done")
        sizes = sizes_leg(vccl, torch, comms, sends, recvs, stream)
        large = large_leg(vccl, torch, comms, sends, stream)
        progress("sizes done")

    cpu = None
    if not args.no_cpu:
        # the launch whose result the CPU leg checks: one more of the timed
        # plan, every element compared
        step()
        torch.cuda.synchronize()
        gpu_out = recvs[0].cpu().numpy()
        cpu = cpu_baseline_leg(pool, nworkers, xs, plan, R, S, args.cpu_seconds, gpu_out)
        del gpu_out
        progress("cpu baseline done")

    grouped = None
    if not args.no_grouped:
        grouped = grouped_leg(vccl, torch, si, comms, stream)
        progress("grouped done")
    for c in comms:
        vccl.vcclCommDestroy(c)
    del sends, recvs
    colls16 = None
    a2a = None
    if not args.no_collectives:
        colls16 = collectives_leg(vccl, torch, si)
        a2a = alltoall_leg(vccl, torch, si)
        progress("16-rank collectives and all-to-all done")
    serving, serving_more = None, {}
    if not args.no_serving:
        rates = [float(x) for x in args.serve_rates.split(",") if x]
        lane_counts = [int(x) for x in args.serve_lanes.split(",") if x]
        for i, L in enumerate(lane_counts):
            res = serving_leg(vccl, torch, si, R, rates, args.serve_requests, args.serve_warmup, lanes=L)
            progress(f"serving with {L} lanes done")
            if i == 0:
                serving = res
            else:
                serving_more[f"serving_lanes{L}"] = res

    out = {
        "metric": METRIC,
        "value": round(busbw, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall_step * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"ring AllReduce sum, {R} virtual ranks, fp32 N(0,1), {args.size_mib} MiB per rank",
                   "nranks": R, "bytes_per_rank": S, "algo": ["ring", "tree"][plan["algo"]],
                   "proto": ["simple", "ll", "ll128"][plan["proto"]], "nchannels": plan["nchannels"],
                   "chunk_bytes": plan["chunkBytes"], "nthreads": plan["nthreads"], "direct": plan["direct"]},
        "per_launch": launch_stats,
        "algbw_gbs": round(algbw, 2),
        "hbm_frac": round(achieved / HBM_PEAK_GBS, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic / ev_step / 1e9, 1),
                     "kernel": "vccl::collKernel", "alg_bytes_per_launch": abytes,
                     "avg_launch_ms": round(ev_step * 1e3, 4),
                     # the bytes no schedule can avoid (every input read and
                     # every output written once, 2 R S) per launch time
                     "compulsory_frac": round(2 * R * S / ev_step / 1e9 / HBM_PEAK_GBS, 4)},
        "protocols": protos,
        "sizes": sizes,
        "large_sizes": large,
        "collectives_r16": colls16,
        "alltoall": a2a,
        "grouped": grouped,
        "serving": serving,
        **serving_more,
        "cpu_baseline": cpu,
    }
    if pool is not None:
        pool.close()
        pool.join()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
