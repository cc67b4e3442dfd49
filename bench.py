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
              several arrival rates: p50 / p99 latency, offered vs achieved rate
  cpu_baseline the CPU oracle (numpy schedule simulation) on the same inputs
              and plan, and a spot check of the timed launch's result
              against the oracle's fold (4096 samples, bit for bit)

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--size-mib 64]
                       [--no-cpu] [--no-protocols] [--no-grouped] [--no-serving]
                       [--no-collectives]
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
                         "nchannels": plan["nchannels"], "direct": plan["direct"]}
    finally:
        vccl.vcclCommSetTuning(comms[0])
        for c in comms:
            vccl.vcclCommDestroy(c)
    return out


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


def grouped_leg(vccl, torch, si, comms, stream, reps=10):
    """64 collectives issued in one group against 64 separate launches:
    time between events on the launch stream around the issue (the host's
    issue and planning included, as a caller sees it), host wall time, and
    the device's own time with the launches queued behind a spin kernel."""
    import numpy as np
    R = len(comms)
    arenas = _send_arenas(torch, si, si.WL_GROUPED, R, 16 << 20)
    codes = {"float32": vccl.vcclFloat32, "bfloat16": vccl.vcclBfloat16, "int32": vccl.vcclInt32}
    result = {}
    for name, lo, hi in (("mixed_4KiB_16MiB", 4 << 10, 16 << 20), ("sub_1MiB", 4 << 10, 1 << 20)):
        specs = _batch_specs(si, 1, 64, lo, hi, R)
        recvs = []
        for coll, dt, n in specs:
            rl = n * R if coll == "allgather" else n
            recvs.append([torch.empty(rl * ELEM[dt], dtype=torch.uint8, device="cuda") for _ in range(R)])

        def issue(group):
            if group:
                vccl.vcclGroupStart()
            for k, (coll, dt, n) in enumerate(specs):
                for r in range(R):
                    s, d = arenas[dt][r], recvs[k][r]
                    if coll == "allreduce":
                        vccl.vcclAllReduce(s, d, n, codes[dt], vccl.vcclSum, comms[r], stream)
                    elif coll == "allgather":
                        vccl.vcclAllGather(s, d, n, codes[dt], comms[r], stream)
                    else:
                        vccl.vcclReduceScatter(s, d, n, codes[dt], vccl.vcclSum, comms[r], stream)
            if group:
                vccl.vcclGroupEnd()

        def timed(group):
            issue(group)
            torch.cuda.synchronize()
            dev, wall = [], []
            for _ in range(reps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                t0 = time.perf_counter()
                e0.record(stream)
                issue(group)
                e1.record(stream)
                torch.cuda.synchronize()
                wall.append(time.perf_counter() - t0)
                dev.append(e0.elapsed_time(e1) / 1e3)
            return float(np.median(dev)), float(np.median(wall))

        def device_only(group):
            # the launches queued behind a spin kernel (about 3 ms) that keeps
            # the device busy while the host issues and plans them, so the
            # events bracket device work only
            spin = getattr(torch.cuda, "_sleep", None)
            if spin is None:
                return None
            dev = []
            for _ in range(reps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                spin(2_000_000)
                e0.record(stream)
                issue(group)
                e1.record(stream)
                torch.cuda.synchronize()
                dev.append(e0.elapsed_time(e1) / 1e3)
            return float(np.median(dev))

        pc_dev, pc_wall = timed(False)
        pc_only = device_only(False)
        snap = [[x.clone() for x in rr] for rr in recvs]
        for rr in recvs:
            for x in rr:
                x.fill_(0x5A)
        g_dev, g_wall = timed(True)
        g_only = device_only(True)
        plan = vccl.vcclCommGetLastPlan(comms[0])
        same = all(bool(torch.equal(a, b)) for ra, rb in zip(snap, recvs) for a, b in zip(ra, rb))
        err = vccl.vcclCommGetAsyncError(comms[0])
        if err != vccl.vcclSuccess:
            raise RuntimeError(f"device error {vccl.vcclGetErrorString(err)} in grouped leg")
        sizes = [n * ELEM[dt] * (R if c != "allreduce" else 1) for c, dt, n in specs]
        result[name] = {"ncolls": len(specs), "bytes_total": int(sum(sizes)),
                        "sub_1MiB_fraction": round(float(np.mean([x < (1 << 20) for x in sizes])), 3),
                        "grouped_ms": round(g_dev * 1e3, 4), "per_call_ms": round(pc_dev * 1e3, 4),
                        "grouped_wall_ms": round(g_wall * 1e3, 4), "per_call_wall_ms": round(pc_wall * 1e3, 4),
                        "speedup": round(pc_dev / g_dev, 3),
                        "grouped_device_ms": None if g_only is None else round(g_only * 1e3, 4),
                        "per_call_device_ms": None if pc_only is None else round(pc_only * 1e3, 4),
                        "device_speedup": None if not (g_only and pc_only) else round(pc_only / g_only, 3),
                        "lanes": plan["nlanes"],
                        "grouped_equals_per_call": same}
        del recvs, snap
    return result


def serving_leg(vccl, torch, si, R, rates, nreq, nwarm, lanes=32, budget=4 << 30):
    """Poisson request streams through the continuous-batching server."""
    import numpy as np
    arena = 128 << 20
    arenas = _send_arenas(torch, si, si.WL_SERVING, R, arena)
    recv = [torch.empty(arena, dtype=torch.uint8, device="cuda") for _ in range(R)]
    base_s = {dt: [t.data_ptr() for t in arenas[dt]] for dt in DTYPES}
    base_r = [t.data_ptr() for t in recv]
    codes = {"float32": vccl.vcclFloat32, "bfloat16": vccl.vcclBfloat16, "int32": vccl.vcclInt32}
    comms = vccl.vcclCommInitAll(R)
    torch.cuda.synchronize()
    srv = vccl.vcclServeCreate(comms, budget, lanes)
    out = {"lanes": lanes, "budget_bytes": budget, "requests_per_rate": nreq, "warmup_per_rate": nwarm,
           "rates": []}
    try:
        for k, lam in enumerate(rates):
            rng = si.rng_for(si.WL_SERVING, 0, 100 + k)
            total = nreq + nwarm
            sizes = si.log_uniform_sizes(rng, total, 1 << 10, 128 << 20)
            reqs, nbytes = [], 0
            for i in range(total):
                u = rng.uniform()
                coll = "allreduce" if u < 0.6 else ("allgather" if u < 0.8 else "reducescatter")
                dt = DTYPES[int(rng.integers(0, 3))]
                E = ELEM[dt]
                n = max(1, int(sizes[i]) // E // (R if coll != "allreduce" else 1))
                span_s = n * E * (R if coll == "reducescatter" else 1)
                span_r = n * E * (R if coll == "allgather" else 1)
                off_s = int(rng.integers(0, (arena - span_s) // 16 + 1)) * 16
                off_r = int(rng.integers(0, (arena - span_r) // 16 + 1)) * 16
                reqs.append(vccl.make_request(COLL_CODES[coll], codes[dt], vccl.vcclSum, 0, n,
                                              [b + off_s for b in base_s[dt]], [b + off_r for b in base_r]))
                nbytes += int(sizes[i])
            arr = si.poisson_arrivals(rng, total, lam)
            lat, st = vccl.vcclServeReplay(srv, reqs, (arr * 1e9).astype(np.int64))
            if any(x != vccl.vcclSuccess for x in st):
                raise RuntimeError("serving: a request failed")
            lat = np.asarray(lat[nwarm:], dtype=np.float64) / 1e3
            done = arr[nwarm:] + lat / 1e6
            span = float(done.max() - arr[nwarm])
            out["rates"].append({"offered_per_s": lam, "achieved_per_s": round(nreq / span, 1),
                                 "p50_us": round(float(np.percentile(lat, 50)), 1),
                                 "p99_us": round(float(np.percentile(lat, 99)), 1),
                                 "mean_bytes": int(nbytes / total)})
    finally:
        vccl.vcclServeDestroy(srv)
        for c in comms:
            vccl.vcclCommDestroy(c)
    return out


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
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--profile-pass", action="store_true",
                    help="for rocprofv3 counter runs: 3 plain 1 GiB device copies (calibration), "
                         "then `steps` AllReduces of the workload; prints nothing else")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: vccl runs all its virtual ranks on one GPU; "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2507_04786_amd as vccl
    import synthetic_inputs as si

    R = args.nranks
    n = args.size_mib * (1 << 20) // 4
    S = n * 4
    torch.cuda.set_device(0)
    xs = si.rank_inputs(si.WL_RING_AR_SWEEP, R, "float32", n)
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
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        plan = vccl.vcclCommGetLastPlan(comms[0])
        for c in comms:
            vccl.vcclCommDestroy(c)
        print(json.dumps({"profile_pass": True, "plan": plan, "copy_bytes": 2 * (1 << 30)}))
        return

    # headline: tuner's plan
    wall_step, ev_step = measure(args.steps, args.warmup)
    plan = vccl.vcclCommGetLastPlan(comms[0])
    algbw = S / wall_step / 1e9
    busbw = algbw * 2 * (R - 1) / R
    abytes = alg_bytes_per_launch(plan, R, S)
    achieved = abytes / ev_step / 1e9
    key = f"collKernel_ring_allreduce_r{R}_{args.size_mib}MiB_fp32"
    traffic = load_traffic(key)

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
        sizes = sizes_leg(vccl, torch, comms, sends, recvs, stream)
        large = large_leg(vccl, torch, comms, sends, stream)

    cpu = None
    if not args.no_cpu:
        # the CPU oracle leg: a spot check of the timed launch's result against
        # the oracle's fold, then the oracle's own timing
        from oracle import folds
        from oracle import simulate as sim
        rng = np.random.default_rng(7)
        idx = rng.integers(0, n, 4096)
        step()
        torch.cuda.synchronize()
        got = recvs[0].cpu().numpy()[idx]
        want = folds.ring_allreduce(xs, "sum", "float32", plan["nchannels"], plan["chunkBytes"] // 4, idx=idx)
        exact = bool(np.array_equal(got.view(np.uint32), want.view(np.uint32)))
        reps, t_cpu, t0 = 0, 0.0, time.perf_counter()
        while reps < 2 or time.perf_counter() - t0 < args.cpu_seconds:
            t1 = time.perf_counter()
            sim.run("allreduce", xs, dtype="float32", nchannels=plan["nchannels"], chunk_bytes=plan["chunkBytes"])
            t_cpu += time.perf_counter() - t1
            reps += 1
        per = t_cpu / reps
        cpu = {"value": round(S / per / 1e9 * 2 * (R - 1) / R, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"the full workload ({R} ranks x {args.size_mib} MiB fp32, same plan), {reps} repetitions, "
                         f"{t_cpu:.1f} s total, numpy single-threaded",
               "gpu_result_bit_exact_on_4096_samples": exact}

    grouped = None
    if not args.no_grouped:
        grouped = grouped_leg(vccl, torch, si, comms, stream)
    for c in comms:
        vccl.vcclCommDestroy(c)
    del sends, recvs
    colls16 = None
    a2a = None
    if not args.no_collectives:
        colls16 = collectives_leg(vccl, torch, si)
        a2a = alltoall_leg(vccl, torch, si)
    serving = None
    if not args.no_serving:
        rates = [float(x) for x in args.serve_rates.split(",") if x]
        serving = serving_leg(vccl, torch, si, R, rates, args.serve_requests, args.serve_warmup)

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
        "algbw_gbs": round(algbw, 2),
        "hbm_frac": round(achieved / HBM_PEAK_GBS, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic / ev_step / 1e9, 1),
                     "kernel": "vccl::collKernel", "alg_bytes_per_launch": abytes,
                     "avg_launch_ms": round(ev_step * 1e3, 4)},
        "protocols": protos,
        "sizes": sizes,
        "large_sizes": large,
        "collectives_r16": colls16,
        "alltoall": a2a,
        "grouped": grouped,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
