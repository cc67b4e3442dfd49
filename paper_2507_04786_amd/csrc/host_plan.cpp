// Planning: algorithm / protocol / channel / chunk choice per collective
// (Section II-C: after the algorithm and protocol, the tuning model picks how
// many of the channels built at init to use; Section III-D: LL/LL128 for
// small messages, Simple for large ones), and the channel partition with
// its loops and chunks (Section V-C).
#include <algorithm>
#include <cmath>

#include "host_internal.h"

namespace vccl {

size_t dtypeBytes(int dtype) { return dtype == vcclBfloat16 ? 2 : 4; }

// Message size in the nccl-tests convention: the larger per-rank buffer.
uint64_t collSizeBytes(uint8_t coll, size_t count, int dtype, int nranks) {
  const uint64_t b = (uint64_t)count * dtypeBytes(dtype);
  if (coll == COLL_SENDRECV) return b;
  if (coll == COLL_ALLGATHER || coll == COLL_REDUCESCATTER) return b * (uint64_t)nranks;
  return b;
}

static uint64_t ceilDiv(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
static uint64_t roundUp(uint64_t a, uint64_t b) { return ceilDiv(a, b) * b; }

// Copies (AllGather, Broadcast, point-to-point) are partitioned in bytes.
static bool copyOnly(uint8_t coll) {
  return coll == COLL_ALLGATHER || coll == COLL_BROADCAST || coll == COLL_SENDRECV;
}

static uint64_t unitBytesOf(uint8_t coll, int dtype) { return copyOnly(coll) ? 1 : dtypeBytes(dtype); }

static uint64_t unitsOf(uint8_t coll, size_t count, int dtype) {
  return copyOnly(coll) ? (uint64_t)count * dtypeBytes(dtype) : (uint64_t)count;
}

// Largest chunk one slot of the algorithm's connections can carry per
// protocol (slot payload): the whole slot under Simple, half of it under LL
// (4 data bytes per 8-byte unit), 120 of every 128 bytes under LL128.
static uint64_t maxChunkBytes(const Clique* c, int proto, int algo = ALGO_RING) {
  const uint64_t slot = algo == ALGO_TREE ? c->host.treeSlotBytes[proto] : c->host.slotBytes[proto];
  if (proto == PROTO_SIMPLE) return slot;
  if (proto == PROTO_LL) return slot / 2;
  return slot / LL128_LINE * LL128_DATA;
}

// Measured plan table: for each (ranks, collective, log2 of the per-rank
// size) the fastest (algorithm, protocol, channels, chunk, threads) of a
// sweep over all of them on this chip (fewest channels among plans within
// 10 % of the best below 16 MiB, within 3 % from 16 MiB up).  chunkKiB and
// nthreads hold what the measured plan ran with (Simple chunks and workgroup
// sizes from 1 MiB, LL / LL128 workgroup sizes from 64 KiB); 0: the formulas
// below.
struct TuneEntry {
  int nranks, coll, log2, algo, proto, nchannels, chunkKiB, nthreads;
  float us;
};
// One table for collectives launched alone and in groups: another plan in a
// group would change a float reduction's order, and so its bits.
static const TuneEntry kTuneTable[] = {
#include "tune_table.inc"
};

// Entry for the measured rank count nearest to R (4, 8 or 16) and the size
// bucket nearest to S on a log scale.
static const TuneEntry* tuneLookup(int R, uint8_t coll, uint64_t S) {
  const int tr = R <= 5 ? 4 : (R <= 11 ? 8 : 16);
  const int lg = S <= 8 ? 3 : (int)std::lround(std::log2((double)S));
  const TuneEntry* best = nullptr;
  int bestDist = 1 << 30;
  for (const TuneEntry& e : kTuneTable) {
    if (e.nranks != tr || e.coll != coll) continue;
    const int dist = std::abs(e.log2 - lg);
    if (dist < bestDist) {
      bestDist = dist;
      best = &e;
    }
  }
  return best;
}

void channelRange(uint64_t n, int nchannels, uint64_t align, int ch, uint64_t* start, uint64_t* count) {
  const uint64_t per = n ? roundUp(ceilDiv(n, (uint64_t)nchannels), align) : 0;
  const uint64_t s = std::min(n, (uint64_t)ch * per);
  const uint64_t e = std::min(n, (uint64_t)(ch + 1) * per);
  *start = s;
  *count = e - s;
}

// Lanes point-to-point copies spread over: one workgroup per CU (at least
// 32 lanes): copies have no waits to hide, and at 8 ranks 64 lanes (two
// workgroups per CU) made the all-to-all 25 % slower than 32.
int p2pLaneCap(const Clique* c) {
  return std::max(1, std::min(c->maxLanes, std::max(32, c->numCUs / c->nranks)));
}

// Point-to-point transfer (Section II-A Send/Recv; Section II-C: grouped
// transfers spread over channels; Section IV-A: P2P_DIRECT): a direct copy
// into the receiver's buffer, a channel per 1 MiB up to the lane cap, every
// workgroup of a lane copying 1/R of each channel, slot-sized pieces.  Only
// the channel count, threads and chunk follow an explicit tuning.
static vcclResult_t planP2p(Clique* c, const Coll& coll, Plan* plan) {
  const int R = c->nranks;
  const uint64_t S = (uint64_t)coll.count * dtypeBytes(coll.dtype);
  auto pickPos = [&](long api, long env, long dflt) { return api > 0 ? api : (env > 0 ? env : dflt); };
  const int laneCap = p2pLaneCap(c);
  const long dfltC = (long)std::min<uint64_t>((uint64_t)laneCap, std::max<uint64_t>(1, ceilDiv(S, 1u << 20)));
  int nch = (int)pickPos(c->apiTune.nchannels, c->envTune.nchannels, dfltC);
  nch = std::max(1, std::min(nch, c->maxLanes));
  int nthreads = (int)pickPos(c->apiTune.nthreads, c->envTune.nthreads, 256);
  nthreads = std::max(64, std::min(1024, nthreads / 64 * 64));
  const int occ = cliqueOccupancy(c, nthreads);
  if (occ <= 0) return vcclInternalError;
  while (nch > 1 && 8 * R * (int)ceilDiv(nch, 8) > c->numCUs * occ) --nch;
  uint64_t chunk = c->apiTune.chunkBytes ? c->apiTune.chunkBytes
                                         : (c->envTune.chunkBytes ? c->envTune.chunkBytes : maxChunkBytes(c, PROTO_SIMPLE));
  chunk = std::max<uint64_t>(16, std::min(chunk, maxChunkBytes(c, PROTO_SIMPLE)) / 16 * 16);
  plan->algo = ALGO_RING;
  plan->proto = PROTO_SIMPLE;
  plan->nchannels = nch;
  plan->nthreads = nthreads;
  plan->direct = 1;
  plan->chunkBytes = chunk;
  plan->scope = (c->host.scope == SCOPE_XCD && S < c->deviceScopeBytes) ? SCOPE_XCD : SCOPE_DEVICE;
  return vcclSuccess;
}

vcclResult_t planColl(Clique* c, const Coll& coll, Plan* plan, bool single) {
  if (coll.coll == COLL_SENDRECV) return planP2p(c, coll, plan);
  const int R = c->nranks;
  const uint64_t S = collSizeBytes(coll.coll, coll.count, coll.dtype, R);
  auto pick = [&](int api, int env, int dflt) { return api >= 0 ? api : (env >= 0 ? env : dflt); };
  auto pickPos = [&](long api, long env, long dflt) { return api > 0 ? api : (env > 0 ? env : dflt); };

  // --- defaults from the measured table (Section III-D: LL / LL128 for small
  // messages, Simple for large ones; Section V-F: tree for small AllReduce,
  // ring for large)
  const TuneEntry* te = tuneLookup(R, coll.coll, S);
  int dfltAlgo = te ? te->algo : ALGO_RING;
  if (coll.coll != COLL_ALLREDUCE || R < 4) dfltAlgo = ALGO_RING;
  const int dfltProto = te ? te->proto : (S <= (1u << 20) ? PROTO_LL : PROTO_SIMPLE);
  // --- algorithm (Tree exists for AllReduce only; a forced tree elsewhere
  // falls back to the ring)
  int algo = pick(c->apiTune.algo, c->envTune.algo, dfltAlgo);
  if (algo == ALGO_TREE && coll.coll != COLL_ALLREDUCE) algo = ALGO_RING;
  int proto = pick(c->apiTune.proto, c->envTune.proto, dfltProto);
  // Section III-C: where LL128's lines are not guaranteed whole (the tear
  // test failed, or VCCL_LL128=0) every LL128 plan, chosen or requested,
  // becomes LL, the other flag protocol
  if (proto == PROTO_LL128 && !c->ll128) proto = PROTO_LL;
  // --- channels: up to two workgroups per CU (while one waits on a flag the
  // other moves data)
  const int laneCap = std::max(1, std::min(c->maxLanes, 2 * c->numCUs / R));
  long dfltC = te ? te->nchannels : (long)std::max<uint64_t>(1, std::min<uint64_t>(laneCap, S / (512 * 1024)));
  // a flag protocol asked for where the table's plan is Simple, at 16 MiB and
  // more: every lane (LL's lines in flight scale with the workgroups; at 8
  // ranks and 64 MiB, 64 lanes of 512 threads beat 32 of 1024 by 7 %); the
  // co-residency rule below trims it to what fits (LL128's 1024-thread
  // workgroups: one per CU)
  if (te && te->proto == PROTO_SIMPLE && proto != PROTO_SIMPLE && S >= (16u << 20)) dfltC = laneCap;
  dfltC = std::max(1L, std::min<long>(dfltC, laneCap));
  int nch = (int)pickPos(c->apiTune.nchannels, c->envTune.nchannels, dfltC);
  nch = std::max(1, std::min(nch, c->maxLanes));
  // --- a Simple tree launched alone runs each channel as two concurrent
  // halves (reduce-up and broadcast-down) on two lanes of one XCD: channel
  // ch's up half on lane ch, its down half on lane 8 ceil(C / 8) + ch, so C
  // channels take 8 ceil(C / 8) + C of the set's lanes
  bool split = single && c->treeSplit && c->xcdMap && algo == ALGO_TREE && proto == PROTO_SIMPLE;
  if (split) {
    int cap = 0;
    while (cap < 32 && 8 * (int)ceilDiv(cap + 1, 8) + cap + 1 <= c->maxLanes) ++cap;
    if (cap == 0) split = false;  // not even one channel's pair of lanes fits
    else nch = std::min(nch, cap);
  }
  // --- workgroup size
  long dfltT = (S >= (256u << 10)) ? 512 : 256;
  // LL128 receives are bound by the lines in flight: from 16 MiB, 1024
  // threads measured 20-30 % faster than 512 (and slower below)
  if (proto == PROTO_LL128 && S >= (16u << 20)) dfltT = 1024;
  if (proto == PROTO_SIMPLE) dfltT = 256;
  // the table's workgroup size, for a collective launched alone (a group runs
  // every item at the largest formula size among its plans, measured faster
  // than the table's; the size never changes a result's bits)
  if (single && te && te->nthreads > 0 && te->algo == algo && te->proto == proto) dfltT = te->nthreads;
  int nthreads = (int)pickPos(c->apiTune.nthreads, c->envTune.nthreads, dfltT);
  nthreads = std::max(64, std::min(1024, nthreads / 64 * 64));
  // co-residency: every workgroup of the launch must be resident at once
  const int occ = cliqueOccupancy(c, nthreads);
  if (occ <= 0) return vcclInternalError;
  if (c->xcdMap) {
    // the XCD map launches 8 * R * ceil(L / 8) workgroups
    while (nch > 1 && 8 * R * (int)ceilDiv(nch, 8) > c->numCUs * occ) --nch;
    // a split tree takes 8 ceil(C / 8) + C lanes
    if (split && 8 * R * (int)ceilDiv(8 * ceilDiv(nch, 8) + nch, 8) > c->numCUs * occ) split = false;
  } else {
    nch = std::min(nch, std::max(1, (c->numCUs * occ) / R));
  }
  // --- chunk
  const uint64_t maxChunk = maxChunkBytes(c, proto, algo);
  uint64_t chunk;
  if (c->apiTune.chunkBytes) chunk = c->apiTune.chunkBytes;
  else if (c->envTune.chunkBytes) chunk = c->envTune.chunkBytes;
  else if (te && te->chunkKiB > 0 && te->algo == algo && te->proto == proto)
    chunk = (uint64_t)te->chunkKiB * 1024;
  else {
    if (proto == PROTO_SIMPLE && algo == ALGO_TREE) {
      // a tree pipelines chunks through 2 log2(R) hops: eight chunks per
      // channel, at most 64 KiB (16 ranks, bf16, 64 MiB, split halves of 16
      // channels x 256 threads: 1.32 ms at 64 KiB against 1.40 ms at the
      // 128 KiB slot)
      const uint64_t chBytes = ceilDiv(S, (uint64_t)nch);
      chunk = std::min<uint64_t>(roundUp(std::max<uint64_t>(ceilDiv(chBytes, 8), 16 * 1024), 4096),
                                 std::min<uint64_t>(maxChunk, 64 * 1024));
    } else if (proto == PROTO_SIMPLE) {
      // a ring loop covers R chunks: take the largest chunk that still gives
      // every channel at least one full loop
      const uint64_t chBytes = ceilDiv(S, (uint64_t)nch);
      chunk = roundUp(std::max<uint64_t>(ceilDiv(chBytes, (uint64_t)R), 16 * 1024), 4096);
      chunk = std::min<uint64_t>(chunk, 128 * 1024);  // measured best for large rings
    } else {
      chunk = maxChunk;
    }
  }
  chunk = std::min(chunk, maxChunk) / 16 * 16;
  if (chunk < 16) chunk = 16;
  int direct = pick(c->apiTune.direct, c->envTune.direct, 1);
  if (proto != PROTO_SIMPLE) direct = 0;
  plan->algo = algo;
  plan->proto = proto;
  plan->nchannels = nch;
  plan->nthreads = nthreads;
  plan->direct = direct;
  plan->chunkBytes = chunk;
  // halves pay off once a channel pipelines at least two chunks
  plan->split = split && ceilDiv(ceilDiv(S, (uint64_t)nch), chunk) >= 2;
  // store policy: XCD scope (lower latency; data a chain forwards is read
  // back from the XCD's L2) except for a large Simple AllGather, the one
  // collective measured faster with write-through stores there
  const bool devScope = proto == PROTO_SIMPLE && coll.coll == COLL_ALLGATHER && S >= c->deviceScopeBytes;
  plan->scope = (c->host.scope == SCOPE_XCD && !devScope) ? SCOPE_XCD : SCOPE_DEVICE;
  return vcclSuccess;
}

void fillItems(const Clique* c, const Coll& coll, const Plan& plan, uint32_t argsIndex, uint32_t doneIndex,
               std::vector<WorkItem>* items) {
  const uint64_t ub = unitBytesOf(coll.coll, coll.dtype);
  const uint64_t n = unitsOf(coll.coll, coll.count, coll.dtype);
  const uint64_t align = 16 / ub;
  for (int ch = 0; ch < plan.nchannels; ++ch) {
    WorkItem w{};
    w.coll = coll.coll;
    w.algo = (uint8_t)plan.algo;
    w.proto = (uint8_t)plan.proto;
    const bool copy = copyOnly(coll.coll);
    w.dtype = copy ? DT_U8 : (uint8_t)(coll.dtype == vcclInt32 ? DT_I32 : coll.dtype == vcclFloat32 ? DT_F32 : DT_BF16);
    w.op = copy ? OP_COPY : (uint8_t)(coll.op == vcclMax ? OP_MAX : OP_SUM);
    w.direct = (uint8_t)plan.direct;
    w.tree = (uint8_t)(ch % 2);
    // ring collectives: channel ch follows ring ch % nrings wherever (on
    // whichever lane) it runs, so grouping keeps the per-call bits
    w.ring = (uint8_t)(plan.algo == ALGO_RING && coll.coll != COLL_SENDRECV ? ch % c->nrings : 0);
    w.peer = (uint8_t)coll.peer;
    w.root = coll.root;
    w.argsIndex = argsIndex;
    w.doneIndex = doneIndex;
    w.unitBytes = (uint32_t)ub;
    w.elemBytes = (uint32_t)(copy ? 1 : dtypeBytes(coll.dtype));
    w.scope = (uint8_t)plan.scope;
    w.count = n;
    channelRange(n, plan.nchannels, align, ch, &w.chOffset, &w.chCount);
    w.chunk = plan.chunkBytes / ub;
    items->push_back(w);
  }
}

// Rough time (us) of one work item, used to balance lanes in grouped launches.
double estimateCost(const Clique* c, const WorkItem& w) {
  const int R = c->nranks;
  const double bytes = (double)w.chCount * w.unitBytes;
  const double fifo = w.proto == PROTO_SIMPLE ? 1.0 : (w.proto == PROTO_LL ? 2.0 : 16.0 / 15.0);
  // measured per-step cost of a ring step (µs) per protocol
  const double lat = w.proto == PROTO_SIMPLE ? 1.4 : (w.proto == PROTO_LL ? 0.7 : 0.8);
  double steps, traffic;
  if (w.coll == COLL_ALLREDUCE) {
    steps = w.algo == ALGO_TREE ? 2.0 * std::ceil(bytes / std::max<double>(1.0, (double)w.chunk * w.unitBytes))
                                : (2.0 * R - 1) * std::ceil(bytes / std::max<double>(1.0, (double)R * w.chunk * w.unitBytes));
    traffic = (2.0 * R + 4.0 * fifo * (R - 1)) * bytes / R;
  } else if (w.coll == COLL_ALLGATHER || w.coll == COLL_REDUCESCATTER) {
    steps = (double)R * std::ceil(bytes / std::max<double>(1.0, (double)w.chunk * w.unitBytes));
    traffic = (R + 1.0 + 2.0 * fifo * (R - 1)) * bytes;
  } else if (w.coll == COLL_SENDRECV) {
    // a read and a direct write per byte, shared by the lane's workgroups
    steps = std::ceil(bytes / std::max<double>(1.0, (double)R * w.chunk * w.unitBytes));
    traffic = 2.0 * bytes;
  } else {
    steps = std::ceil(bytes / std::max<double>(1.0, (double)w.chunk * w.unitBytes)) + R;
    traffic = (R + 1.0 + 2.0 * fifo * (R - 1)) * bytes;
  }
  // bytes per µs one lane moves, all its ranks together, while every lane is
  // busy: about 6 TB/s of traffic shared by 32 lanes
  const double laneBW = 180e3;
  return steps * lat + traffic / laneBW;
}

}  // namespace vccl
