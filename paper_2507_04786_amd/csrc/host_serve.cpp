// Serving: continuous batching over one persistent kernel.
//
// Requests are admitted oldest first as soon as enough lanes are free and the
// in-flight bytes (request buffers plus the FIFOs of the lanes they hold) fit
// the budget; a request that does not fit lets younger ones pass for a bounded
// time.  Requests admitted while others run execute concurrently on their own
// lanes.  The plan of a request (protocol, channels, chunk) depends
// only on the request, never on the load, so a request gives the same bits
// alone and in a mix.
#include <time.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <deque>
#include <unordered_map>
#include <vector>

#include "host_internal.h"

using namespace vccl;

namespace {

uint64_t nowNs() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

struct Req {
  uint64_t id;
  vcclRequest_t r;
  Plan plan;
  uint64_t bytes;
  int nlanes;
  int lanes[MAX_LANES];
  uint64_t seqs[MAX_LANES];
  int state;  // 0 waiting, 1 in flight, 2 done
  uint64_t tSubmit, tDone;
  vcclResult_t status;
};

}  // namespace

struct vcclServer {
  Clique* c = nullptr;
  int L = 0;
  int block = 512;
  size_t budget = 0, used = 0;
  int maxLanesPerReq = 1;
  uint64_t fullPlanBytes = 0;
  uint64_t bypassNs = 0;
  hipStream_t stream = nullptr;
  ServeDesc desc{};
  int grid = 0;
  bool running = false;
  ServeEntry* hQueue = nullptr;
  uint64_t* hPosted = nullptr;
  uint64_t* hDone = nullptr;
  uint32_t* hStop = nullptr;
  uint64_t* hDbg = nullptr;
  ServeEntry* dMirror = nullptr;
  uint64_t* dLaneSeq = nullptr;
  uint64_t posted[MAX_LANES] = {0};
  bool laneBusy[MAX_LANES] = {false};
  std::deque<Req*> waiting;
  std::vector<Req*> inflight;
  std::unordered_map<uint64_t, Req*> reqs;
  uint64_t nextId = 1;
};

namespace {

// Releases everything a server holds (null-safe; the kernel has ended).
void freeServer(vcclServer* s) {
  if (s->stream) hipStreamDestroy(s->stream);
  for (auto& kv : s->reqs) delete kv.second;
  if (s->hQueue) hipHostFree(s->hQueue);
  if (s->hPosted) hipHostFree(s->hPosted);
  if (s->hDone) hipHostFree(s->hDone);
  if (s->hStop) hipHostFree(s->hStop);
  if (s->hDbg) hipHostFree(s->hDbg);
  if (s->dMirror) hipFree(s->dMirror);
  if (s->dLaneSeq) hipFree(s->dLaneSeq);
  delete s;
}

uint64_t laneDone(vcclServer* s, int lane) {
  uint64_t m = UINT64_MAX;
  for (int r = 0; r < s->c->nranks; ++r)
    m = std::min(m, __atomic_load_n(s->hDone + ((uint64_t)lane * s->c->nranks + r) * SERVE_STRIDE_U64,
                                    __ATOMIC_ACQUIRE));
  return m;
}

// Host words the persistent kernel polls: the stop word (host) and, 128 bytes
// further, the idle word (raised by the kernel).
constexpr int kIdleWord = 32;

bool kernelLeaving(vcclServer* s) {
  return __atomic_load_n(s->hStop, __ATOMIC_ACQUIRE) != 0 || __atomic_load_n(s->hStop + kIdleWord, __ATOMIC_ACQUIRE) != 0;
}

vcclResult_t launchKernel(vcclServer* s) {
  for (int l = 0; l < s->L; ++l) s->desc.startSeq[l] = laneDone(s, l);
  __atomic_store_n(s->hStop, 0u, __ATOMIC_RELEASE);
  __atomic_store_n(s->hStop + kIdleWord, 0u, __ATOMIC_RELEASE);
  // the release counters restart from zero: the previous kernel (same stream)
  // has ended, and the exit markers its leaders left must not reach this one
  hipError_t me = hipMemsetAsync(s->dLaneSeq, 0, sizeof(uint64_t) * SERVE_STRIDE_U64 * s->L, s->stream);
  if (me != hipSuccess) {
    logError("hipMemsetAsync(laneSeq)", me, __FILE__, __LINE__);
    return vcclUnhandledHipError;
  }
  s->desc.perXcd = (uint32_t)(s->c->nranks * ((s->L + 7) / 8));
  s->desc.claimBase = s->c->claimBase;
  hipError_t e = vcclLaunchServe(s->desc, s->grid, s->block, s->stream);
  if (e != hipSuccess) {
    logError("serve launch", e, __FILE__, __LINE__);
    return vcclUnhandledHipError;
  }
  if (s->c->xcdMap) s->c->claimBase += s->desc.perXcd;
  s->running = true;
  return vcclSuccess;
}

uint64_t requestBytes(const Clique* c, const vcclRequest_t& r, const Plan& p) {
  const int R = c->nranks;
  const uint64_t E = dtypeBytes(r.datatype);
  const uint64_t b = (uint64_t)r.count * E;
  uint64_t send = b, recv = b;
  if (r.coll == COLL_ALLGATHER) recv = b * R;
  if (r.coll == COLL_REDUCESCATTER) send = b * R;
  const uint64_t fifo = p.algo == ALGO_TREE ? (uint64_t)R * NTREE_CONN * NSLOTS * c->host.treeSlotBytes[p.proto]
                                            : (uint64_t)R * NSLOTS * c->host.slotBytes[p.proto];
  return (uint64_t)R * (send + recv) + (uint64_t)p.nchannels * fifo;
}

// Retire finished requests, then admit waiting ones in arrival order.
vcclResult_t progress(vcclServer* s) {
  Clique* c = s->c;
  const bool failed = __atomic_load_n(c->hError, __ATOMIC_ACQUIRE) != 0 || c->aborted;
  for (size_t i = 0; i < s->inflight.size();) {
    Req* q = s->inflight[i];
    bool done = true;
    for (int k = 0; k < q->nlanes && done; ++k) done = laneDone(s, q->lanes[k]) >= q->seqs[k] + 1;
    if (done || failed) {
      q->state = 2;
      q->tDone = nowNs();
      q->status = done ? vcclSuccess : vcclRemoteError;
      for (int k = 0; k < q->nlanes; ++k) s->laneBusy[q->lanes[k]] = false;
      s->used -= q->bytes;
      s->inflight[i] = s->inflight.back();
      s->inflight.pop_back();
    } else {
      ++i;
    }
  }
  if (failed) {
    while (!s->waiting.empty()) {
      Req* q = s->waiting.front();
      s->waiting.pop_front();
      q->state = 2;
      q->tDone = nowNs();
      q->status = vcclRemoteError;
    }
    return vcclSuccess;
  }
  // Admission: oldest first.  A request that does not fit yet (lanes or
  // budget) lets younger ones that fit go ahead until it has waited
  // bypassNs; from then on nothing overtakes it, so it cannot starve.
  bool admitted = false;
  int freeLanes = 0;
  for (int l = 0; l < s->L; ++l) freeLanes += s->laneBusy[l] ? 0 : 1;
  const uint64_t now = nowNs();
  for (auto wi = s->waiting.begin(); wi != s->waiting.end() && freeLanes > 0;) {
    Req* q = *wi;
    if (freeLanes < q->plan.nchannels || s->used + q->bytes > s->budget) {
      if (now - q->tSubmit >= s->bypassNs) break;
      ++wi;
      continue;
    }
    wi = s->waiting.erase(wi);
    Coll coll{};
    coll.coll = (uint8_t)q->r.coll;
    coll.dtype = q->r.datatype;
    coll.op = q->r.op;
    coll.root = q->r.root;
    coll.count = q->r.count;
    for (int r = 0; r < c->nranks; ++r) {
      coll.args.send[r] = (const char*)q->r.send[r];
      coll.args.recv[r] = (char*)q->r.recv[r];
    }
    std::vector<WorkItem> items;
    fillItems(c, coll, q->plan, 0, 0xFFFFFFFFu, &items);
    q->nlanes = (int)items.size();
    int k = 0;
    for (int l = 0; l < s->L && k < q->nlanes; ++l) {
      if (s->laneBusy[l]) continue;
      s->laneBusy[l] = true;
      q->lanes[k] = l;
      q->seqs[k] = s->posted[l];
      ServeEntry* e = s->hQueue + (uint64_t)l * SERVE_QUEUE + s->posted[l] % SERVE_QUEUE;
      e->item = items[k];
      e->args = coll.args;
      ++k;
    }
    std::atomic_thread_fence(std::memory_order_release);
    for (k = 0; k < q->nlanes; ++k) {
      const int l = q->lanes[k];
      ++s->posted[l];
      __atomic_store_n(s->hPosted + (uint64_t)l * SERVE_STRIDE_U64, s->posted[l], __ATOMIC_RELEASE);
    }
    s->used += q->bytes;
    freeLanes -= q->nlanes;
    q->state = 1;
    s->inflight.push_back(q);
    admitted = true;
  }
  // the kernel leaves after an idle period; bring it back when work is pending
  // (the kernel only ends after the stop or idle word was raised, so the
  // runtime is asked only then).  Entries posted to lanes whose leader had
  // already left are run by the relaunched kernel: it starts every lane at
  // the lane's completed count.
  if (s->running && kernelLeaving(s) && hipStreamQuery(s->stream) == hipSuccess) s->running = false;
  if (!s->running && (admitted || !s->inflight.empty())) return launchKernel(s);
  return vcclSuccess;
}

}  // namespace

extern "C" {

vcclResult_t vcclServeCreate(vcclComm_t* comms, size_t budgetBytes, int lanes, vcclServer_t* out) {
  if (!comms || !out || !comms[0] || lanes < 1) return vcclInvalidArgument;
  Clique* c = cliqueOf(comms[0]);
  if (!c || c->serving || c->aborted) return vcclInvalidUsage;
  if (lanes > c->maxLanes) return vcclInvalidArgument;
  VCCL_HIPCHECK(hipSetDevice(c->device));
  // every allocation happens before the persistent kernel starts: a device
  // synchronisation while it runs would wait for its idle exit
  // requests may plan trees under any protocol the set allows
  for (int p = 0; p < 3; ++p) {
    if (p == PROTO_LL128 && !c->ll128) continue;
    vcclResult_t tr = cliqueEnsureTreeFifos(c, p);
    if (tr != vcclSuccess) return tr;
  }
  VCCL_HIPCHECK(hipDeviceSynchronize());
  vcclServer* s = new vcclServer();
  s->c = c;
  s->L = lanes;
  s->budget = budgetBytes;
  s->block = (int)envLong("VCCL_SERVE_NTHREADS", 512);
  // one request takes at most half the lanes (fewer lanes per request use the
  // device more efficiently and let two large requests overlap)
  s->maxLanesPerReq = (int)std::max(1L, std::min<long>(lanes, envLong("VCCL_SERVE_MAX_LANES_PER_REQUEST",
                                                                      std::max(1, lanes / 2))));
  s->fullPlanBytes = (uint64_t)envLong("VCCL_SERVE_FULL_PLAN_BYTES", 16 << 20);
  s->bypassNs = (uint64_t)envLong("VCCL_SERVE_BYPASS_US", 500) * 1000ull;
  int occ = 0;
  if (vcclServeOccupancy(s->block, &occ) != hipSuccess || occ < 1) {
    delete s;
    return vcclInternalError;
  }
  const int R = c->nranks;
  s->grid = c->xcdMap ? 8 * R * ((lanes + 7) / 8) : R * lanes;
  if (s->grid > c->numCUs * occ) {
    delete s;
    return vcclInvalidArgument;
  }
  hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipHostMalloc((void**)&s->hQueue, sizeof(ServeEntry) * lanes * SERVE_QUEUE, hipHostMallocCoherent);
  if (e == hipSuccess) e = hipHostMalloc((void**)&s->hPosted, sizeof(uint64_t) * SERVE_STRIDE_U64 * MAX_LANES, hipHostMallocCoherent);
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&s->hDone, sizeof(uint64_t) * SERVE_STRIDE_U64 * MAX_LANES * MAX_RANKS, hipHostMallocCoherent);
  if (e == hipSuccess) e = hipHostMalloc((void**)&s->hStop, 256, hipHostMallocCoherent);
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&s->hDbg, sizeof(uint64_t) * SERVE_STRIDE_U64 * MAX_LANES * MAX_RANKS, hipHostMallocCoherent);
  if (e == hipSuccess) e = hipMalloc((void**)&s->dMirror, sizeof(ServeEntry) * lanes * SERVE_QUEUE);
  if (e == hipSuccess) e = hipMalloc((void**)&s->dLaneSeq, sizeof(uint64_t) * SERVE_STRIDE_U64 * lanes);
  if (e == hipSuccess) e = hipMemset(s->dLaneSeq, 0, sizeof(uint64_t) * SERVE_STRIDE_U64 * lanes);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    logError("serve create", e, __FILE__, __LINE__);
    freeServer(s);
    return vcclUnhandledHipError;
  }
  memset(s->hQueue, 0, sizeof(ServeEntry) * lanes * SERVE_QUEUE);
  memset(s->hPosted, 0, sizeof(uint64_t) * SERVE_STRIDE_U64 * MAX_LANES);
  memset(s->hDone, 0, sizeof(uint64_t) * SERVE_STRIDE_U64 * MAX_LANES * MAX_RANKS);
  memset(s->hStop, 0, 256);
  s->desc.comm = c->dcomm;
  s->desc.queue = s->hQueue;
  s->desc.posted = s->hPosted;
  s->desc.done = s->hDone;
  s->desc.stop = s->hStop;
  s->desc.idle = s->hStop + kIdleWord;
  memset(s->hDbg, 0, sizeof(uint64_t) * SERVE_STRIDE_U64 * MAX_LANES * MAX_RANKS);
  s->desc.dbg = s->hDbg;
  s->desc.mirror = s->dMirror;
  s->desc.laneSeq = s->dLaneSeq;
  s->desc.idleTicks = (uint64_t)((double)envLong("VCCL_SERVE_IDLE_US", 1000000) * c->ticksPerUs);
  s->desc.nlanes = (uint32_t)lanes;
  s->desc.nranks = (uint32_t)R;
  s->desc.xcdMap = (uint32_t)c->xcdMap;
  c->serving = true;
  vcclResult_t r = launchKernel(s);
  if (r != vcclSuccess) {
    c->serving = false;
    freeServer(s);
    return r;
  }
  *out = s;
  return vcclSuccess;
}

vcclResult_t vcclServeSubmit(vcclServer_t s, const vcclRequest_t* req, uint64_t* id) {
  if (!s || !req || !id) return vcclInvalidArgument;
  Clique* c = s->c;
  const int R = c->nranks;
  if (req->coll < COLL_ALLREDUCE || req->coll > COLL_REDUCESCATTER) return vcclInvalidArgument;
  if (req->datatype < vcclInt32 || req->datatype > vcclBfloat16 || req->op < vcclSum || req->op > vcclMax)
    return vcclInvalidArgument;
  if ((req->coll == COLL_BROADCAST || req->coll == COLL_REDUCE) && (req->root < 0 || req->root >= R))
    return vcclInvalidArgument;
  if (req->count == 0) return vcclInvalidArgument;
  const size_t E = dtypeBytes(req->datatype);
  for (int r = 0; r < R; ++r) {
    const bool needSend = !(req->coll == COLL_BROADCAST && r != req->root);
    const bool needRecv = !(req->coll == COLL_REDUCE && r != req->root);
    if ((needSend && !req->send[r]) || (needRecv && !req->recv[r])) return vcclInvalidArgument;
    if (((uintptr_t)req->send[r] % E) || ((uintptr_t)req->recv[r] % E)) return vcclInvalidArgument;
  }
  Req* q = new Req();
  q->id = s->nextId++;
  q->r = *req;
  Coll coll{};
  coll.coll = (uint8_t)req->coll;
  coll.dtype = req->datatype;
  coll.op = req->op;
  coll.root = req->root;
  coll.count = req->count;
  vcclResult_t r = planColl(c, coll, &q->plan);
  if (r != vcclSuccess) {
    delete q;
    return r;
  }
  // at most half the lanes, unless the request holds more than half the
  // budget: then nothing of its size can run beside it and it takes the
  // lanes its plan asks for
  // A request keeps its per-call plan's channels (up to the server's lanes)
  // when it is at least fullPlanBytes large, so it is served as fast as the
  // same call launched alone, or when its bits depend on the channel count,
  // so it gives the per-call bits: a floating-point sum AllReduce (the
  // ring's segments and the tree's per-channel trees follow the channels),
  // and, on a set with more than one ring order, a floating-point sum
  // ReduceScatter or Reduce (each channel folds along its own ring).  Every
  // other request takes at most maxLanesPerReq lanes, so that several
  // overlap; their results do not depend on the channel count.  The cap
  // depends only on the request.
  const Plan full = q->plan;
  const bool large = collSizeBytes((uint8_t)req->coll, req->count, req->datatype, R) >= s->fullPlanBytes;
  const bool floatSum = req->op == vcclSum && req->datatype != vcclInt32;
  const bool channelBits = floatSum && (req->coll == COLL_ALLREDUCE ||
                                        (c->nrings > 1 && (req->coll == COLL_REDUCESCATTER || req->coll == COLL_REDUCE)));
  q->plan.nchannels = std::min(full.nchannels, (large || channelBits) ? s->L : s->maxLanesPerReq);
  q->bytes = requestBytes(c, *req, q->plan);
  if (q->bytes > s->budget / 2) {
    q->plan.nchannels = std::min(full.nchannels, s->L);
    q->bytes = requestBytes(c, *req, q->plan);
  }
  if (q->bytes > s->budget) {
    delete q;
    return vcclInvalidArgument;  // could never be admitted
  }
  q->state = 0;
  q->tSubmit = nowNs();
  s->reqs[q->id] = q;
  s->waiting.push_back(q);
  *id = q->id;
  return progress(s);
}

vcclResult_t vcclServeTest(vcclServer_t s, uint64_t id, int* done, vcclResult_t* status, uint64_t* t_done_ns) {
  if (!s || !done) return vcclInvalidArgument;
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return vcclInvalidArgument;
  vcclResult_t r = progress(s);
  if (r != vcclSuccess) return r;
  Req* q = it->second;
  *done = q->state == 2;
  if (status) *status = q->state == 2 ? q->status : vcclInProgress;
  if (t_done_ns) *t_done_ns = q->state == 2 ? q->tDone : 0;
  if (q->state == 2) {
    s->reqs.erase(it);
    delete q;
  }
  return vcclSuccess;
}

vcclResult_t vcclServeReplay(vcclServer_t s, const vcclRequest_t* reqs, const uint64_t* arrival_ns, int n,
                             uint64_t* latency_ns, vcclResult_t* statuses) {
  if (!s || !reqs || !arrival_ns || !latency_ns || n < 0) return vcclInvalidArgument;
  std::vector<uint64_t> ids(n, 0), tArr(n, 0);
  std::vector<int> pending;  // submitted, not yet seen complete
  int next = 0, finished = 0;
  const uint64_t t0 = nowNs();
  while (finished < n) {
    const uint64_t now = nowNs();
    while (next < n && now - t0 >= arrival_ns[next]) {
      tArr[next] = t0 + arrival_ns[next];
      vcclResult_t r = vcclServeSubmit(s, &reqs[next], &ids[next]);
      if (r != vcclSuccess) return r;
      pending.push_back(next);
      ++next;
    }
    vcclResult_t r = progress(s);
    if (r != vcclSuccess) return r;
    for (size_t k = 0; k < pending.size();) {
      const int i = pending[k];
      auto it = s->reqs.find(ids[i]);
      if (it == s->reqs.end() || it->second->state != 2) {
        ++k;
        continue;
      }
      latency_ns[i] = it->second->tDone - tArr[i];
      if (statuses) statuses[i] = it->second->status;
      delete it->second;
      s->reqs.erase(it);
      pending[k] = pending.back();
      pending.pop_back();
      ++finished;
    }
  }
  return vcclSuccess;
}

vcclResult_t vcclServeGetPlan(vcclServer_t s, uint64_t id, vcclPlanInfo_t* info) {
  if (!s || !info) return vcclInvalidArgument;
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return vcclInvalidArgument;
  const Req* q = it->second;
  const Plan& p = q->plan;
  vcclPlanInfo_t o{};
  o.algo = p.algo;
  o.proto = p.proto;
  o.nchannels = p.nchannels;
  o.nthreads = s->block;
  o.direct = p.direct;
  o.nlanes = p.nchannels;
  o.nitems = p.nchannels;
  o.ncolls = 1;
  o.chunkBytes = (size_t)p.chunkBytes;
  o.grid = s->grid;
  o.scope = p.scope;
  o.treeRanksPerNode = s->c->ranksPerNode;
  o.ll128 = s->c->ll128 ? 1 : 0;
  *info = o;
  return vcclSuccess;
}

vcclResult_t vcclReplayPerCall(vcclComm_t* comms, const vcclRequest_t* reqs, const uint64_t* arrival_ns, int n,
                               void* stream, uint64_t* latency_ns, vcclResult_t* statuses) {
  if (!comms || !comms[0] || !reqs || !arrival_ns || !latency_ns || n < 0) return vcclInvalidArgument;
  Clique* c = cliqueOf(comms[0]);
  if (!c) return vcclInvalidArgument;
  const int R = c->nranks;
  for (int r = 0; r < R; ++r)
    if (!comms[r] || cliqueOf(comms[r]) != c || rankOf(comms[r]) != r) return vcclInvalidArgument;
  hipStream_t st = (hipStream_t)stream;
  VCCL_HIPCHECK(hipSetDevice(c->device));
  // one event per request in flight, reused round robin; the stream runs the
  // launches in issue order, so they complete in that order
  constexpr int kEvents = 256;
  std::vector<hipEvent_t> ev(kEvents, nullptr);
  vcclResult_t result = vcclSuccess;
  for (auto& e : ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) result = vcclUnhandledHipError;
  std::vector<uint64_t> tArr(n, 0);
  int next = 0, finished = 0;
  const uint64_t t0 = nowNs();
  auto retire = [&](bool block) {
    while (finished < next) {
      hipEvent_t e = ev[finished % kEvents];
      hipError_t q = block ? hipEventSynchronize(e) : hipEventQuery(e);
      if (q == hipErrorNotReady) return;
      if (q != hipSuccess) result = vcclUnhandledHipError;
      latency_ns[finished] = nowNs() - tArr[finished];
      ++finished;
      block = false;
    }
  };
  while (result == vcclSuccess && finished < n) {
    const uint64_t now = nowNs();
    while (result == vcclSuccess && next < n && now - t0 >= arrival_ns[next]) {
      if (next - finished >= kEvents) retire(true);  // every event is in flight: wait for the oldest
      const vcclRequest_t& q = reqs[next];
      tArr[next] = t0 + arrival_ns[next];
      vcclResult_t r = vcclSuccess;
      for (int k = 0; k < R && r == vcclSuccess; ++k) {
        const void* sb = q.send[k];
        void* rb = q.recv[k];
        switch (q.coll) {
          case COLL_ALLREDUCE:
            r = vcclAllReduce(sb, rb, q.count, (vcclDataType_t)q.datatype, (vcclRedOp_t)q.op, comms[k], st);
            break;
          case COLL_BROADCAST:
            r = vcclBroadcast(sb, rb, q.count, (vcclDataType_t)q.datatype, q.root, comms[k], st);
            break;
          case COLL_REDUCE:
            r = vcclReduce(sb, rb, q.count, (vcclDataType_t)q.datatype, (vcclRedOp_t)q.op, q.root, comms[k], st);
            break;
          case COLL_ALLGATHER:
            r = vcclAllGather(sb, rb, q.count, (vcclDataType_t)q.datatype, comms[k], st);
            break;
          case COLL_REDUCESCATTER:
            r = vcclReduceScatter(sb, rb, q.count, (vcclDataType_t)q.datatype, (vcclRedOp_t)q.op, comms[k], st);
            break;
          default:
            r = vcclInvalidArgument;
        }
      }
      if (statuses) statuses[next] = r;
      if (r != vcclSuccess) {
        result = r;
        break;
      }
      if (hipEventRecord(ev[next % kEvents], st) != hipSuccess) result = vcclUnhandledHipError;
      ++next;
    }
    retire(false);
  }
  if (result != vcclSuccess) hipStreamSynchronize(st);
  for (auto e : ev)
    if (e) hipEventDestroy(e);
  if (result == vcclSuccess && statuses) {
    vcclResult_t a = vcclSuccess;
    vcclCommGetAsyncError(comms[0], &a);
    if (a != vcclSuccess)
      for (int i = 0; i < n; ++i) statuses[i] = a;
  }
  return result;
}

// Debug view: for every (lane, rank): posted (host), last posted value the
// device saw, items the device picked up, done (device), poll iterations, and
// the device clock (100 MHz) when the last item was picked up and finished.
vcclResult_t vcclServeDebugState(vcclServer_t s, uint64_t* out, int maxEntries) {
  if (!s || !out) return vcclInvalidArgument;
  const int R = s->c->nranks;
  int k = 0;
  for (int l = 0; l < s->L; ++l)
    for (int r = 0; r < R && k < maxEntries; ++r, ++k) {
      const uint64_t* d = s->hDbg + ((uint64_t)l * R + r) * SERVE_STRIDE_U64;
      uint64_t* o = out + (uint64_t)VCCL_SERVE_DEBUG_WORDS * k;
      o[0] = __atomic_load_n(s->hPosted + (uint64_t)l * SERVE_STRIDE_U64, __ATOMIC_ACQUIRE);
      o[1] = __atomic_load_n(d, __ATOMIC_ACQUIRE);
      o[2] = __atomic_load_n(d + 1, __ATOMIC_ACQUIRE);
      o[3] = __atomic_load_n(s->hDone + ((uint64_t)l * R + r) * SERVE_STRIDE_U64, __ATOMIC_ACQUIRE);
      o[4] = __atomic_load_n(d + 2, __ATOMIC_ACQUIRE);
      o[5] = __atomic_load_n(d + 3, __ATOMIC_ACQUIRE);
      o[6] = __atomic_load_n(d + 4, __ATOMIC_ACQUIRE);
    }
  return vcclSuccess;
}

vcclResult_t vcclServeDestroy(vcclServer_t s) {
  if (!s) return vcclInvalidArgument;
  Clique* c = s->c;
  // drain: every admitted or waiting request completes (or the set failed)
  const uint64_t deadline = nowNs() + 60ull * 1000000000ull;
  while ((!s->waiting.empty() || !s->inflight.empty()) && nowNs() < deadline) progress(s);
  __atomic_store_n(s->hStop, 1u, __ATOMIC_RELEASE);
  hipStreamSynchronize(s->stream);
  c->serving = false;
  freeServer(s);
  return vcclSuccess;
}

}  // extern "C"
