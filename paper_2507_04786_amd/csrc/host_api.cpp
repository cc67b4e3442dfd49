// The C ABI: communicator management, per-rank call matching, group calls
// (Section II-A) and the launch of one kernel per matched call or group.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "host_internal.h"

using namespace vccl;

namespace vccl {

Clique* cliqueOf(vcclComm_t comm) { return comm ? comm->clique : nullptr; }
int rankOf(vcclComm_t comm) { return comm ? comm->rank : -1; }

namespace {

struct GroupState {
  int depth = 0;
  std::vector<std::pair<Clique*, Coll>> colls;
  std::vector<Clique*> touched;
  vcclResult_t firstError = vcclSuccess;
};
thread_local GroupState tlsGroup;

bool validHandle(vcclComm_t comm) { return comm && comm->clique && !comm->destroyed; }

vcclResult_t asyncStatus(Clique* c) {
  const uint32_t e = __atomic_load_n(c->hError, __ATOMIC_ACQUIRE);
  if (e & ERR_PLACEMENT) return vcclInternalError;
  if (c->aborted || e) return vcclRemoteError;
  return vcclSuccess;
}

// Joins the streams of every rank involved: the launch stream waits for all
// of them before the kernel, and all of them wait for the kernel after it.
struct StreamSet {
  hipStream_t list[2 * MAX_RANKS + 1];
  int n = 0;
  void add(hipStream_t s) {
    for (int i = 0; i < n; ++i)
      if (list[i] == s) return;
    list[n++] = s;
  }
};

vcclResult_t launchPrepared(Clique* c, LaunchDesc& d, int grid, int block, const StreamSet& ss) {
  hipStream_t ls = ss.list[ss.n - 1];
  int ev = 0;
  // collectives of one set run in issue order: follow the previous launch
  VCCL_HIPCHECK(hipStreamWaitEvent(ls, c->lastLaunchDone, 0));
  for (int i = 0; i < ss.n - 1; ++i) {
    VCCL_HIPCHECK(hipEventRecord(c->joinEvents[ev], ss.list[i]));
    VCCL_HIPCHECK(hipStreamWaitEvent(ls, c->joinEvents[ev], 0));
    ++ev;
  }
  hipError_t e = vcclLaunchColl(d, grid, block, ls, c->cooperative);
  if (e != hipSuccess) {
    logError("kernel launch", e, __FILE__, __LINE__);
    return vcclUnhandledHipError;
  }
  if (c->xcdMap) c->claimBase += d.perXcd;
  VCCL_HIPCHECK(hipEventRecord(c->lastLaunchDone, ls));
  for (int i = 0; i < ss.n - 1; ++i) VCCL_HIPCHECK(hipStreamWaitEvent(ss.list[i], c->lastLaunchDone, 0));
  return vcclSuccess;
}

// A split tree's lanes: channel ch's up half on lane ch, its down half on
// lane off + ch (off = 8 ceil(C / 8), a multiple of 8, so both halves run on
// one XCD); lanes between the two groups stay idle.
void splitTreeLanes(std::vector<WorkItem>* items) {
  const int C = (int)items->size(), off = 8 * ((C + 7) / 8);
  std::vector<WorkItem> byLane((size_t)(off + C));
  for (int l = 0; l < off; ++l) {
    byLane[l] = (*items)[l < C ? l : 0];
    byLane[l].role = l < C ? ROLE_UP : ROLE_IDLE;
    byLane[l].connLane = (uint8_t)l;
  }
  for (int ch = 0; ch < C; ++ch) {
    byLane[off + ch] = (*items)[ch];
    byLane[off + ch].role = ROLE_DOWN;
    byLane[off + ch].connLane = (uint8_t)ch;
  }
  items->swap(byLane);
}

// Work list in device memory: `items` in lane order, lane l running items
// laneStart[l] .. laneStart[l + 1] - 1, and the collectives' pointer tables,
// written to the pinned staging buffer and copied to the device in one copy
// on the launch stream (after the previous launch, which may still read the
// list).  The capacity must have been ensured.
vcclResult_t stageWork(Clique* c, const StreamSet& ss, const std::vector<WorkItem>& items,
                       const std::vector<uint32_t>& laneStart, const std::vector<Coll>& colls, LaunchDesc* d) {
  const int k = c->stageNext;
  c->stageNext ^= 1;
  VCCL_HIPCHECK(hipEventSynchronize(c->stageEvent[k]));
  char* stage = (char*)c->hStage[k];
  const WorkLayout wl = workLayout(items.size());
  memcpy(stage, items.data(), items.size() * sizeof(WorkItem));
  memcpy(stage + wl.laneOff, laneStart.data(), laneStart.size() * sizeof(uint32_t));
  CollArgs* sArgs = (CollArgs*)(stage + wl.argsOff);
  for (size_t g = 0; g < colls.size(); ++g) sArgs[g] = colls[g].args;
  hipStream_t ls = ss.list[ss.n - 1];
  VCCL_HIPCHECK(hipStreamWaitEvent(ls, c->lastLaunchDone, 0));
  VCCL_HIPCHECK(hipMemcpyAsync(c->dWork, stage, wl.argsOff + colls.size() * sizeof(CollArgs), hipMemcpyHostToDevice,
                               ls));
  VCCL_HIPCHECK(hipEventRecord(c->stageEvent[k], ls));
  d->items = (const WorkItem*)c->dWork;
  d->laneStart = (const uint32_t*)(c->dWork + wl.laneOff);
  d->args = (const CollArgs*)(c->dWork + wl.argsOff);
  d->stamps = c->dStamps;
  return vcclSuccess;
}

}  // namespace

vcclResult_t launchColls(Clique* c, const std::vector<Coll>& collsIn) {
  vcclResult_t st = asyncStatus(c);
  if (st != vcclSuccess) return st;
  if (c->serving) return vcclInvalidUsage;  // the serving kernel owns the lanes
  std::vector<Coll> colls;
  for (const auto& x : collsIn)
    if (x.count > 0) colls.push_back(x);
  if (colls.empty()) return vcclSuccess;
  const int R = c->nranks;
  VCCL_HIPCHECK(hipSetDevice(c->device));

  std::vector<Plan> plans(colls.size());
  for (size_t g = 0; g < colls.size(); ++g) {
    vcclResult_t r = planColl(c, colls[g], &plans[g], colls.size() == 1);
    if (r != vcclSuccess) return r;
    if (plans[g].algo == ALGO_TREE) {
      r = cliqueEnsureTreeFifos(c, plans[g].proto);
      if (r != vcclSuccess) return r;
    }
  }
  // Point-to-point transfers of a group share the lanes: channels in
  // proportion to each transfer's bytes, about two items per lane in all
  // (their results do not depend on the split; an explicit channel count
  // is kept)
  if (colls.size() > 1 && c->apiTune.nchannels <= 0 && c->envTune.nchannels <= 0) {
    double p2pBytes = 0;
    for (const auto& x : colls)
      if (x.coll == COLL_SENDRECV) p2pBytes += (double)x.count * dtypeBytes(x.dtype);
    const int L = p2pLaneCap(c);
    for (size_t g = 0; g < colls.size() && p2pBytes > 0; ++g) {
      if (colls[g].coll != COLL_SENDRECV) continue;
      const double share = (double)colls[g].count * dtypeBytes(colls[g].dtype) / p2pBytes;
      plans[g].nchannels = std::max(1, std::min(plans[g].nchannels, (int)std::ceil(share * 2 * L)));
    }
  }
  StreamSet ss;
  for (const auto& x : colls)
    for (int r = 0; r < R; ++r) ss.add(x.streams[r]);

  vcclResult_t r = cliqueEnsureWorkCapacity(c, 0, 0, colls.size() * (size_t)R);
  if (r != vcclSuccess) return r;

  LaunchDesc d;
  memset((void*)&d, 0, sizeof(d));
  d.comm = c->dcomm;
  d.nranks = (uint32_t)R;
  d.xcdMap = (uint32_t)c->xcdMap;
  d.stamps = c->dStamps;
  int block = 64;
  for (const auto& p : plans) block = std::max(block, p.nthreads);

  int nlanes = 0;
  size_t nitems = 0;
  // a single collective whose lanes fit the descriptor runs from kernel
  // arguments; a split tree takes 8 ceil(C / 8) + C lanes
  const int singleLanes =
      colls.size() == 1 ? (plans[0].split ? 8 * ((plans[0].nchannels + 7) / 8) : 0) + plans[0].nchannels : 0;
  if (colls.size() == 1 && plans[0].split) {
    // one item per lane: the work list takes the lanes as arranged
    std::vector<WorkItem> items;
    fillItems(c, colls[0], plans[0], 0, 0, &items);
    splitTreeLanes(&items);
    if ((int)items.size() <= MAX_INLINE) {
      d.items = nullptr;
      d.inlineArgs = colls[0].args;
      for (size_t i = 0; i < items.size(); ++i) d.inlineItems[i] = items[i];
    } else {
      r = cliqueEnsureWorkCapacity(c, items.size(), 1, (size_t)R);
      if (r != vcclSuccess) return r;
      std::vector<uint32_t> laneStart(items.size() + 1);
      std::iota(laneStart.begin(), laneStart.end(), 0u);
      r = stageWork(c, ss, items, laneStart, colls, &d);
      if (r != vcclSuccess) return r;
    }
    nlanes = (int)items.size();
    nitems = items.size();
  } else if (colls.size() == 1 && singleLanes <= MAX_INLINE) {
    std::vector<WorkItem> items;
    fillItems(c, colls[0], plans[0], 0, 0, &items);
    d.items = nullptr;
    d.inlineArgs = colls[0].args;
    for (size_t i = 0; i < items.size(); ++i) d.inlineItems[i] = items[i];
    nlanes = (int)items.size();
    nitems = items.size();
  } else {
    // work list: every collective's channel items placed on lanes, longest
    // first onto the least-loaded lane; each lane keeps issue order
    std::vector<WorkItem> items;
    for (size_t g = 0; g < colls.size(); ++g) fillItems(c, colls[g], plans[g], (uint32_t)g, (uint32_t)g, &items);
    const int occ = cliqueOccupancy(c, block);
    int capLanes = c->xcdMap ? (c->numCUs * occ / (8 * R)) * 8 : c->numCUs * occ / R;
    capLanes = std::max(1, std::min(capLanes, c->maxLanes));
    int maxCh = 1;
    for (const auto& p : plans) maxCh = std::max(maxCh, p.nchannels);
    nlanes = std::min<int>(capLanes, std::max<int>(maxCh, std::min<int>((int)items.size(), c->maxLanes)));
    // a group of point-to-point copies only: one workgroup per CU
    bool p2pOnly = true;
    for (const auto& x : colls) p2pOnly = p2pOnly && x.coll == COLL_SENDRECV;
    if (p2pOnly) nlanes = std::max(1, std::min(nlanes, p2pLaneCap(c)));
    std::vector<double> cost(items.size());
    for (size_t i = 0; i < items.size(); ++i) cost[i] = estimateCost(c, items[i]);
    std::vector<size_t> order(items.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return cost[a] > cost[b]; });
    std::vector<double> load(nlanes, 0.0);
    std::vector<int> laneOf(items.size());
    for (size_t k : order) {
      int best = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      laneOf[k] = best;
      load[best] += cost[k];
    }
    std::vector<std::vector<uint32_t>> perLane(nlanes);
    for (size_t i = 0; i < items.size(); ++i) perLane[laneOf[i]].push_back((uint32_t)i);
    r = cliqueEnsureWorkCapacity(c, items.size(), colls.size(), colls.size() * (size_t)R);
    if (r != vcclSuccess) return r;
    std::vector<WorkItem> ordered;
    ordered.reserve(items.size());
    std::vector<uint32_t> laneStart((size_t)nlanes + 1);
    for (int l = 0; l < nlanes; ++l) {
      laneStart[l] = (uint32_t)ordered.size();
      for (uint32_t i : perLane[l]) ordered.push_back(items[i]);
    }
    laneStart[nlanes] = (uint32_t)ordered.size();
    r = stageWork(c, ss, ordered, laneStart, colls, &d);
    if (r != vcclSuccess) return r;
    nitems = items.size();
  }
  d.nlanes = (uint32_t)nlanes;
  const int grid = c->xcdMap ? 8 * R * ((nlanes + 7) / 8) : R * nlanes;
  d.perXcd = (uint32_t)(R * ((nlanes + 7) / 8));
  d.claimBase = c->claimBase;
  const int occ = cliqueOccupancy(c, block);
  if (grid > c->numCUs * occ) return vcclInternalError;
  if (c->profile) {
    d.profile = c->dProfile;
    VCCL_HIPCHECK(hipMemsetAsync(c->dProfile, 0, (size_t)MAX_LANES * R * PROFILE_WORDS * sizeof(uint64_t),
                                 ss.list[ss.n - 1]));
  }
  r = launchPrepared(c, d, grid, block, ss);
  if (r != vcclSuccess) return r;
  c->lastStampColls = (int)colls.size();
  c->lastLanes = nlanes;
  vcclPlanInfo_t& info = c->lastPlan;
  info.algo = plans[0].algo;
  info.proto = plans[0].proto;
  info.nchannels = plans[0].nchannels;
  info.nthreads = block;
  info.direct = plans[0].direct;
  info.chunkBytes = (size_t)plans[0].chunkBytes;
  info.nlanes = nlanes;
  info.nitems = (int)nitems;
  info.ncolls = (int)colls.size();
  info.grid = grid;
  info.scope = plans[0].scope;
  info.treeRanksPerNode = c->ranksPerNode;
  info.ll128 = c->ll128 ? 1 : 0;
  return vcclSuccess;
}

// LL128 tear test (Section III-C: LL128 is used only where 128-byte stores
// are never observed split).  `pairs` writer/reader workgroup pairs exchange
// `lines` lines for `rounds` rounds under the store policy `scope`; every
// wait is bounded by maxUs.  Allocates and frees its own buffers on every
// path.
hipError_t tearProbe(int device, int pairs, int lines, int rounds, int scope, uint64_t maxUs, uint64_t* torn,
                     uint64_t* checked, bool* timedOut) {
  char* bufs = nullptr;
  uint64_t* acks = nullptr;
  unsigned long long* counts = nullptr;
  uint32_t* failed = nullptr;
  const size_t bytes = (size_t)pairs * lines * LL128_LINE;
  const size_t ackBytes = (size_t)pairs * 32 * sizeof(uint64_t);
  hipError_t e = hipMalloc((void**)&bufs, bytes);
  if (e == hipSuccess) e = hipMalloc((void**)&acks, ackBytes);
  if (e == hipSuccess) e = hipMalloc((void**)&counts, 2 * sizeof(unsigned long long));
  if (e == hipSuccess) e = hipMalloc((void**)&failed, sizeof(uint32_t));
  if (e == hipSuccess) e = hipMemset(bufs, 0, bytes);
  if (e == hipSuccess) e = hipMemset(acks, 0, ackBytes);
  if (e == hipSuccess) e = hipMemset(counts, 0, 2 * sizeof(unsigned long long));
  if (e == hipSuccess) e = hipMemset(failed, 0, sizeof(uint32_t));
  int wallKHz = 100000;
  if (hipDeviceGetAttribute(&wallKHz, hipDeviceAttributeWallClockRate, device) != hipSuccess || wallKHz <= 0)
    wallKHz = 100000;
  const uint64_t maxTicks = (uint64_t)wallKHz * maxUs / 1000ull;
  if (e == hipSuccess) e = vcclLaunchTearProbe(bufs, acks, pairs, lines, rounds, counts, maxTicks, failed, scope, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  unsigned long long h[2] = {0, 0};
  uint32_t hf = 0;
  if (e == hipSuccess) e = hipMemcpy(h, counts, sizeof(h), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(&hf, failed, sizeof(hf), hipMemcpyDeviceToHost);
  if (bufs) hipFree(bufs);
  if (acks) hipFree(acks);
  if (counts) hipFree(counts);
  if (failed) hipFree(failed);
  *torn = h[0];
  *checked = h[1];
  *timedOut = hf != 0;
  return e;
}

// Whether LL128 may be planned on `device`: VCCL_LL128=0 turns it off and
// VCCL_LL128=1 on without a test; otherwise the tear test runs once per
// device and process, under both store policies (XCD scope: writer and
// reader on one XCD; device scope: on different XCDs), each wait bounded by
// 100 ms.  Any torn line, a wait past its bound or a failed HIP call turns
// LL128 off for every set on that device.
bool ll128Allowed(int device) {
  static int8_t state[64] = {0};  // 0 untested, 1 allowed, 2 off
  const std::string env = envStr("VCCL_LL128");
  if (env == "0") return false;
  if (env == "1") return true;
  if (device < 0 || device >= 64) return false;
  if (state[device] == 0) {
    bool ok = true;
    const int cfg[2][2] = {{SCOPE_XCD, 16}, {SCOPE_DEVICE, 4}};
    for (const auto& pc : cfg) {
      uint64_t torn = 0, checked = 0;
      bool timedOut = false;
      hipError_t e = tearProbe(device, pc[1], 2048, 6, pc[0], 100000, &torn, &checked, &timedOut);
      if (e != hipSuccess || timedOut || torn != 0 || checked == 0) {
        logInfo("LL128 off: tear test (scope %d) %s, %llu torn of %llu lines", pc[0],
                e != hipSuccess ? hipGetErrorString(e) : (timedOut ? "timed out" : "ran"),
                (unsigned long long)torn, (unsigned long long)checked);
        ok = false;
        break;
      }
    }
    state[device] = ok ? 1 : 2;
  }
  return state[device] == 1;
}

}  // namespace vccl

// ------------------------------------------------------------------ C ABI

extern "C" {

const char* vcclGetErrorString(vcclResult_t r) {
  switch (r) {
    case vcclSuccess: return "no error";
    case vcclUnhandledHipError: return "unhandled HIP error";
    case vcclSystemError: return "system error";
    case vcclInternalError: return "internal error";
    case vcclInvalidArgument: return "invalid argument";
    case vcclInvalidUsage: return "invalid usage";
    case vcclRemoteError: return "remote error (peer timeout or abort)";
    case vcclInProgress: return "operation in progress";
  }
  return "unknown result";
}

vcclResult_t vcclGetVersion(int* version) {
  if (!version) return vcclInvalidArgument;
  *version = VCCL_MAJOR * 100 + VCCL_MINOR;
  return vcclSuccess;
}

vcclResult_t vcclCommInitAllRings(vcclComm_t* comms, int nranks, const int* devlist, int nrings, const int* rings) {
  if (!comms || nranks < 2 || nranks > VCCL_MAX_RANKS) return vcclInvalidArgument;
  if (rings) {
    if (nrings < 1 || nrings > VCCL_MAX_RINGS) return vcclInvalidArgument;
    for (int k = 0; k < nrings; ++k) {  // every row a permutation of 0..nranks-1
      bool seen[VCCL_MAX_RANKS] = {false};
      for (int q = 0; q < nranks; ++q) {
        const int r = rings[k * nranks + q];
        if (r < 0 || r >= nranks || seen[r]) return vcclInvalidArgument;
        seen[r] = true;
      }
    }
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return vcclUnhandledHipError;
  int dev = 0;
  if (devlist) {
    dev = devlist[0];
    for (int i = 1; i < nranks; ++i)
      if (devlist[i] != dev) return vcclInvalidArgument;
  } else {
    if (hipGetDevice(&dev) != hipSuccess) return vcclUnhandledHipError;
  }
  if (dev < 0 || dev >= ndev) return vcclInvalidArgument;
  Clique* c = nullptr;
  vcclResult_t r = cliqueCreate(nranks, dev, nrings, rings, &c);
  if (r != vcclSuccess) return r;
  for (int i = 0; i < nranks; ++i) {
    vcclComm* h = new vcclComm{c, i, false};
    c->handles.push_back(h);
    comms[i] = h;
  }
  logInfo("init %d virtual ranks on device %d, %d channels max, %d ring order(s)", nranks, dev, c->maxLanes,
          c->nrings);
  return vcclSuccess;
}

vcclResult_t vcclCommInitAll(vcclComm_t* comms, int nranks, const int* devlist) {
  return vcclCommInitAllRings(comms, nranks, devlist, 0, nullptr);
}

vcclResult_t vcclCommGetRings(vcclComm_t comm, int* nrings, int* rings) {
  if (!validHandle(comm) || !nrings) return vcclInvalidArgument;
  Clique* c = comm->clique;
  *nrings = c->nrings;
  if (rings)
    for (int k = 0; k < c->nrings; ++k)
      for (int q = 0; q < c->nranks; ++q) rings[k * c->nranks + q] = c->host.ringRank[k][q];
  return vcclSuccess;
}

vcclResult_t vcclCommDestroy(vcclComm_t comm) {
  if (!validHandle(comm)) return vcclInvalidArgument;
  Clique* c = comm->clique;
  hipSetDevice(c->device);
  hipDeviceSynchronize();
  comm->destroyed = true;
  if (++c->destroyedHandles == c->nranks) cliqueFree(c);
  return vcclSuccess;
}

vcclResult_t vcclCommAbort(vcclComm_t comm) {
  if (!validHandle(comm)) return vcclInvalidArgument;
  Clique* c = comm->clique;
  __atomic_store_n(c->hAbort, 1u, __ATOMIC_RELEASE);
  c->aborted = true;
  for (auto& q : c->pending) q.clear();
  hipSetDevice(c->device);
  hipDeviceSynchronize();
  return vcclSuccess;
}

vcclResult_t vcclCommGetAsyncError(vcclComm_t comm, vcclResult_t* asyncError) {
  if (!validHandle(comm) || !asyncError) return vcclInvalidArgument;
  *asyncError = asyncStatus(comm->clique);
  return vcclSuccess;
}

vcclResult_t vcclCommCount(vcclComm_t comm, int* count) {
  if (!validHandle(comm) || !count) return vcclInvalidArgument;
  *count = comm->clique->nranks;
  return vcclSuccess;
}

vcclResult_t vcclCommUserRank(vcclComm_t comm, int* rank) {
  if (!validHandle(comm) || !rank) return vcclInvalidArgument;
  *rank = comm->rank;
  return vcclSuccess;
}

static vcclResult_t enqueueCall(vcclComm_t comm, const Call& call) {
  if (!validHandle(comm)) return vcclInvalidArgument;
  Clique* c = comm->clique;
  if (c->aborted) return vcclRemoteError;
  const int R = c->nranks;
  if (call.dtype < vcclInt32 || call.dtype > vcclBfloat16) return vcclInvalidArgument;
  const bool reduces = call.coll == COLL_ALLREDUCE || call.coll == COLL_REDUCE || call.coll == COLL_REDUCESCATTER;
  if (reduces && (call.op < vcclSum || call.op > vcclMax)) return vcclInvalidArgument;
  const bool rooted = call.coll == COLL_BROADCAST || call.coll == COLL_REDUCE;
  if (rooted && (call.root < 0 || call.root >= R)) return vcclInvalidArgument;
  const size_t E = dtypeBytes(call.dtype);
  const int me = comm->rank;
  const bool needSend = !(call.coll == COLL_BROADCAST && me != call.root);
  const bool needRecv = !(call.coll == COLL_REDUCE && me != call.root);
  if (call.count > 0) {
    if (needSend && !call.send) return vcclInvalidArgument;
    if (needRecv && !call.recv) return vcclInvalidArgument;
  }
  if (((uintptr_t)call.send % E) || ((uintptr_t)call.recv % E)) return vcclInvalidArgument;
  if (call.count > ((size_t)1 << 40)) return vcclInvalidArgument;
  c->pending[me].push_back(call);
  if (tlsGroup.depth > 0 &&
      std::find(tlsGroup.touched.begin(), tlsGroup.touched.end(), c) == tlsGroup.touched.end())
    tlsGroup.touched.push_back(c);  // checked for unmatched calls at GroupEnd
  for (int r = 0; r < R; ++r)
    if (c->pending[r].empty()) return vcclSuccess;  // wait for the other ranks
  Coll coll{};
  const Call& f = c->pending[0].front();
  coll.coll = f.coll;
  coll.dtype = f.dtype;
  coll.op = f.op;
  coll.root = f.root;
  coll.count = f.count;
  vcclResult_t mismatch = vcclSuccess;
  for (int r = 0; r < R; ++r) {
    const Call& x = c->pending[r].front();
    if (x.coll != f.coll || x.count != f.count || x.dtype != f.dtype || (reduces && x.op != f.op) ||
        (rooted && x.root != f.root))
      mismatch = vcclInvalidUsage;
    coll.args.send[r] = (const char*)x.send;
    coll.args.recv[r] = (char*)x.recv;
    coll.streams[r] = x.stream;
  }
  for (int r = 0; r < R; ++r) c->pending[r].pop_front();
  if (mismatch != vcclSuccess) return mismatch;
  if (tlsGroup.depth > 0) {
    tlsGroup.colls.push_back({c, coll});
    return vcclSuccess;
  }
  std::vector<Coll> one{coll};
  return launchColls(c, one);
}

// Send / Recv (Section II-A): the k-th send from rank a to rank b pairs with
// the k-th receive posted by b from a.  A pair is issued once both sides are
// posted: inside a group at GroupEnd, together with the group's other work,
// outside a group at once.
static vcclResult_t enqueueP2p(vcclComm_t comm, bool isSend, void* buf, size_t count, int dtype, int peer,
                               hipStream_t stream) {
  if (!validHandle(comm)) return vcclInvalidArgument;
  Clique* c = comm->clique;
  if (c->aborted) return vcclRemoteError;
  const int R = c->nranks;
  if (dtype < vcclInt32 || dtype > vcclBfloat16) return vcclInvalidArgument;
  if (peer < 0 || peer >= R) return vcclInvalidArgument;
  if (count > 0 && !buf) return vcclInvalidArgument;
  if ((uintptr_t)buf % dtypeBytes(dtype)) return vcclInvalidArgument;
  if (count > ((size_t)1 << 40)) return vcclInvalidArgument;
  const int me = comm->rank;
  const int sender = isSend ? me : peer, receiver = isSend ? peer : me;
  const size_t key = (size_t)sender * R + receiver;
  (isSend ? c->p2pSends : c->p2pRecvs)[key].push_back(P2pOp{buf, count, dtype, stream});
  if (tlsGroup.depth > 0 &&
      std::find(tlsGroup.touched.begin(), tlsGroup.touched.end(), c) == tlsGroup.touched.end())
    tlsGroup.touched.push_back(c);
  auto& sq = c->p2pSends[key];
  auto& rq = c->p2pRecvs[key];
  if (sq.empty() || rq.empty()) return vcclSuccess;  // wait for the partner
  const P2pOp snd = sq.front(), rcv = rq.front();
  sq.pop_front();
  rq.pop_front();
  if (snd.count != rcv.count || snd.dtype != rcv.dtype) return vcclInvalidUsage;
  Coll coll{};
  coll.coll = COLL_SENDRECV;
  coll.dtype = snd.dtype;
  coll.op = vcclSum;
  coll.root = sender;
  coll.peer = receiver;
  coll.count = snd.count;
  coll.args.send[sender] = (const char*)snd.buf;
  coll.args.recv[receiver] = (char*)rcv.buf;
  for (int r = 0; r < R; ++r) coll.streams[r] = snd.stream;
  coll.streams[receiver] = rcv.stream;
  if (tlsGroup.depth > 0) {
    tlsGroup.colls.push_back({c, coll});
    return vcclSuccess;
  }
  std::vector<Coll> one{coll};
  return launchColls(c, one);
}

vcclResult_t vcclSend(const void* sendbuff, size_t count, vcclDataType_t datatype, int peer, vcclComm_t comm,
                      void* stream) {
  return enqueueP2p(comm, true, const_cast<void*>(sendbuff), count, (int)datatype, peer, (hipStream_t)stream);
}

vcclResult_t vcclRecv(void* recvbuff, size_t count, vcclDataType_t datatype, int peer, vcclComm_t comm, void* stream) {
  return enqueueP2p(comm, false, recvbuff, count, (int)datatype, peer, (hipStream_t)stream);
}

vcclResult_t vcclAllReduce(const void* sendbuff, void* recvbuff, size_t count, vcclDataType_t datatype,
                           vcclRedOp_t op, vcclComm_t comm, void* stream) {
  Call x{COLL_ALLREDUCE, (int)datatype, (int)op, 0, count, sendbuff, recvbuff, (hipStream_t)stream};
  return enqueueCall(comm, x);
}

vcclResult_t vcclBroadcast(const void* sendbuff, void* recvbuff, size_t count, vcclDataType_t datatype, int root,
                           vcclComm_t comm, void* stream) {
  Call x{COLL_BROADCAST, (int)datatype, (int)vcclSum, root, count, sendbuff, recvbuff, (hipStream_t)stream};
  return enqueueCall(comm, x);
}

vcclResult_t vcclReduce(const void* sendbuff, void* recvbuff, size_t count, vcclDataType_t datatype,
                        vcclRedOp_t op, int root, vcclComm_t comm, void* stream) {
  Call x{COLL_REDUCE, (int)datatype, (int)op, root, count, sendbuff, recvbuff, (hipStream_t)stream};
  return enqueueCall(comm, x);
}

vcclResult_t vcclAllGather(const void* sendbuff, void* recvbuff, size_t sendcount, vcclDataType_t datatype,
                           vcclComm_t comm, void* stream) {
  Call x{COLL_ALLGATHER, (int)datatype, (int)vcclSum, 0, sendcount, sendbuff, recvbuff, (hipStream_t)stream};
  return enqueueCall(comm, x);
}

vcclResult_t vcclReduceScatter(const void* sendbuff, void* recvbuff, size_t recvcount, vcclDataType_t datatype,
                               vcclRedOp_t op, vcclComm_t comm, void* stream) {
  Call x{COLL_REDUCESCATTER, (int)datatype, (int)op, 0, recvcount, sendbuff, recvbuff, (hipStream_t)stream};
  return enqueueCall(comm, x);
}

vcclResult_t vcclGroupStart(void) {
  ++tlsGroup.depth;
  return vcclSuccess;
}

vcclResult_t vcclGroupEnd(void) {
  if (tlsGroup.depth <= 0) return vcclInvalidUsage;
  if (--tlsGroup.depth > 0) return vcclSuccess;
  vcclResult_t result = vcclSuccess;
  std::vector<Clique*> touched;
  touched.swap(tlsGroup.touched);
  auto colls = std::move(tlsGroup.colls);
  tlsGroup.colls.clear();
  for (Clique* c : touched) {
    bool incomplete = false;
    for (auto& q : c->pending)
      if (!q.empty()) incomplete = true;
    for (auto* qs : {&c->p2pSends, &c->p2pRecvs})
      for (auto& q : *qs)
        if (!q.empty()) incomplete = true;
    if (incomplete) {
      // a call whose partners never came (a collective not called by every
      // rank, a send without its receive): nothing of this set is launched
      for (auto& q : c->pending) q.clear();
      for (auto* qs : {&c->p2pSends, &c->p2pRecvs})
        for (auto& q : *qs) q.clear();
      result = vcclInvalidUsage;
      continue;
    }
    std::vector<Coll> mine;
    for (auto& pc : colls)
      if (pc.first == c) mine.push_back(pc.second);
    vcclResult_t r = launchColls(c, mine);
    if (r != vcclSuccess && result == vcclSuccess) result = r;
  }
  return result;
}

vcclResult_t vcclCommSetTuning(vcclComm_t comm, const vcclTuning_t* t) {
  if (!validHandle(comm) || !t) return vcclInvalidArgument;
  if (t->algo < -1 || t->algo > 1 || t->proto < -1 || t->proto > 2) return vcclInvalidArgument;
  if (t->nchannels < 0 || t->nchannels > VCCL_MAX_CHANNELS) return vcclInvalidArgument;
  if (t->nthreads != 0 && (t->nthreads < 64 || t->nthreads > 1024 || t->nthreads % 64)) return vcclInvalidArgument;
  if (t->chunkBytes % 16) return vcclInvalidArgument;
  Clique* c = comm->clique;
  if (t->nchannels > c->maxLanes) return vcclInvalidArgument;
  c->apiTune.algo = t->algo;
  c->apiTune.proto = t->proto;
  c->apiTune.nchannels = t->nchannels;
  c->apiTune.nthreads = t->nthreads;
  c->apiTune.chunkBytes = t->chunkBytes;
  c->apiTune.direct = t->direct;
  return vcclSuccess;
}

vcclResult_t vcclCommGetLastPlan(vcclComm_t comm, vcclPlanInfo_t* info) {
  if (!validHandle(comm) || !info) return vcclInvalidArgument;
  *info = comm->clique->lastPlan;
  return vcclSuccess;
}

vcclResult_t vcclCommGetLastTimestamps(vcclComm_t comm, uint64_t* stamps_ns, int n, int* written) {
  if (!validHandle(comm) || !stamps_ns || !written) return vcclInvalidArgument;
  Clique* c = comm->clique;
  const int R = c->nranks;
  const int nc = std::min(n, c->lastStampColls);
  *written = 0;
  if (nc <= 0) return vcclSuccess;
  VCCL_HIPCHECK(hipEventSynchronize(c->lastLaunchDone));
  std::vector<uint64_t> raw((size_t)nc * R);
  VCCL_HIPCHECK(hipMemcpy(raw.data(), c->dStamps, raw.size() * sizeof(uint64_t), hipMemcpyDeviceToHost));
  for (int g = 0; g < nc; ++g) {
    uint64_t m = 0;
    for (int r = 0; r < R; ++r) m = std::max(m, raw[(size_t)g * R + r]);
    stamps_ns[g] = (uint64_t)((double)m / c->ticksPerUs * 1000.0);
  }
  *written = nc;
  return vcclSuccess;
}

vcclResult_t vcclCommDebugProfile(vcclComm_t comm, int enable) {
  if (!validHandle(comm)) return vcclInvalidArgument;
  Clique* c = comm->clique;
  VCCL_HIPCHECK(hipSetDevice(c->device));
  VCCL_HIPCHECK(hipDeviceSynchronize());
  if (enable && !c->dProfile)
    VCCL_HIPCHECK(hipMalloc((void**)&c->dProfile, (size_t)MAX_LANES * c->nranks * PROFILE_WORDS * sizeof(uint64_t)));
  c->profile = enable != 0;
  return vcclSuccess;
}

vcclResult_t vcclCommDebugReadProfile(vcclComm_t comm, uint64_t* out, int maxEntries, int* written) {
  if (!validHandle(comm) || !out || !written) return vcclInvalidArgument;
  Clique* c = comm->clique;
  *written = 0;
  if (!c->dProfile || c->lastLanes <= 0 || maxEntries <= 0) return vcclSuccess;
  VCCL_HIPCHECK(hipEventSynchronize(c->lastLaunchDone));
  const int n = std::min(maxEntries, c->lastLanes * c->nranks);
  std::vector<uint64_t> raw((size_t)n * PROFILE_WORDS);
  VCCL_HIPCHECK(hipMemcpy(raw.data(), c->dProfile, raw.size() * sizeof(uint64_t), hipMemcpyDeviceToHost));
  const double nsPerTick = 1000.0 / c->ticksPerUs;
  for (int k = 0; k < n; ++k) {
    const uint64_t* rec = &raw[(size_t)k * PROFILE_WORDS];
    out[4 * k + 0] = (uint64_t)((double)rec[0] * nsPerTick);
    out[4 * k + 1] = (uint64_t)((double)rec[1] * nsPerTick);
    out[4 * k + 2] = (uint64_t)((double)rec[2] * nsPerTick);
    out[4 * k + 3] = rec[3];
  }
  *written = n;
  return vcclSuccess;
}

vcclResult_t vcclCommGetTree(vcclComm_t comm, int tree, int* parents) {
  if (!validHandle(comm) || !parents || tree < 0 || tree > 1) return vcclInvalidArgument;
  const Clique* c = comm->clique;
  for (int r = 0; r < c->nranks; ++r) parents[r] = c->host.parent[tree][r];
  return vcclSuccess;
}

vcclResult_t vcclCommSetTimeout(vcclComm_t comm, uint64_t timeout_us) {
  if (!validHandle(comm) || timeout_us == 0) return vcclInvalidArgument;
  Clique* c = comm->clique;
  VCCL_HIPCHECK(hipSetDevice(c->device));
  VCCL_HIPCHECK(hipDeviceSynchronize());
  c->host.timeoutTicks = (uint64_t)((double)timeout_us * c->ticksPerUs);
  VCCL_HIPCHECK(hipMemcpy(c->dcomm, &c->host, sizeof(DevComm), hipMemcpyHostToDevice));
  return vcclSuccess;
}

vcclResult_t vcclCommDebugSetDeadRanks(vcclComm_t comm, uint32_t mask) {
  if (!validHandle(comm)) return vcclInvalidArgument;
  Clique* c = comm->clique;
  VCCL_HIPCHECK(hipSetDevice(c->device));
  VCCL_HIPCHECK(hipDeviceSynchronize());
  c->host.deadMask = mask;
  VCCL_HIPCHECK(hipMemcpy(c->dcomm, &c->host, sizeof(DevComm), hipMemcpyHostToDevice));
  return vcclSuccess;
}

vcclResult_t vcclCommDebugReadFifo(vcclComm_t comm, int channel, int rank, int proto, size_t offset, void* dst,
                                   size_t bytes) {
  if (!validHandle(comm) || !dst) return vcclInvalidArgument;
  Clique* c = comm->clique;
  if (channel < 0 || channel >= c->maxLanes || rank < 0 || rank >= c->nranks || proto < 0 || proto > 2)
    return vcclInvalidArgument;
  const uint64_t fifoBytes = (uint64_t)NSLOTS * c->host.slotBytes[proto];
  if (offset > fifoBytes || bytes > fifoBytes - offset) return vcclInvalidArgument;  // no wrap for huge offsets
  const uint64_t id = (uint64_t)channel * c->nranks + rank;
  VCCL_HIPCHECK(hipSetDevice(c->device));
  VCCL_HIPCHECK(hipDeviceSynchronize());
  VCCL_HIPCHECK(hipMemcpy(dst, c->fifo[proto] + id * fifoBytes + offset, bytes, hipMemcpyDeviceToHost));
  return vcclSuccess;
}

vcclResult_t vcclDebugPlanHost(int nranks, int coll, size_t count, vcclDataType_t datatype, int ll128, int single,
                               const vcclTuning_t* tuning, vcclPlanInfo_t* info) {
  if (!info || nranks < 2 || nranks > VCCL_MAX_RANKS || coll < COLL_ALLREDUCE || coll > COLL_REDUCESCATTER ||
      datatype < vcclInt32 || datatype > vcclBfloat16 || count == 0)
    return vcclInvalidArgument;
  // the model device: nothing here reaches the HIP runtime (every occupancy
  // the planner may ask for is filled in)
  Clique c;
  c.nranks = nranks;
  c.numCUs = 256;
  c.maxLanes = defaultLaneLimit(c.numCUs, nranks);
  for (int i = 1; i <= 16; ++i) c.occupancy[i] = std::max(1, 16 / i);
  c.host.scope = SCOPE_XCD;
  c.host.slotBytes[PROTO_SIMPLE] = SLOT_BYTES_SIMPLE;
  c.host.slotBytes[PROTO_LL] = SLOT_BYTES_LL;
  c.host.slotBytes[PROTO_LL128] = SLOT_BYTES_LL128;
  c.host.treeSlotBytes[PROTO_SIMPLE] = TREE_SLOT_BYTES_SIMPLE;
  c.host.treeSlotBytes[PROTO_LL] = TREE_SLOT_BYTES_LL;
  c.host.treeSlotBytes[PROTO_LL128] = TREE_SLOT_BYTES_LL128;
  c.deviceScopeBytes = 16 << 20;
  c.ll128 = ll128 != 0;
  buildTrees(nranks, 1, c.host.parent, c.host.child, c.host.childIdx, c.host.nchild);
  if (tuning) {
    const vcclTuning_t* t = tuning;
    if (t->algo < -1 || t->algo > 1 || t->proto < -1 || t->proto > 2 || t->nchannels < 0 ||
        t->nchannels > c.maxLanes || (t->nthreads != 0 && (t->nthreads < 64 || t->nthreads > 1024 || t->nthreads % 64)) ||
        t->chunkBytes % 16)
      return vcclInvalidArgument;
    c.apiTune.algo = t->algo;
    c.apiTune.proto = t->proto;
    c.apiTune.nchannels = t->nchannels;
    c.apiTune.nthreads = t->nthreads;
    c.apiTune.chunkBytes = t->chunkBytes;
    c.apiTune.direct = t->direct;
  }
  Coll x{};
  x.coll = (uint8_t)coll;
  x.dtype = (int)datatype;
  x.op = vcclSum;
  x.count = count;
  Plan p;
  vcclResult_t r = planColl(&c, x, &p, single != 0);
  if (r != vcclSuccess) return r;
  const int nlanes = p.split ? 8 * ((p.nchannels + 7) / 8) + p.nchannels : p.nchannels;
  vcclPlanInfo_t o{};
  o.algo = p.algo;
  o.proto = p.proto;
  o.nchannels = p.nchannels;
  o.nthreads = p.nthreads;
  o.direct = p.direct;
  o.nlanes = nlanes;
  o.nitems = nlanes;
  o.ncolls = 1;
  o.chunkBytes = (size_t)p.chunkBytes;
  o.grid = 8 * nranks * ((nlanes + 7) / 8);
  o.scope = p.scope;
  o.treeRanksPerNode = 1;
  o.ll128 = c.ll128 ? 1 : 0;
  *info = o;
  return vcclSuccess;
}

vcclResult_t vcclProbeXccIds(int n, int* ids) {
  if (n <= 0 || !ids) return vcclInvalidArgument;
  int* d = nullptr;
  VCCL_HIPCHECK(hipMalloc((void**)&d, (size_t)n * sizeof(int)));
  hipError_t e = vcclLaunchXccProbe(d, n, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(ids, d, (size_t)n * sizeof(int), hipMemcpyDeviceToHost);
  hipFree(d);
  if (e != hipSuccess) {
    logError("xcc probe", e, __FILE__, __LINE__);
    return vcclUnhandledHipError;
  }
  return vcclSuccess;
}

vcclResult_t vcclProbeLL128Tear(int pairs, int lines, int rounds, int scope, uint64_t* torn, uint64_t* checked) {
  if (pairs < 1 || pairs > 64 || lines < 1 || lines > 65536 || rounds < 1 || !torn || !checked)
    return vcclInvalidArgument;
  if (scope != SCOPE_DEVICE && scope != SCOPE_XCD) return vcclInvalidArgument;
  if (scope == SCOPE_XCD && pairs % 8) return vcclInvalidArgument;  // plain stores: each pair on one XCD
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return vcclUnhandledHipError;
  bool timedOut = false;
  hipError_t e = tearProbe(dev, pairs, lines, rounds, scope, 5000000, torn, checked, &timedOut);
  if (e != hipSuccess) {
    logError("tear probe", e, __FILE__, __LINE__);
    return vcclUnhandledHipError;
  }
  return timedOut ? vcclRemoteError : vcclSuccess;
}

}  // extern "C"
