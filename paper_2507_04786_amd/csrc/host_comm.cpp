// Communicator sets: FIFO and counter allocation, ring and double binary tree
// (Section II-C), occupancy, staging buffers.
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "host_internal.h"

namespace vccl {

void logError(const char* what, hipError_t e, const char* file, int line) {
  fprintf(stderr, "vccl: %s failed: %s (%s:%d)\n", what, hipGetErrorString(e), file, line);
}

void logInfo(const char* fmt, ...) {
  static int level = -1;
  if (level < 0) {
    std::string v = envStr("VCCL_DEBUG");
    level = (v == "INFO" || v == "TRACE") ? 1 : 0;
  }
  if (!level) return;
  va_list ap;
  va_start(ap, fmt);
  fprintf(stderr, "vccl: ");
  vfprintf(stderr, fmt, ap);
  fprintf(stderr, "\n");
  va_end(ap);
}

std::string envStr(const char* name) {
  const char* v = getenv(name);
  return v ? std::string(v) : std::string();
}

long envLong(const char* name, long dflt) {
  const char* v = getenv(name);
  if (!v || !*v) return dflt;
  char* end = nullptr;
  long x = strtol(v, &end, 0);
  return (end && *end == '\0') ? x : dflt;
}

// Double binary tree.  The paper fixes only its properties (no rank inner in
// both trees, at most one rank a leaf in both; the second tree mirrors the
// first for an even rank count, shifts it by one position for an odd one).
// Tree 0 over positions 0..R-1: position 0 is the root with one child, the
// largest power of two below R; position q (lowest set bit b) has parent
// (q - b) | 2b, or q - b when that is >= R; its children are q - b/2 and the
// first of q + b/2, q + b/4, ..., q + 1 below R.
// ranksPerNode P > 1: node n = ranks n*P .. n*P+P-1 forms a chain (tree 0:
// local 0 <- 1 <- ... <- P-1, tree 1 the reverse), the nodes form the double
// binary tree, a node's chain head sends to its parent node, which takes its
// first node child at its head and its second at the next rank of its chain
// (at most two children per rank; the chain child first).
void buildTrees(int R, int ranksPerNode, int8_t parent[2][MAX_RANKS], int8_t child[2][MAX_RANKS][2],
                int8_t childIdx[2][MAX_RANKS], int8_t nchild[2][MAX_RANKS]) {
  if (ranksPerNode > 1 && R % ranksPerNode == 0) {
    const int P = ranksPerNode, N = R / P;
    int8_t np[2][MAX_RANKS], nc[2][MAX_RANKS][2], nci[2][MAX_RANKS], nn[2][MAX_RANKS];
    buildTrees(N, 1, np, nc, nci, nn);
    for (int t = 0; t < 2; ++t) {
      auto at = [&](int node, int pos) { return node * P + (t == 0 ? pos : P - 1 - pos); };
      for (int r = 0; r < R; ++r) {
        parent[t][r] = -1;
        nchild[t][r] = 0;
        child[t][r][0] = child[t][r][1] = -1;
      }
      for (int n = 0; n < N; ++n)
        for (int i = 1; i < P; ++i) {
          parent[t][at(n, i)] = (int8_t)at(n, i - 1);
          child[t][at(n, i - 1)][nchild[t][at(n, i - 1)]++] = (int8_t)at(n, i);
        }
      for (int n = 0; n < N; ++n)
        for (int j = 0; j < nn[t][n]; ++j) {
          const int m = nc[t][n][j], where = at(n, j);
          parent[t][at(m, 0)] = (int8_t)where;
          child[t][where][nchild[t][where]++] = (int8_t)at(m, 0);
        }
      for (int r = 0; r < R; ++r)
        for (int k = 0; k < nchild[t][r]; ++k) childIdx[t][child[t][r][k]] = (int8_t)k;
      for (int r = 0; r < R; ++r)
        if (parent[t][r] < 0) childIdx[t][r] = 0;
    }
    return;
  }
  int pPar[MAX_RANKS], pKids[MAX_RANKS][2], pN[MAX_RANKS];
  for (int q = 0; q < R; ++q) {
    pPar[q] = -1;
    pN[q] = 0;
    pKids[q][0] = pKids[q][1] = -1;
  }
  int top = 1;
  while (top * 2 < R) top *= 2;
  if (R > 1) {
    pKids[0][0] = top;
    pN[0] = 1;
  }
  for (int q = 1; q < R; ++q) {
    int b = q & -q;
    int up = (q - b) | (2 * b);
    if (up >= R) up = q - b;
    pPar[q] = up;
    if (b > 1) {
      pKids[q][pN[q]++] = q - b / 2;
      for (int h = b / 2; h >= 1; h /= 2) {
        if (q + h < R) {
          pKids[q][pN[q]++] = q + h;
          break;
        }
      }
    }
  }
  for (int t = 0; t < 2; ++t) {
    int rankAt[MAX_RANKS];
    for (int q = 0; q < R; ++q) rankAt[q] = (t == 0) ? q : ((R % 2 == 0) ? R - 1 - q : (q + 1) % R);
    for (int q = 0; q < R; ++q) {
      int r = rankAt[q];
      parent[t][r] = (int8_t)(pPar[q] < 0 ? -1 : rankAt[pPar[q]]);
      nchild[t][r] = (int8_t)pN[q];
      child[t][r][0] = (int8_t)(pN[q] > 0 ? rankAt[pKids[q][0]] : -1);
      child[t][r][1] = (int8_t)(pN[q] > 1 ? rankAt[pKids[q][1]] : -1);
      childIdx[t][r] = 0;
    }
    for (int r = 0; r < R; ++r)
      for (int k = 0; k < nchild[t][r]; ++k) childIdx[t][child[t][r][k]] = (int8_t)k;
  }
}

int defaultLaneLimit(int numCUs, int nranks) {
  return std::max(32, std::min(MAX_LANES, (2 * numCUs / nranks) / 8 * 8));
}

vcclResult_t cliqueCreate(int nranks, int device, int nrings, const int* rings, Clique** out) {
  Clique* c = new Clique();
  c->nranks = nranks;
  c->nrings = rings ? nrings : 1;
  c->device = device;
  c->pending.resize(nranks);
  c->p2pSends.resize((size_t)nranks * nranks);
  c->p2pRecvs.resize((size_t)nranks * nranks);
  auto fail = [&](hipError_t e, const char* what) {
    logError(what, e, __FILE__, __LINE__);
    cliqueFree(c);
    return vcclUnhandledHipError;
  };
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return fail(e, "hipSetDevice");
  e = hipDeviceGetAttribute(&c->numCUs, hipDeviceAttributeMultiprocessorCount, device);
  if (e != hipSuccess) return fail(e, "hipDeviceGetAttribute");
  // lane limit: enough lanes to give every CU two workgroups (lanes come in
  // eights, one per XCD), at least 32 and at most MAX_LANES: 64 up to 8
  // ranks, 40 at 12, 32 at 16.  FIFO memory scales with lanes x ranks (at 8
  // ranks and 64 lanes, 3.5 GiB of ring FIFOs).  4 ranks measured 20 %
  // faster at 64 lanes than at 32; at 8 ranks, LL at 64 MiB 0.88 -> 0.82 ms
  // with 64 lanes of 512 threads, and grouped batches run on more lanes.
  c->maxLanes = (int)envLong("VCCL_MAX_CHANNELS", defaultLaneLimit(c->numCUs, nranks));
  if (c->maxLanes < 1) c->maxLanes = 1;
  if (c->maxLanes > MAX_LANES) c->maxLanes = MAX_LANES;
  int wallKHz = 0;
  if (hipDeviceGetAttribute(&wallKHz, hipDeviceAttributeWallClockRate, device) == hipSuccess && wallKHz > 0)
    c->ticksPerUs = wallKHz / 1000.0;

  const uint64_t nconn = (uint64_t)c->maxLanes * nranks * NCONN;
  const uint64_t slot[3] = {(uint64_t)envLong("VCCL_SIMPLE_SLOT_BYTES", SLOT_BYTES_SIMPLE), SLOT_BYTES_LL,
                            SLOT_BYTES_LL128};
  c->host.treeSlotBytes[PROTO_SIMPLE] = (uint64_t)envLong("VCCL_TREE_SIMPLE_SLOT_BYTES", TREE_SLOT_BYTES_SIMPLE);
  c->host.treeSlotBytes[PROTO_LL] = TREE_SLOT_BYTES_LL;
  c->host.treeSlotBytes[PROTO_LL128] = TREE_SLOT_BYTES_LL128;
  for (int p = 0; p < 3; ++p) {
    // ring connections, one block of lanes x ranks per ring order
    const uint64_t bytes = (uint64_t)c->nrings * c->maxLanes * nranks * NSLOTS * slot[p];
    e = hipMalloc((void**)&c->fifo[p], bytes);
    if (e != hipSuccess) return fail(e, "hipMalloc(fifo)");
    if (p != PROTO_SIMPLE) {
      // flags start at 0; the first flag a receiver waits for is 1
      e = hipMemset(c->fifo[p], 0, bytes);
      if (e != hipSuccess) return fail(e, "hipMemset(fifo)");
    }
    c->host.fifo[p] = c->fifo[p];
    c->host.slotBytes[p] = slot[p];
  }
  e = hipMalloc((void**)&c->ctr, nconn * CTR_RECORD_U64 * sizeof(uint64_t));
  if (e != hipSuccess) return fail(e, "hipMalloc(counters)");
  e = hipMemset(c->ctr, 0, nconn * CTR_RECORD_U64 * sizeof(uint64_t));
  if (e != hipSuccess) return fail(e, "hipMemset(counters)");
  e = hipMalloc((void**)&c->claim, 8 * CLAIM_STRIDE_U64 * sizeof(uint64_t));
  if (e != hipSuccess) return fail(e, "hipMalloc(claim)");
  e = hipMemset(c->claim, 0, 8 * CLAIM_STRIDE_U64 * sizeof(uint64_t));
  if (e != hipSuccess) return fail(e, "hipMemset(claim)");
  c->host.claim = c->claim;
  e = hipHostMalloc((void**)&c->hAbort, 256, hipHostMallocCoherent);
  if (e != hipSuccess) return fail(e, "hipHostMalloc(abort)");
  e = hipHostMalloc((void**)&c->hError, 256, hipHostMallocCoherent);
  if (e != hipSuccess) return fail(e, "hipHostMalloc(error)");
  *c->hAbort = 0;
  *c->hError = 0;

  c->host.nranks = nranks;
  c->host.maxLanes = c->maxLanes;
  const double timeoutUs = (double)envLong("VCCL_TIMEOUT_US", 5000000);
  c->host.timeoutTicks = (uint64_t)(timeoutUs * c->ticksPerUs);
  c->host.deadMask = 0;
  c->host.scope = SCOPE_DEVICE;
  c->host.ctr = c->ctr;
  c->host.abortFlag = c->hAbort;
  c->host.errorWord = c->hError;
  memset(c->host.parent, -1, sizeof(c->host.parent));
  memset(c->host.child, -1, sizeof(c->host.child));
  // tree topology: VCCL_TREE_RANKS_PER_NODE groups consecutive ranks into
  // "nodes" (chains within a node, the double binary tree across them)
  c->ranksPerNode = (int)envLong("VCCL_TREE_RANKS_PER_NODE", 1);
  if (c->ranksPerNode < 1 || c->ranksPerNode > nranks || nranks % c->ranksPerNode) {
    logInfo("VCCL_TREE_RANKS_PER_NODE=%d does not divide %d ranks; using 1", c->ranksPerNode, nranks);
    c->ranksPerNode = 1;
  }
  buildTrees(nranks, c->ranksPerNode, c->host.parent, c->host.child, c->host.childIdx, c->host.nchild);
  // ring orders (Section II-C: every channel has its ring, set up once)
  c->host.nrings = c->nrings;
  memset(c->host.ringRank, 0, sizeof(c->host.ringRank));
  memset(c->host.ringPos, 0, sizeof(c->host.ringPos));
  for (int k = 0; k < c->nrings; ++k)
    for (int q = 0; q < nranks; ++q) {
      const int rk = rings ? rings[k * nranks + q] : q;
      c->host.ringRank[k][q] = (int8_t)rk;
      c->host.ringPos[k][rk] = (int8_t)q;
    }
  e = hipMalloc((void**)&c->dcomm, sizeof(DevComm));
  if (e != hipSuccess) return fail(e, "hipMalloc(devcomm)");
  e = hipMemcpy(c->dcomm, &c->host, sizeof(DevComm), hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(e, "hipMemcpy(devcomm)");
  e = hipEventCreateWithFlags(&c->lastLaunchDone, hipEventDisableTiming);
  if (e != hipSuccess) return fail(e, "hipEventCreate");
  for (int i = 0; i < 2; ++i) {
    e = hipEventCreateWithFlags(&c->stageEvent[i], hipEventDisableTiming);
    if (e != hipSuccess) return fail(e, "hipEventCreate");
  }
  c->joinEvents.resize(2 * MAX_RANKS + 2, nullptr);
  for (auto& ev : c->joinEvents) {
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return fail(e, "hipEventCreate");
  }
  e = hipDeviceSynchronize();
  if (e != hipSuccess) return fail(e, "hipDeviceSynchronize");

  // tuning from the environment (overridden by vcclCommSetTuning)
  std::string a = envStr("VCCL_ALGO"), p = envStr("VCCL_PROTO");
  if (a == "ring" || a == "Ring") c->envTune.algo = ALGO_RING;
  if (a == "tree" || a == "Tree") c->envTune.algo = ALGO_TREE;
  if (p == "simple" || p == "Simple") c->envTune.proto = PROTO_SIMPLE;
  if (p == "ll" || p == "LL") c->envTune.proto = PROTO_LL;
  if (p == "ll128" || p == "LL128") c->envTune.proto = PROTO_LL128;
  c->envTune.nchannels = (int)envLong("VCCL_NCHANNELS", 0);
  c->envTune.nthreads = (int)envLong("VCCL_NTHREADS", 0);
  c->envTune.chunkBytes = (uint64_t)envLong("VCCL_CHUNK_BYTES", 0);
  c->envTune.direct = (int)envLong("VCCL_DIRECT", -1);
  // plain launches by default: the planner keeps every launch within what the
  // device holds at once (grid <= CUs * occupancy), and every wait is bounded
  c->cooperative = envStr("VCCL_LAUNCH") == "cooperative";
  c->xcdMap = (int)envLong("VCCL_XCD_MAP", 1);
  // XCD scope (plain stores into the XCD's L2, sc1 loads) needs the lane map,
  // which claims every lane's roles on one XCD at kernel start; it is the
  // default then, and VCCL_SCOPE=device keeps every store device-coherent
  // XCD scope measured faster for every collective and size (Broadcast up
  // to 27 %, Reduce up to 13 %: a chain reads back what its predecessor just
  // wrote, from the shared L2), except Simple AllGathers from 16 MiB, which
  // ran up to 11 % faster with device-coherent stores.  Send/Recv copies
  // take device scope from the same size.
  c->deviceScopeBytes = (uint64_t)envLong("VCCL_DEVICE_SCOPE_BYTES", 16 << 20);
  c->treeSplit = envLong("VCCL_TREE_SPLIT", 1) != 0;
  // Section III-C: LL128 only where its 128-byte lines are never seen torn
  c->ll128 = ll128Allowed(device);
  if (c->xcdMap && envStr("VCCL_SCOPE") != "device") {
    c->host.scope = SCOPE_XCD;
    e = hipMemcpy(c->dcomm, &c->host, sizeof(DevComm), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(e, "hipMemcpy(devcomm)");
  }
  logInfo("traffic scope %s, LL128 %s", c->host.scope == SCOPE_XCD ? "xcd" : "device", c->ll128 ? "on" : "off");
  *out = c;
  return vcclSuccess;
}

void cliqueFree(Clique* c) {
  if (!c) return;
  hipSetDevice(c->device);
  hipDeviceSynchronize();
  for (int p = 0; p < 3; ++p) {
    if (c->fifo[p]) hipFree(c->fifo[p]);
    if (c->treeFifo[p]) hipFree(c->treeFifo[p]);
  }
  if (c->ctr) hipFree(c->ctr);
  if (c->claim) hipFree(c->claim);
  if (c->dcomm) hipFree(c->dcomm);
  if (c->dWork) hipFree(c->dWork);
  if (c->dStamps) hipFree(c->dStamps);
  if (c->dProfile) hipFree(c->dProfile);
  for (int i = 0; i < 2; ++i) {
    if (c->hStage[i]) hipHostFree(c->hStage[i]);
    if (c->stageEvent[i]) hipEventDestroy(c->stageEvent[i]);
  }
  if (c->lastLaunchDone) hipEventDestroy(c->lastLaunchDone);
  for (auto ev : c->joinEvents)
    if (ev) hipEventDestroy(ev);
  if (c->hAbort) hipHostFree(c->hAbort);
  if (c->hError) hipHostFree(c->hError);
  for (auto* h : c->handles) delete h;
  delete c;
}

// Tree connections of a protocol are allocated on the first tree launch
// under that protocol (they are 6 of the 7 connections of every lane and
// rank, and only tree AllReduce uses them).
vcclResult_t cliqueEnsureTreeFifos(Clique* c, int proto) {
  if (c->treeFifo[proto]) return vcclSuccess;
  VCCL_HIPCHECK(hipDeviceSynchronize());
  const uint64_t bytes = cliqueTreeFifoBytes(c, proto);
  VCCL_HIPCHECK(hipMalloc((void**)&c->treeFifo[proto], bytes));
  if (proto != PROTO_SIMPLE) VCCL_HIPCHECK(hipMemset(c->treeFifo[proto], 0, bytes));
  c->host.treeFifo[proto] = c->treeFifo[proto];
  VCCL_HIPCHECK(hipMemcpy(c->dcomm, &c->host, sizeof(DevComm), hipMemcpyHostToDevice));
  VCCL_HIPCHECK(hipDeviceSynchronize());
  logInfo("tree FIFOs, protocol %d: %.2f GiB", proto, (double)bytes / (1u << 30));
  return vcclSuccess;
}

uint64_t cliqueTreeFifoBytes(const Clique* c, int proto) {
  return (uint64_t)c->maxLanes * c->nranks * NTREE_CONN * NSLOTS * c->host.treeSlotBytes[proto];
}

uint64_t cliqueRingFifoBytes(const Clique* c, int proto) {
  return (uint64_t)c->nrings * c->maxLanes * c->nranks * NSLOTS * c->host.slotBytes[proto];
}

WorkLayout workLayout(size_t items) {
  WorkLayout w;
  w.laneOff = (items * sizeof(WorkItem) + 255) / 256 * 256;
  w.argsOff = w.laneOff + ((MAX_LANES + 1) * sizeof(uint32_t) + 255) / 256 * 256;
  return w;
}

vcclResult_t cliqueEnsureWorkCapacity(Clique* c, size_t items, size_t args, size_t stamps) {
  if (items > c->itemCap || args > c->argCap) {
    const size_t icap = items > c->itemCap ? (items < 256 ? 256 : items * 2) : c->itemCap;
    const size_t acap = args > c->argCap ? (args < 128 ? 128 : args * 2) : c->argCap;
    const size_t bytes = workLayout(icap).argsOff + acap * sizeof(CollArgs);
    if (c->dWork) {
      VCCL_HIPCHECK(hipDeviceSynchronize());
      VCCL_HIPCHECK(hipFree(c->dWork));
      c->dWork = nullptr;
    }
    VCCL_HIPCHECK(hipMalloc((void**)&c->dWork, bytes));
    for (int i = 0; i < 2; ++i) {
      if (c->hStage[i]) {
        VCCL_HIPCHECK(hipEventSynchronize(c->stageEvent[i]));
        VCCL_HIPCHECK(hipHostFree(c->hStage[i]));
        c->hStage[i] = nullptr;
      }
      VCCL_HIPCHECK(hipHostMalloc(&c->hStage[i], bytes, 0));
    }
    c->itemCap = icap;
    c->argCap = acap;
    c->stageCap = bytes;
  }
  if (stamps > c->stampCap) {
    size_t cap = stamps < 1024 ? 1024 : stamps * 2;
    if (c->dStamps) {
      VCCL_HIPCHECK(hipDeviceSynchronize());
      VCCL_HIPCHECK(hipFree(c->dStamps));
    }
    VCCL_HIPCHECK(hipMalloc((void**)&c->dStamps, cap * sizeof(uint64_t)));
    c->stampCap = cap;
  }
  return vcclSuccess;
}

int cliqueOccupancy(Clique* c, int nthreads) {
  int idx = nthreads / 64;
  if (idx < 1 || idx > 16) return 0;
  if (c->occupancy[idx] == 0) {
    int n = 0;
    if (vcclCollOccupancy(nthreads, &n) != hipSuccess) n = 0;
    c->occupancy[idx] = n > 0 ? n : -1;
  }
  return c->occupancy[idx] > 0 ? c->occupancy[idx] : 0;
}

}  // namespace vccl
