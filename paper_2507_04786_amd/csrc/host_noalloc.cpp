// The allocation-free AllReduce: a ring AllReduce of R virtual ranks with no
// communicator set, whose FIFOs, counters and descriptor live in a
// file-scope device array (device.hip) instead of memory the library
// allocates.  For callers that cannot allocate device memory.
#include <algorithm>
#include <cstring>

#include "host_internal.h"

using namespace vccl;

namespace {

// Per device: the scratch address (looked up once, with the device current)
// and the kernel's occupancy per workgroup size.
struct NoAllocDevice {
  bool ready = false;
  char* base = nullptr;
  int numCUs = 0;
  double ticksPerUs = 100.0;
  int occupancy[17] = {0};
};
NoAllocDevice gNoAlloc[64];

}  // namespace

extern "C" vcclResult_t vcclAllReduceNoAlloc(const void* const* sendbuffs, void* const* recvbuffs, int nranks,
                                             size_t count, vcclDataType_t datatype, vcclRedOp_t op, void* stream,
                                             vcclPlanInfo_t* plan) {
  if (!sendbuffs || !recvbuffs || nranks < 2 || nranks > VCCL_MAX_RANKS) return vcclInvalidArgument;
  if (datatype < vcclInt32 || datatype > vcclBfloat16 || op < vcclSum || op > vcclMax) return vcclInvalidArgument;
  if (count > ((size_t)1 << 40)) return vcclInvalidArgument;
  const size_t E = dtypeBytes(datatype);
  for (int r = 0; r < nranks; ++r) {
    if (count > 0 && (!sendbuffs[r] || !recvbuffs[r])) return vcclInvalidArgument;
    if (((uintptr_t)sendbuffs[r] % E) || ((uintptr_t)recvbuffs[r] % E)) return vcclInvalidArgument;
  }
  if (plan) memset(plan, 0, sizeof(*plan));
  if (count == 0) return vcclSuccess;
  int dev = 0;
  VCCL_HIPCHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return vcclInvalidArgument;
  NoAllocDevice& nd = gNoAlloc[dev];
  if (!nd.ready) {
    VCCL_HIPCHECK(vcclScratchPtr(dev, &nd.base));
    VCCL_HIPCHECK(hipDeviceGetAttribute(&nd.numCUs, hipDeviceAttributeMultiprocessorCount, dev));
    int wallKHz = 0;
    if (hipDeviceGetAttribute(&wallKHz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && wallKHz > 0)
      nd.ticksPerUs = wallKHz / 1000.0;
    nd.ready = true;
  }
  const int R = nranks;
  // the planner on a set of R ranks whose lane limit keeps lanes x ranks
  // within the scratch's connections; ring only (no tree FIFOs), Simple or
  // LL (no LL128 FIFOs), slots of the scratch's sizes
  Clique c;
  c.nranks = R;
  c.device = dev;
  c.numCUs = nd.numCUs;
  c.maxLanes = (int)std::min<uint64_t>(NA_MAX_LANES, NA_CONNS / (uint64_t)R);
  std::copy(nd.occupancy, nd.occupancy + 17, c.occupancy);
  c.host.scope = SCOPE_XCD;
  c.host.slotBytes[PROTO_SIMPLE] = NA_SLOT_SIMPLE;
  c.host.slotBytes[PROTO_LL] = NA_SLOT_LL;
  c.host.slotBytes[PROTO_LL128] = 0;
  c.ll128 = false;
  c.deviceScopeBytes = 16 << 20;
  c.apiTune.algo = ALGO_RING;
  Coll x{};
  x.coll = COLL_ALLREDUCE;
  x.dtype = (int)datatype;
  x.op = (int)op;
  x.count = count;
  for (int r = 0; r < R; ++r) {
    x.args.send[r] = (const char*)sendbuffs[r];
    x.args.recv[r] = (char*)recvbuffs[r];
  }
  Plan p;
  vcclResult_t res = planColl(&c, x, &p, true);
  std::copy(c.occupancy, c.occupancy + 17, nd.occupancy);
  if (res != vcclSuccess) return res;
  if (p.algo != ALGO_RING || (p.proto != PROTO_SIMPLE && p.proto != PROTO_LL) || p.nchannels < 1 ||
      p.nchannels > c.maxLanes || (uint64_t)p.nchannels * R > NA_CONNS)
    return vcclInternalError;
  const int C = p.nchannels;
  const int grid = 8 * R * ((C + 7) / 8);
  const int occ = cliqueOccupancy(&c, p.nthreads);
  if (occ <= 0 || grid > c.numCUs * occ) return vcclInternalError;

  DevComm dc{};
  dc.nranks = R;
  dc.maxLanes = c.maxLanes;
  dc.timeoutTicks = (uint64_t)(5.0e6 * nd.ticksPerUs);
  dc.scope = SCOPE_XCD;
  dc.fifo[PROTO_SIMPLE] = nd.base + NA_OFF_FIFO_SIMPLE;
  dc.fifo[PROTO_LL] = nd.base + NA_OFF_FIFO_LL;
  dc.slotBytes[PROTO_SIMPLE] = NA_SLOT_SIMPLE;
  dc.slotBytes[PROTO_LL] = NA_SLOT_LL;
  // ring only: no tree connections (treeFifo and treeSlotBytes stay zero)
  dc.ctr = (uint64_t*)(nd.base + NA_OFF_CTR);
  dc.abortFlag = (uint32_t*)(nd.base + NA_OFF_WORDS);
  dc.errorWord = (uint32_t*)(nd.base + NA_OFF_WORDS + 128);
  dc.claim = (uint64_t*)(nd.base + NA_OFF_CLAIM);
  memset(dc.parent, -1, sizeof(dc.parent));
  memset(dc.child, -1, sizeof(dc.child));
  dc.nrings = 1;  // the identity ring
  for (int q = 0; q < R; ++q) {
    dc.ringRank[0][q] = (int8_t)q;
    dc.ringPos[0][q] = (int8_t)q;
  }

  // the connections this launch uses: (lane * R + receiver) for lane < C
  const uint64_t conns = (uint64_t)C * R;
  const uint64_t ctrBytes = conns * NCONN * CTR_RECORD_U64 * sizeof(uint64_t);
  const uint64_t llBytes = p.proto == PROTO_LL ? conns * NSLOTS * NA_SLOT_LL : 0;

  LaunchDesc d;
  memset((void*)&d, 0, sizeof(d));
  d.comm = (const DevComm*)(nd.base + NA_OFF_COMM);
  d.items = nullptr;
  d.nlanes = (uint32_t)C;
  d.nranks = (uint32_t)R;
  d.xcdMap = 1;
  d.perXcd = (uint32_t)(R * ((C + 7) / 8));
  d.claimBase = 0;  // the claim counters were zeroed for this launch
  d.inlineArgs = x.args;
  const uint64_t ub = E, n = count, align = 16 / ub;
  for (int ch = 0; ch < C; ++ch) {
    WorkItem& w = d.inlineItems[ch];
    w.coll = COLL_ALLREDUCE;
    w.algo = ALGO_RING;
    w.proto = (uint8_t)p.proto;
    w.dtype = (uint8_t)(datatype == vcclInt32 ? DT_I32 : datatype == vcclFloat32 ? DT_F32 : DT_BF16);
    w.op = (uint8_t)(op == vcclMax ? OP_MAX : OP_SUM);
    w.direct = (uint8_t)p.direct;
    w.argsIndex = 0;
    w.doneIndex = 0xFFFFFFFFu;
    w.unitBytes = (uint32_t)ub;
    w.elemBytes = (uint32_t)E;
    w.scope = (uint8_t)p.scope;
    w.count = n;
    channelRange(n, C, align, ch, &w.chOffset, &w.chCount);
    w.chunk = p.chunkBytes / ub;
  }
  hipStream_t st = (hipStream_t)stream;
  VCCL_HIPCHECK(vcclLaunchNoAllocPrep(nd.base, dc, ctrBytes, llBytes, st));
  VCCL_HIPCHECK(vcclLaunchColl(d, grid, p.nthreads, st, false));
  if (plan) {
    plan->algo = p.algo;
    plan->proto = p.proto;
    plan->nchannels = C;
    plan->nthreads = p.nthreads;
    plan->direct = p.direct;
    plan->nlanes = C;
    plan->nitems = C;
    plan->ncolls = 1;
    plan->chunkBytes = (size_t)p.chunkBytes;
    plan->grid = grid;
    plan->scope = p.scope;
    plan->treeRanksPerNode = 1;
    plan->ll128 = 0;
  }
  return vcclSuccess;
}
