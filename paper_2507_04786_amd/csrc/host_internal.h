// Host runtime internals: communicator sets ("cliques"), call matching,
// planning and launching.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <deque>
#include <string>
#include <vector>

#include "vccl.h"
#include "vccl_dev.h"

// device-side launchers (device.hip)
hipError_t vcclLaunchColl(const vccl::LaunchDesc& d, int grid, int block, hipStream_t stream, bool cooperative);
hipError_t vcclCollOccupancy(int block, int* blocksPerCU);
hipError_t vcclLaunchXccProbe(int* dIds, int n, hipStream_t stream);
hipError_t vcclLaunchServe(const vccl::ServeDesc& d, int grid, int block, hipStream_t stream);
hipError_t vcclServeOccupancy(int block, int* blocksPerCU);
hipError_t vcclScratchPtr(int device, char** ptr);
hipError_t vcclLaunchNoAllocPrep(char* base, const vccl::DevComm& comm, uint64_t ctrBytes, uint64_t llBytes,
                                 hipStream_t stream);
hipError_t vcclLaunchTearProbe(char* bufs, uint64_t* acks, int pairs, int lines, int rounds,
                               unsigned long long* counts, uint64_t maxTicks, uint32_t* failed, int scope,
                               hipStream_t stream);

namespace vccl {

struct Clique;

// One rank's call, waiting for the other ranks of its set.
struct Call {
  uint8_t coll;
  int dtype, op, root;
  size_t count;
  const void* send;
  void* recv;
  hipStream_t stream;
};

// A posted Send or Recv waiting for its partner.
struct P2pOp {
  void* buf;
  size_t count;
  int dtype;
  hipStream_t stream;
};

// A collective whose R per-rank calls have all arrived, or a matched
// point-to-point transfer (coll COLL_SENDRECV: root = sender, peer = receiver).
struct Coll {
  uint8_t coll;
  int dtype, op, root;
  size_t count;
  CollArgs args;
  hipStream_t streams[MAX_RANKS];
  int peer = 0;
};

struct Plan {
  int algo, proto, nchannels, nthreads, direct;
  uint64_t chunkBytes;
  int scope = SCOPE_DEVICE;
  bool split = false;  // tree channels run as concurrent up and down halves on two lanes
};

struct Tuning {
  int algo = -1, proto = -1, nchannels = 0, nthreads = 0, direct = -1;
  uint64_t chunkBytes = 0;
};

struct Clique {
  int nranks = 0;
  int device = 0;
  int maxLanes = 0;
  int numCUs = 0;
  double ticksPerUs = 100.0;
  DevComm host{};             // host copy of the device descriptor
  DevComm* dcomm = nullptr;   // device copy
  char* fifo[3] = {nullptr, nullptr, nullptr};
  char* treeFifo[3] = {nullptr, nullptr, nullptr};
  uint64_t* ctr = nullptr;
  uint32_t* hAbort = nullptr; // pinned
  uint32_t* hError = nullptr; // pinned
  // group / work-list staging
  // a grouped launch's work list: items, lane starts and pointer tables in
  // one device buffer, laid out as workLayout gives, filled from a pinned
  // staging copy of the same layout by one copy
  char* dWork = nullptr;
  size_t itemCap = 0, argCap = 0;
  void* hStage[2] = {nullptr, nullptr};
  size_t stageCap = 0;
  hipEvent_t stageEvent[2] = {nullptr, nullptr};
  int stageNext = 0;
  uint64_t* dStamps = nullptr;
  uint64_t* dProfile = nullptr;   // per-workgroup records of profiling launches
  bool profile = false;
  int lastLanes = 0;              // lanes of the most recent launch
  size_t stampCap = 0;
  int lastStampColls = 0;
  hipEvent_t lastLaunchDone = nullptr;
  std::vector<hipEvent_t> joinEvents;
  // matching
  std::vector<std::deque<Call>> pending;  // per rank
  // point-to-point: [sender * nranks + receiver] posted sends and receives,
  // matched in order per ordered pair
  std::vector<std::deque<P2pOp>> p2pSends, p2pRecvs;
  // tuning
  Tuning envTune, apiTune;
  bool cooperative = true;
  int xcdMap = 1;
  vcclPlanInfo_t lastPlan{};
  int destroyedHandles = 0;
  bool aborted = false;
  std::vector<vcclComm*> handles;
  int occupancy[17] = {0};    // blocks per CU for nthreads = 64 * index
  bool serving = false;       // a persistent serving kernel owns the lanes
  uint64_t deviceScopeBytes = 0;  // Simple AllGathers and Send/Recv copies this large use device scope
  bool treeSplit = true;          // split Simple tree channels into concurrent halves
  int ranksPerNode = 1;           // tree topology: chains of this many ranks, trees across them
  bool ll128 = true;              // LL128 may be planned (its tear test passed on this device)
  int nrings = 1;                 // ring orders (host.ringRank / host.ringPos); channel c follows c % nrings
  uint64_t* claim = nullptr;  // per-XCD role counters (device)
  uint64_t claimBase = 0;     // role claims of all launches so far, per XCD
};

Clique* cliqueOf(vcclComm_t comm);
int rankOf(vcclComm_t comm);

// host_comm.cpp
// rings: nrings rows of nranks ranks (ring orders, validated by the caller), or
// null for the identity ring
vcclResult_t cliqueCreate(int nranks, int device, int nrings, const int* rings, Clique** out);
int defaultLaneLimit(int numCUs, int nranks);
void cliqueFree(Clique* c);
vcclResult_t cliqueEnsureTreeFifos(Clique* c, int proto);
uint64_t cliqueTreeFifoBytes(const Clique* c, int proto);
uint64_t cliqueRingFifoBytes(const Clique* c, int proto);
vcclResult_t cliqueEnsureWorkCapacity(Clique* c, size_t items, size_t args, size_t stamps);
// Work-list layout for `items` items: byte offsets of the lane starts and of
// the pointer tables, each 256-byte aligned after the items
struct WorkLayout {
  size_t laneOff, argsOff;
};
WorkLayout workLayout(size_t items);
int cliqueOccupancy(Clique* c, int nthreads);
void buildTrees(int nranks, int ranksPerNode, int8_t parent[2][MAX_RANKS], int8_t child[2][MAX_RANKS][2],
                int8_t childIdx[2][MAX_RANKS], int8_t nchild[2][MAX_RANKS]);

// host_plan.cpp
size_t dtypeBytes(int dtype);
uint64_t collSizeBytes(uint8_t coll, size_t count, int dtype, int nranks);
// single: the collective is launched alone (a tree may then be split).
vcclResult_t planColl(Clique* c, const Coll& coll, Plan* plan, bool single = false);
// Channel regions [start, end) in units: per = roundUp(ceil(n / C), align).
void channelRange(uint64_t n, int nchannels, uint64_t align, int ch, uint64_t* start, uint64_t* count);
void fillItems(const Clique* c, const Coll& coll, const Plan& plan, uint32_t argsIndex, uint32_t doneIndex,
               std::vector<WorkItem>* items);
double estimateCost(const Clique* c, const WorkItem& w);
int p2pLaneCap(const Clique* c);

// host_api.cpp
vcclResult_t launchColls(Clique* c, const std::vector<Coll>& colls);
hipError_t tearProbe(int device, int pairs, int lines, int rounds, int scope, uint64_t maxUs, uint64_t* torn,
                     uint64_t* checked, bool* timedOut);
bool ll128Allowed(int device);

// env helpers
std::string envStr(const char* name);
long envLong(const char* name, long dflt);

#define VCCL_HIPCHECK(cmd)                                   \
  do {                                                       \
    hipError_t e_ = (cmd);                                   \
    if (e_ != hipSuccess) {                                  \
      vccl::logError(#cmd, e_, __FILE__, __LINE__);          \
      return vcclUnhandledHipError;                          \
    }                                                        \
  } while (0)

void logError(const char* what, hipError_t e, const char* file, int line);
void logInfo(const char* fmt, ...);

}  // namespace vccl

struct vcclComm {
  vccl::Clique* clique;
  int rank;
  bool destroyed;
};
