// Structures shared by the host runtime and the gfx950 kernels.
//
// Memory layout in HBM (one communicator set, "clique"):
//   * FIFOs: for every protocol p, one region for the ring connections,
//       maxLanes * nranks connections of NSLOTS slots * slotBytes[p] each
//       (index lane * nranks + receivingRank), and one for the tree
//       connections (6 per lane and rank, index (lane * nranks + rank) * 6 +
//       kind - 1), allocated on the first tree launch.
//     Connection id = (lane * nranks + receivingRank) * NCONN + kind, where kind
//       0      ring: from the ring predecessor
//       1, 2   tree 0: upward from the receiver's first / second child
//       3      tree 0: downward from the receiver's parent
//       4..6   the same three for tree 1.
//     A FIFO lives with its receiver (the sender stores into it).
//   * Counters: one 256-byte record per connection; `tail` (steps published by
//     the sender) at byte 0 and `head` (steps consumed by the receiver) at byte
//     128, so the two writers never share a cache line.
//   * Step numbering is per connection and counts every step the connection
//     ever took, across protocols and launches; slot = step % NSLOTS.
#pragma once
#include <stdint.h>

namespace vccl {

enum : uint8_t { COLL_ALLREDUCE = 0, COLL_BROADCAST = 1, COLL_REDUCE = 2, COLL_ALLGATHER = 3, COLL_REDUCESCATTER = 4 };
enum : uint8_t { ALGO_RING = 0, ALGO_TREE = 1 };
enum : uint8_t { PROTO_SIMPLE = 0, PROTO_LL = 1, PROTO_LL128 = 2 };
enum : uint8_t { DT_I32 = 0, DT_F32 = 1, DT_BF16 = 2, DT_U8 = 3 };
enum : uint8_t { OP_SUM = 0, OP_MAX = 1, OP_COPY = 2 };

constexpr int NSLOTS = 8;
constexpr int NCONN = 7;
constexpr int MAX_RANKS = 16;
constexpr int MAX_LANES = 32;
constexpr int MAX_INLINE = 32;
constexpr uint32_t SLOT_BYTES_SIMPLE = 512u * 1024u;
constexpr uint32_t SLOT_BYTES_LL = 32u * 1024u;
constexpr uint32_t SLOT_BYTES_LL128 = 600u * 1024u;
constexpr uint32_t LL128_LINE = 128, LL128_DATA = 120;
constexpr uint32_t CTR_RECORD_U64 = 32;  // 256 B per connection
constexpr uint32_t CTR_HEAD_U64 = 16;    // head at +128 B

// Simple-protocol synchronisation modes.
//  SIMPLE_FENCE: plain stores, device-scope release fence (L2 write-back)
//    before the tail store; device-scope acquire (L2 invalidate) after it.
//  SIMPLE_COHERENT: the chunk itself is stored and loaded with device-scope
//    coherent accesses (sc1, as relaxed device-scope atomics are), so a drain
//    of the stores before the tail store orders them and no cache-wide
//    write-back or invalidate is needed.
constexpr uint32_t SIMPLE_FENCE = 0, SIMPLE_COHERENT = 1;

// device-side error codes (bit flags in the error word)
constexpr uint32_t ERR_TIMEOUT = 1u, ERR_ABORT = 2u;

struct DevComm {
  int32_t nranks;
  int32_t maxLanes;
  uint64_t timeoutTicks;        // device wall-clock ticks a single wait may take
  uint32_t deadMask;            // test hook: ranks whose workgroups do nothing
  uint32_t simpleMode;          // Simple protocol synchronisation, SIMPLE_* below
  char* fifo[3];                // ring connections, per protocol
  char* treeFifo[3];            // tree connections, per protocol (null until first used)
  uint64_t slotBytes[3];
  uint64_t* ctr;                // counters
  uint32_t* abortFlag;          // host-pinned, written by the host
  uint32_t* errorWord;          // host-pinned, written by the device
  int8_t parent[2][MAX_RANKS];
  int8_t child[2][MAX_RANKS][2];
  int8_t childIdx[2][MAX_RANKS];  // my position among my parent's children
  int8_t nchild[2][MAX_RANKS];
};

// One channel-slice of one collective, run by one lane (one workgroup per rank).
struct WorkItem {
  uint8_t coll, algo, proto, dtype;
  uint8_t op, direct, tree, pad;
  int32_t root;
  uint32_t argsIndex;
  uint32_t doneIndex;        // completion record index, 0xFFFFFFFF = none
  uint32_t unitBytes;        // 1 (AllGather, Broadcast) or the element size
  uint32_t elemBytes;
  uint64_t count;            // units per rank (per block for AllGather / ReduceScatter)
  uint64_t chOffset;         // workOffset of this channel, units
  uint64_t chCount;          // channelCount, units
  uint64_t chunk;            // chunkCount, units
};

struct CollArgs {
  const char* send[MAX_RANKS];
  char* recv[MAX_RANKS];
};

struct LaunchDesc {
  const DevComm* comm;
  const WorkItem* items;        // work list in device memory, or null: inline items
  const uint32_t* laneStart;    // nlanes + 1 offsets into items
  const CollArgs* args;         // pointer tables in device memory
  uint64_t* stamps;             // completion stamps [doneIndex * nranks + rank]
  uint32_t nlanes;
  uint32_t nranks;
  uint32_t xcdMap;              // 1: lane l's workgroups share XCD (l % 8)
  uint32_t pad;
  CollArgs inlineArgs;
  WorkItem inlineItems[MAX_INLINE];
};

}  // namespace vccl
