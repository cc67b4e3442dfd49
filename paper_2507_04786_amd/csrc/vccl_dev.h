// Structures shared by the host runtime and the gfx950 kernels.
//
// Memory layout in HBM (one communicator set, "clique"):
//   * FIFOs: for every protocol p, one region for the ring connections,
//       nrings * maxLanes * nranks connections of NSLOTS slots * slotBytes[p]
//       each (index (ring * maxLanes + lane) * nranks + receivingRank), and
//       one for the tree
//       connections (6 per lane and rank, index (lane * nranks + rank) * 6 +
//       kind - 1, slots of treeSlotBytes[p]), allocated on the first tree
//       launch under protocol p.
//     Connection id = (lane * nranks + receivingRank) * NCONN + kind, where kind
//       0      ring 0: from the receiver's predecessor on ring 0
//       1, 2   tree 0: upward from the receiver's first / second child
//       3      tree 0: downward from the receiver's parent
//       4..6   the same three for tree 1
//       7..9   rings 1..3: from the receiver's predecessor on that ring.
//     A FIFO lives with its receiver (the sender stores into it).
//   * Counters: one 256-byte record per connection; `tail` (steps published by
//     the sender) at byte 0 and `head` (steps consumed by the receiver) at byte
//     128, so the two writers never share a cache line.
//   * Step numbering is per connection and counts every step the connection
//     ever took, across protocols and launches; slot = step % NSLOTS.
#pragma once
#include <stdint.h>

namespace vccl {

enum : uint8_t { COLL_ALLREDUCE = 0, COLL_BROADCAST = 1, COLL_REDUCE = 2, COLL_ALLGATHER = 3, COLL_REDUCESCATTER = 4,
                  COLL_SENDRECV = 5 };
enum : uint8_t { ALGO_RING = 0, ALGO_TREE = 1 };
enum : uint8_t { PROTO_SIMPLE = 0, PROTO_LL = 1, PROTO_LL128 = 2 };
enum : uint8_t { DT_I32 = 0, DT_F32 = 1, DT_BF16 = 2, DT_U8 = 3 };
enum : uint8_t { OP_SUM = 0, OP_MAX = 1, OP_COPY = 2 };

constexpr int NSLOTS = 8;
constexpr int NTREE_CONN = 6;   // tree connection kinds 1..6
// Ring orders of a set (Section II-C: each channel has its ring, fixed at
// initialisation): channel c of a ring collective follows ring c % nrings.
constexpr int MAX_RINGS = 4;
constexpr int NCONN = 1 + NTREE_CONN + (MAX_RINGS - 1);
// connection kind of ring k's connections
__host__ __device__ constexpr int ringKind(int k) { return k == 0 ? 0 : NTREE_CONN + k; }
constexpr int MAX_RANKS = 16;
constexpr int MAX_LANES = 64;
constexpr int MAX_INLINE = 32;
// Slot sizes, ring and tree connections (Section V-C's channel-buffer table
// gives NCCL's 512 KiB / 32 KiB / 600 KiB; a slot here holds the largest
// chunk the planner can give its connections, no more): Simple 256 KiB for
// the ring (the tuner's largest chunk), 128 KiB for the tree (its formula's
// cap); LL 32 KiB (16 KiB of payload) for both; LL128 600 KiB (562.5 KiB of
// payload) for the ring and 128 KiB (120 KiB) for the tree.
constexpr uint32_t SLOT_BYTES_SIMPLE = 256u * 1024u;
constexpr uint32_t SLOT_BYTES_LL = 32u * 1024u;
constexpr uint32_t SLOT_BYTES_LL128 = 600u * 1024u;
constexpr uint32_t TREE_SLOT_BYTES_SIMPLE = 128u * 1024u;
constexpr uint32_t TREE_SLOT_BYTES_LL = 32u * 1024u;
constexpr uint32_t TREE_SLOT_BYTES_LL128 = 128u * 1024u;
constexpr uint32_t LL128_LINE = 128, LL128_DATA = 120;
constexpr uint32_t CTR_RECORD_U64 = 32;  // 256 B per connection
constexpr uint32_t CTR_HEAD_U64 = 16;    // head at +128 B
constexpr uint32_t CLAIM_STRIDE_U64 = 16;
// per-workgroup record of a profiling launch: first tick, last tick, ticks
// spent waiting for counters, items run
constexpr uint32_t PROFILE_WORDS = 4;

// Store policy of a work item's traffic between the workgroups of a lane
// (data, protocol lines and step counters; see device.hip): SCOPE_DEVICE --
// sc1 stores, seen from any XCD; SCOPE_XCD -- plain stores into the L2 of
// the XCD the lane's workgroups share.  Loads are device-coherent (sc1)
// under both.
constexpr uint32_t SCOPE_DEVICE = 0, SCOPE_XCD = 1;

// device-side error codes (bit flags in the error word)
constexpr uint32_t ERR_TIMEOUT = 1u, ERR_ABORT = 2u, ERR_PLACEMENT = 4u;

struct DevComm {
  int32_t nranks;
  int32_t maxLanes;
  uint64_t timeoutTicks;        // device wall-clock ticks a single wait may take
  uint32_t deadMask;            // test hook: ranks whose workgroups do nothing
  uint32_t scope;               // SCOPE_DEVICE or SCOPE_XCD for every launch of the set
  char* fifo[3];                // ring connections, per protocol
  char* treeFifo[3];            // tree connections, per protocol (null until first used)
  uint64_t slotBytes[3];        // slot size of the ring connections, per protocol
  uint64_t treeSlotBytes[3];    // slot size of the tree connections, per protocol
  uint64_t* ctr;                // counters
  uint32_t* abortFlag;          // host-pinned, written by the host
  uint32_t* errorWord;          // host-pinned, written by the device
  uint64_t* claim;              // per-XCD role counters (CLAIM_STRIDE_U64 apart)
  int8_t parent[2][MAX_RANKS];
  int8_t child[2][MAX_RANKS][2];
  int8_t childIdx[2][MAX_RANKS];  // my position among my parent's children
  int8_t nchild[2][MAX_RANKS];
  int32_t nrings;                   // ring orders, 1..MAX_RINGS
  int8_t ringRank[MAX_RINGS][MAX_RANKS];  // the rank at each position of ring k
  int8_t ringPos[MAX_RINGS][MAX_RANKS];   // the position of each rank on ring k
};

// One channel-slice of one collective, run by one lane (one workgroup per rank).
struct WorkItem {
  uint8_t coll, algo, proto, dtype;
  uint8_t op, direct, tree, peer;  // peer: receiving rank of a point-to-point transfer
  int32_t root;                    // root, or the sending rank of a point-to-point transfer
  uint32_t argsIndex;
  uint32_t doneIndex;        // completion record index, 0xFFFFFFFF = none
  uint32_t unitBytes;        // 1 (AllGather, Broadcast) or the element size
  uint32_t elemBytes;
  uint8_t scope;             // SCOPE_DEVICE or SCOPE_XCD: store policy of this item's traffic
  uint8_t role;              // tree: ROLE_FUSED, or the up / down half of a split channel, or idle
  uint8_t connLane;          // tree halves: the lane whose connections both halves use
  uint8_t ring;              // ring collectives: the ring order the channel follows
  uint64_t count;            // units per rank (per block for AllGather / ReduceScatter)
  uint64_t chOffset;         // workOffset of this channel, units
  uint64_t chCount;          // channelCount, units
  uint64_t chunk;            // chunkCount, units
};

static_assert(sizeof(WorkItem) == 64, "work items are 64 bytes");
enum : uint8_t { ROLE_FUSED = 0, ROLE_UP = 1, ROLE_DOWN = 2, ROLE_IDLE = 3 };

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
  uint64_t* profile;            // profiling launches: PROFILE_WORDS per (lane, rank), else null
  uint32_t nlanes;
  uint32_t nranks;
  uint32_t xcdMap;              // 1: lane l's workgroups share XCD (l % 8)
  uint32_t perXcd;              // roles per XCD in this launch (grid = 8 * perXcd)
  uint64_t claimBase;           // role claims of all earlier launches, per XCD
  CollArgs inlineArgs;
  WorkItem inlineItems[MAX_INLINE];
};

// ---------------------------------------------------------------- serving
// Per-lane request queues live in pinned host memory: the host writes an
// entry, then bumps the lane's `posted` counter.  Only the lane's rank-0
// workgroup (the leader) polls host memory: it copies the entry into a
// device-memory mirror and releases the lane's other workgroups through a
// device counter, so host memory sees one poller per lane instead of R.
// Every workgroup of the lane runs the entry and then publishes its own
// `done` counter (with a system-scope release, so the outputs are visible to
// later work).
// Only the leader decides when its lane stops taking work: it leaves on the
// host's stop word, on the idle word (raised by any leader that waited
// idleTicks without work), or on a failure, and then stores SERVE_EXIT into
// the lane's release counter.  The other workgroups of the lane leave only
// on that marker, the host's stop word or a failure, so an entry the leader
// accepted is always run by the whole lane.
constexpr uint64_t SERVE_EXIT = 1ull << 63;
constexpr int SERVE_QUEUE = 4;
constexpr int SERVE_STRIDE_U64 = 16;  // counters 128 B apart
constexpr int SERVE_DBG_WORDS = 5;    // per (lane, rank): seen, picked, polls, pickup tick, finish tick

struct ServeEntry {
  WorkItem item;
  CollArgs args;
};

struct ServeDesc {
  const DevComm* comm;
  ServeEntry* queue;        // [nlanes][SERVE_QUEUE]
  uint64_t* posted;         // [nlanes] * SERVE_STRIDE_U64
  uint64_t* done;           // [nlanes * nranks] * SERVE_STRIDE_U64
  uint32_t* stop;           // set by the host to end the kernel
  uint32_t* idle;           // set by the first leader that waited idleTicks without work
  uint64_t* dbg;            // per (lane, rank): SERVE_DBG_WORDS words, SERVE_STRIDE_U64 apart
  ServeEntry* mirror;       // device memory: [nlanes][SERVE_QUEUE] copies made by the leaders
  uint64_t* laneSeq;        // device memory: [nlanes] * SERVE_STRIDE_U64, entries released
                            // (zeroed before every launch), or SERVE_EXIT | seq
  uint64_t idleTicks;       // the kernel exits after this long without work
  uint32_t nlanes, nranks, xcdMap, perXcd;
  uint64_t claimBase;
  uint64_t startSeq[MAX_LANES];
};

// ---------------------------------------------------------------- allocation-free AllReduce
// vcclAllReduceNoAlloc keeps everything it needs beyond the caller's buffers
// in one file-scope device array (device.hip), laid out as below: the
// DevComm it runs with, the abort and error words, the per-XCD claim
// counters, the counters of up to NA_CONNS ring connections (lanes x ranks)
// and their FIFOs, Simple slots of NA_SLOT_SIMPLE bytes and LL slots of
// NA_SLOT_LL bytes.  Every call rewrites the DevComm and zeroes the words,
// the claim counters, the counters it uses and, under LL, the LL slots it
// uses, so each call starts from step 0 whatever ran before.
constexpr uint64_t NA_CONNS = 128;
constexpr uint64_t NA_MAX_LANES = 32;
constexpr uint64_t NA_SLOT_SIMPLE = 32u * 1024u;
constexpr uint64_t NA_SLOT_LL = 8u * 1024u;
constexpr uint64_t NA_OFF_COMM = 0;
constexpr uint64_t NA_OFF_WORDS = 1024;  // abort word at +0, error word at +128
constexpr uint64_t NA_OFF_CLAIM = 2048;  // 8 counters, CLAIM_STRIDE_U64 apart
constexpr uint64_t NA_OFF_CTR = 4096;
constexpr uint64_t NA_CTR_BYTES = NA_CONNS * NCONN * CTR_RECORD_U64 * 8;
constexpr uint64_t NA_OFF_FIFO_SIMPLE = 512u * 1024u;
constexpr uint64_t NA_OFF_FIFO_LL = NA_OFF_FIFO_SIMPLE + NA_CONNS * NSLOTS * NA_SLOT_SIMPLE;
constexpr uint64_t NA_SCRATCH_BYTES = NA_OFF_FIFO_LL + NA_CONNS * NSLOTS * NA_SLOT_LL;
static_assert(sizeof(DevComm) <= NA_OFF_WORDS - NA_OFF_COMM, "DevComm fits its scratch slot");
static_assert(NA_OFF_CLAIM + 8 * CLAIM_STRIDE_U64 * 8 <= NA_OFF_CTR, "claim counters fit");
static_assert(NA_OFF_CTR + NA_CTR_BYTES <= NA_OFF_FIFO_SIMPLE, "counters fit before the FIFOs");
static_assert(NA_MAX_LANES <= MAX_INLINE, "one inline work item per lane");

}  // namespace vccl
