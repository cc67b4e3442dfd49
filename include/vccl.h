/*
 * vccl -- virtual-rank collective communication on one AMD MI355X (gfx950).
 *
 * R virtual ranks (2..16) live on one GPU.  Every rank owns its own send and
 * receive buffers (device memory supplied by the caller) and its own FIFO
 * regions (device memory owned by the library).  A collective is split into
 * channels; each channel runs as one workgroup per rank, and the workgroups
 * of a channel hand data to each other through bounded FIFOs of slots,
 * synchronised by counters (Simple protocol) or by flags embedded in every
 * line (LL: 4 B data + 4 B flag; LL128: 120 B data + 8 B flag).
 *
 * The API follows the paper's description of NCCL's (Section II-A):
 * communicators created together for all ranks by one thread
 * (CommInitAll), Destroy and Abort, the five collectives, and
 * GroupStart/GroupEnd to fuse several calls into one kernel launch.  The
 * launch model is "one CPU thread for multiple GPUs" (Section II-B): one host
 * thread issues every rank's call.
 *
 * Conventions shared by every entry point:
 *  - Buffers: plain device pointers (hipMalloc'ed or torch tensors on the same
 *    device), aligned to the element size, owned by the caller and alive until
 *    the stream has completed the call.  Counts are elements of the data type.
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *    stream).  When ranks pass different streams, the library joins them with
 *    events so the single launch follows all of them and all of them follow it.
 *  - Matching: a collective is issued once all R ranks of the communicator set
 *    have called it (same call number per rank).  Arguments that must agree
 *    across ranks (count, type, op, root) are checked at that point; a
 *    mismatch returns vcclInvalidUsage to the call that completes the set.
 *  - Errors: argument errors are returned synchronously and nothing is
 *    enqueued.  Errors that happen on the device (a wait that exceeded the
 *    timeout, an abort) are reported by vcclCommGetAsyncError; after such an
 *    error the communicator set must be destroyed.
 *  - Threads: the API is not thread-safe; drive one communicator set from one
 *    host thread (Section II-B, "one CPU thread for multiple GPUs").
 */
#ifndef VCCL_H
#define VCCL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VCCL_MAJOR 0
#define VCCL_MINOR 1
#define VCCL_MAX_RANKS 16
#define VCCL_MAX_CHANNELS 64
#define VCCL_MAX_RINGS 4

typedef struct vcclComm* vcclComm_t;

typedef enum {
  vcclSuccess = 0,
  vcclUnhandledHipError = 1,
  vcclSystemError = 2,
  vcclInternalError = 3,
  vcclInvalidArgument = 4,
  vcclInvalidUsage = 5,
  vcclRemoteError = 6, /* a peer did not answer within the timeout, or abort */
  vcclInProgress = 7
} vcclResult_t;

typedef enum { vcclInt32 = 0, vcclFloat32 = 1, vcclBfloat16 = 2 } vcclDataType_t;
typedef enum { vcclSum = 0, vcclMax = 1 } vcclRedOp_t;

/* Algorithms and protocols (Section V-A support table: Tree only for AllReduce). */
typedef enum { vcclAlgoAuto = -1, vcclAlgoRing = 0, vcclAlgoTree = 1 } vcclAlgo_t;
typedef enum { vcclProtoAuto = -1, vcclProtoSimple = 0, vcclProtoLL = 1, vcclProtoLL128 = 2 } vcclProto_t;

const char* vcclGetErrorString(vcclResult_t result);
vcclResult_t vcclGetVersion(int* version); /* major*100 + minor */

/* ---------------------------------------------------------------- communicators */

/* Section II-A, "Communicator Management": ncclCommInitAll creates all
 * communicators of a single process/thread at once.  Creates `nranks`
 * (2..16) virtual-rank communicators on one device: devlist == NULL uses the
 * current HIP device, otherwise devlist[0] names it and every other entry
 * must name the same device.  Allocates the FIFOs and counters of every
 * (channel, rank, connection) and builds the ring (rank p sends to p + 1 on
 * every channel) and the double binary tree (Section II-C).  The set's lane limit (most channels a collective can use)
 * is the environment's VCCL_MAX_CHANNELS, else 2 CUs / nranks rounded down to
 * a multiple of 8 and held to 32..64 (64 up to 8 ranks on 256 CUs).  comms[] (caller-owned array of nranks
 * handles) receives one handle per rank.  Errors: vcclInvalidArgument for a bad count or device,
 * vcclUnhandledHipError if device memory cannot be obtained. */
vcclResult_t vcclCommInitAll(vcclComm_t* comms, int nranks, const int* devlist);

/* vcclCommInitAll with the ring of every channel given (Section II-C: each
 * channel has its own ring, in which every rank knows its predecessor and
 * successor, set up at initialisation and kept for every collective).
 * rings: a caller-owned host array of nrings rows of nranks entries; row k
 * lists the ranks in ring order (rank rings[k*nranks + q] sends to the rank
 * at q + 1, the last to the first) and must be a permutation of
 * 0..nranks-1.  Channel c of a ring collective follows row c mod nrings,
 * wherever it runs (launched alone, in a group or served), so a collective's
 * bits depend on its channel count, not on how it was launched.  Tree
 * AllReduce and Send/Recv do not use the rings.  Ring-order k > 0 has FIFOs
 * of its own: the set's ring FIFO memory grows nrings-fold.  rings == NULL
 * (nrings ignored) is vcclCommInitAll.  vcclInvalidArgument for nrings
 * outside 1..VCCL_MAX_RINGS or a row that is not a permutation, otherwise as
 * vcclCommInitAll. */
vcclResult_t vcclCommInitAllRings(vcclComm_t* comms, int nranks, const int* devlist, int nrings, const int* rings);

/* The set's ring orders: *nrings receives their count, and, when rings is
 * not NULL, rings[k*nranks + q] the rank at position q of ring k (a
 * caller-owned host array of at least *nrings x nranks entries; ask with
 * rings == NULL first for the count).  vcclInvalidArgument for an unknown
 * handle or a null nrings. */
vcclResult_t vcclCommGetRings(vcclComm_t comm, int* nrings, int* rings);

/* Section II-A: ncclCommDestroy completes pending operations, then frees.
 * Destroying any rank's handle waits for all work of the set and frees the
 * set's resources once every rank's handle has been destroyed.  Destroy every
 * set before the process exits: the library runs no code at exit, so a set
 * left alive is released by the HIP runtime's own teardown. */
vcclResult_t vcclCommDestroy(vcclComm_t comm);

/* Section II-A: ncclCommAbort terminates at once and cancels ongoing
 * operations.  Sets the set's abort word (host memory the device polls in every
 * wait loop); running kernels leave their waits and exit; pending unmatched
 * calls are dropped.  The handles stay valid only for Destroy. */
vcclResult_t vcclCommAbort(vcclComm_t comm);

/* vcclSuccess, or the first device-side error of the set (vcclRemoteError
 * after a timeout or an abort).  Does not synchronise. */
vcclResult_t vcclCommGetAsyncError(vcclComm_t comm, vcclResult_t* asyncError);

/* Section II-A: *count receives the number of ranks of comm's set, *rank the
 * rank comm stands for (0 .. nranks-1).  vcclInvalidArgument for an unknown
 * or destroyed handle or a null output. */
vcclResult_t vcclCommCount(vcclComm_t comm, int* count);
vcclResult_t vcclCommUserRank(vcclComm_t comm, int* rank);

/* ---------------------------------------------------------------- collectives
 * Section II-A, "Collective Communication": the five collectives.  Step
 * sequences: Section V-E.  Every call below is made once per rank with that
 * rank's comm handle and buffers. */

/* recv[i] = op over ranks of send[i], i < count, on every rank.  In place
 * when send == recv.  Ring (Section V-E, Ring AllReduce) or double binary
 * tree (Section V-E, Tree AllReduce). */
vcclResult_t vcclAllReduce(const void* sendbuff, void* recvbuff, size_t count, vcclDataType_t datatype,
                           vcclRedOp_t op, vcclComm_t comm, void* stream);

/* recv = send of `root` on every rank (a chain from the root along the ring,
 * Section V-E, Ring Broadcast).  sendbuff is read on the root only (other
 * ranks may pass NULL); in place when the root's send == recv. */
vcclResult_t vcclBroadcast(const void* sendbuff, void* recvbuff, size_t count, vcclDataType_t datatype, int root,
                           vcclComm_t comm, void* stream);

/* recv (root only) = op over ranks of send (a chain ending at the root,
 * Section V-E, Ring Reduce).  Non-root recvbuff is neither read nor written
 * (may be NULL). */
vcclResult_t vcclReduce(const void* sendbuff, void* recvbuff, size_t count, vcclDataType_t datatype,
                        vcclRedOp_t op, int root, vcclComm_t comm, void* stream);

/* recv[q*sendcount + i] = send of rank q [i] (Section V-E, Ring AllGather).
 * recvbuff holds nranks*sendcount elements.  In place when
 * send == recv + rank*sendcount. */
vcclResult_t vcclAllGather(const void* sendbuff, void* recvbuff, size_t sendcount, vcclDataType_t datatype,
                           vcclComm_t comm, void* stream);

/* recv[i] = op over ranks of send[rank*recvcount + i] (Section V-E, Ring
 * ReduceScatter).  sendbuff holds nranks*recvcount elements.  In place when
 * recv == send + rank*recvcount. */
vcclResult_t vcclReduceScatter(const void* sendbuff, void* recvbuff, size_t recvcount, vcclDataType_t datatype,
                               vcclRedOp_t op, vcclComm_t comm, void* stream);

/* Section II-A, "Point-to-Point Communication": vcclSend moves `count`
 * elements of sendbuff from the calling rank to rank `peer`; vcclRecv receives
 * them into recvbuff (count elements) on `peer`'s partner.  The k-th Send from
 * rank a to rank b pairs with the k-th Recv that b posts from a; count and
 * datatype must agree (vcclInvalidUsage otherwise, returned to the call that
 * completes the pair).  A pair is issued as soon as both sides are posted:
 * outside a group at once, inside a group at GroupEnd together with the
 * group's other calls, so that Send/Recv pairs between every two ranks give
 * all-to-all, scatter or gather patterns in one launch.  A transfer is split
 * over channels (one per MiB, Section II-C) and its bytes go straight from
 * sendbuff into recvbuff with no intermediate FIFO, as in P2P_DIRECT
 * (Section IV-A); every workgroup of a channel's lane copies a share.  The
 * launch itself orders the two buffers against all other work, so no head /
 * tail synchronisation is needed inside it.  peer may be the caller itself
 * (a local copy).  Buffers are device memory aligned to the
 * element size, caller-owned, not overlapping; peer outside [0, nranks) or a
 * null buffer with count > 0 is vcclInvalidArgument.  A group that ends with
 * a Send or Recv still unpaired returns vcclInvalidUsage and issues nothing. */
vcclResult_t vcclSend(const void* sendbuff, size_t count, vcclDataType_t datatype, int peer, vcclComm_t comm,
                      void* stream);
vcclResult_t vcclRecv(void* recvbuff, size_t count, vcclDataType_t datatype, int peer, vcclComm_t comm,
                      void* stream);

/* Section II-A, "Group Calls": calls between GroupStart and GroupEnd are
 * deferred and executed together as part of one launch.  Groups nest; the
 * outermost GroupEnd plans every collective matched inside the group (per
 * communicator set: one persistent kernel over a work list, each collective
 * split into channels placed on lanes) and launches it.  A group that ends
 * with unmatched calls returns vcclInvalidUsage and issues nothing. */
vcclResult_t vcclGroupStart(void);
vcclResult_t vcclGroupEnd(void);

/* Stream capture: collective calls must not be captured into a HIP graph.
 * Each launch's workgroups claim their roles relative to a base the host
 * advances per launch, which a replay would repeat. */

/* ---------------------------------------------------------------- tuning
 * Section III-D and Section II-C: the algorithm and protocol are chosen per
 * call (user setting, else a tuning model), then the channel count.  The
 * library's tuner takes algorithm, protocol, channels, chunk (Simple) and
 * workgroup size (for a collective launched alone) from a table
 * measured on this device for 4, 8 and 16 ranks and power-of-two sizes,
 * using the nearest entry.  These calls and the environment variables
 * VCCL_ALGO, VCCL_PROTO (simple|ll|ll128), VCCL_NCHANNELS, VCCL_CHUNK_BYTES,
 * VCCL_NTHREADS, VCCL_DIRECT override it for the whole communicator set.
 * A negative / zero field means "tuner decides".  A grouped collective gets
 * the same plan as the same call launched alone, so its result has the same
 * bits; only the workgroup size of a group is the largest among its plans. */
typedef struct {
  int algo;           /* vcclAlgo_t */
  int proto;          /* vcclProto_t */
  int nchannels;      /* 1..VCCL_MAX_CHANNELS */
  int nthreads;       /* workgroup size: 64..1024, multiple of 64 */
  size_t chunkBytes;  /* elementary-step chunk, multiple of 16, <= slot payload */
  int direct;         /* 1: P2P_DIRECT-style copies into peer buffers (Simple only) */
} vcclTuning_t;

/* Copies *tuning (caller-owned, read during the call only).  Applies to every
 * later call of the set.  vcclInvalidArgument, with nothing changed, for an
 * unknown handle, a null tuning, an algorithm or protocol out of range,
 * nchannels above the set's lane limit, an illegal nthreads or a chunkBytes
 * that is not a multiple of 16.  A chunk larger than the slot payload, or a
 * tree for a collective other than AllReduce, is clamped when planned (the
 * plan actually used is reported by vcclCommGetLastPlan). */
vcclResult_t vcclCommSetTuning(vcclComm_t comm, const vcclTuning_t* tuning);

/* What the most recent launch of the set used (for tests and benchmarks). */
typedef struct {
  int algo, proto, nchannels, nthreads, direct, nlanes, nitems, ncolls;
  size_t chunkBytes;
  int grid;           /* workgroups launched */
  int scope;          /* store policy chosen for the (first) collective: 0 device-coherent
                         stores, 1 plain stores into the XCD's L2 (each channel's
                         workgroups share an XCD; loads are device-coherent in both) */
  int treeRanksPerNode; /* tree topology of the set (VCCL_TREE_RANKS_PER_NODE at init):
                           chains of this many consecutive ranks, double binary tree
                           across the chains; 1 = the plain double binary tree */
  int ll128;          /* 1: LL128 may be planned on the set's device; 0: LL128 is off
                         (Section III-C: its tear test found a torn line or did not
                         finish, or VCCL_LL128=0) and every LL128 plan, tuned or
                         requested, runs as LL */
} vcclPlanInfo_t;
/* Host-side copy; does not synchronise.  All zero before the first launch.
 * vcclInvalidArgument for an unknown handle or a null info. */
vcclResult_t vcclCommGetLastPlan(vcclComm_t comm, vcclPlanInfo_t* info);

/* Device-side completion time (ns, device wall clock) of each collective of
 * the most recent launch, in issue order: the latest finish over its ranks.
 * Waits for that launch.  n is the capacity of stamps_ns (host array,
 * caller-owned); *written receives the count (0 for n <= 0 or before the
 * first launch).  vcclInvalidArgument for an unknown handle or a null
 * pointer. */
vcclResult_t vcclCommGetLastTimestamps(vcclComm_t comm, uint64_t* stamps_ns, int n, int* written);

/* ---------------------------------------------------------------- allocation-free AllReduce */

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the ring
 * AllReduce of vcclAllReduce for `nranks` (2..16) virtual ranks, with no
 * communicator set and no allocation.  sendbuffs[r] / recvbuffs[r] (host
 * arrays of nranks device pointers, caller-owned, element-aligned; in place
 * when equal) are rank r's buffers of `count` elements; recv[r][i] = op over
 * ranks of send[q][i].  `stream` is a hipStream_t as void*; plan (may be
 * NULL, caller-owned host memory) receives the plan that ran.
 * Everything beyond the caller's buffers lives in one file-scope device
 * array of 40.5 MiB per device (the descriptor, the counters of at most 128
 * lanes x ranks, 8 Simple slots of 32 KiB and 8 LL slots of 8 KiB per
 * connection): channels are limited to min(32, 128 / nranks), Simple chunks
 * to 32 KiB, LL chunks to 4 KiB; the protocol is Simple or LL, never LL128,
 * and the algorithm the ring, so results are the oracle's ring fold for the
 * reported plan.  The first call on a device looks the array up with that
 * device current; every call then enqueues two launches on `stream` (one
 * that rewrites the descriptor and zeroes the counters and LL slots it
 * uses, then the collective), and calls nothing that allocates.  Both
 * launches may be captured in a HIP graph (call once outside capture first,
 * so the array is looked up): the clearing is a kernel, not a memset, so every
 * replay starts afresh like a call.  All calls
 * on one device share its array: calls that overlap on that device (other
 * streams, other threads) race and must not be made.  Every wait is bounded
 * (5 s); a wait that runs out leaves the output undefined and is not
 * reported here (there is no communicator to query), and the next call
 * starts afresh.  Errors: vcclInvalidArgument for a null array or buffer
 * (count > 0), nranks outside 2..16, an unknown datatype or op, a
 * misaligned buffer or count above 2^40; vcclUnhandledHipError when a HIP
 * call fails; vcclSuccess with nothing enqueued for count == 0. */
vcclResult_t vcclAllReduceNoAlloc(const void* const* sendbuffs, void* const* recvbuffs, int nranks, size_t count,
                                  vcclDataType_t datatype, vcclRedOp_t op, void* stream, vcclPlanInfo_t* plan);

/* ---------------------------------------------------------------- failure handling
 * Every wait on the device is bounded: after `timeout_us` microseconds without
 * progress the waiting workgroup records vcclRemoteError and exits.  Applies
 * to the whole set from its next launch; the default is VCCL_TIMEOUT_US, else
 * 5 s.  Synchronises the device.  vcclInvalidArgument for an unknown handle
 * or a zero timeout. */
vcclResult_t vcclCommSetTimeout(vcclComm_t comm, uint64_t timeout_us);

/* Test hook: the workgroups of every rank whose bit is set in `mask` skip all
 * their work, so their peers must time out (see vcclCommSetTimeout); mask 0
 * restores normal operation.  Applies to the whole set from its next launch.
 * Synchronises the device.  vcclInvalidArgument for an unknown handle. */
vcclResult_t vcclCommDebugSetDeadRanks(vcclComm_t comm, uint32_t mask);

/* Test and tuning hook: with enable != 0, every later launch of the set
 * records, for each of its workgroups, when it started and ended, how long
 * it waited for step counters (Simple's head and tail, LL / LL128 send
 * credits; the workgroup's thread 0 in its waits) and how many work items it
 * ran; enable == 0 stops recording.  Synchronises the device; the first
 * enable allocates the records (64 lanes x nranks x 4 words).
 * vcclInvalidArgument for an unknown handle; vcclUnhandledHipError if the
 * allocation fails. */
vcclResult_t vcclCommDebugProfile(vcclComm_t comm, int enable);
/* The records of the set's most recent launch (recorded when profiling was
 * on), one per (lane, rank) in lane-major order, lanes 0 .. nlanes-1 of that
 * launch: out[4k .. 4k+3] = start, end and waiting time in ns of the device
 * wall clock, items run (all zero for a workgroup that ran nothing).  Waits
 * for that launch.  out is a caller-owned host array of 4 * maxEntries words;
 * *written receives the entries written (0 when nothing was recorded).
 * vcclInvalidArgument for an unknown handle or a null pointer. */
vcclResult_t vcclCommDebugReadProfile(vcclComm_t comm, uint64_t* out, int maxEntries, int* written);

/* Copies `bytes` bytes of the FIFO of connection (channel, receiving rank,
 * connection 0 = ring) for protocol `proto` starting at byte `offset` into the
 * host buffer `dst` (caller-owned).  Synchronises the device.  For
 * line-format checks.  vcclInvalidArgument for an unknown handle, a null
 * dst, channel outside [0, lane limit), rank outside [0, nranks), proto
 * outside 0..2, or a range that runs past the connection's FIFO
 * (8 slots of 256 KiB Simple (VCCL_SIMPLE_SLOT_BYTES), 32 KiB LL or
 * 600 KiB LL128). */
vcclResult_t vcclCommDebugReadFifo(vcclComm_t comm, int channel, int rank, int proto, size_t offset, void* dst,
                                   size_t bytes);

/* ---------------------------------------------------------------- probes
 * Section III-C: LL128 depends on 128-byte stores that are never split or
 * reordered; NCCL disables it where that is not guaranteed.  The tear test
 * runs `pairs` writer/reader workgroup pairs that exchange `lines` lines per
 * round for `rounds` rounds, every payload word derived from (flag, index);
 * *torn receives the number of lines whose flag was current but whose
 * payload was not.  scope selects the store policy of the lines: 0 device
 * scope (sc1 stores; with pairs = 4 writer and reader sit on different XCDs),
 * 1 XCD scope (plain stores into the shared L2; pairs must be a multiple of 8
 * so that each pair shares an XCD).  Synchronises the device; allocates and
 * frees its own buffers.  vcclInvalidArgument for pairs outside 1..64, lines
 * outside 1..65536, rounds < 1, a null output, an unknown scope or XCD scope
 * with pairs not a multiple of 8; vcclRemoteError if a wait ran past its 5 s
 * bound (the counts are then still written); vcclUnhandledHipError if a HIP
 * call failed. */
vcclResult_t vcclProbeLL128Tear(int pairs, int lines, int rounds, int scope, uint64_t* torn, uint64_t* checked);

/* The planner's choice for one collective, computed on the host with no
 * device (for tests and tuning studies): `coll` 0 AllReduce .. 4
 * ReduceScatter, `count` and `datatype` as the per-call API's, `single` 1
 * for a collective launched alone (a tree may then run as split halves), 0
 * for one inside a group.  The model device has 256 compute units, the lane
 * limit vcclCommInitAll gives `nranks` ranks there, the XCD lane map and
 * store policy, 1024 / nthreads resident workgroups per compute unit, and
 * LL128 enabled when `ll128` is 1 (0: as after a failed tear test).
 * `tuning` (may be NULL) overrides the tuner as vcclCommSetTuning does.
 * Fills *info (caller-owned) as vcclCommGetLastPlan would after that launch.
 * vcclInvalidArgument for nranks outside 2..16, an unknown coll or datatype,
 * a zero count, a null info, or a tuning vcclCommSetTuning would refuse. */
vcclResult_t vcclDebugPlanHost(int nranks, int coll, size_t count, vcclDataType_t datatype, int ll128, int single,
                               const vcclTuning_t* tuning, vcclPlanInfo_t* info);

/* The set's double binary tree `tree` (0 or 1; Section II-C): parents[r]
 * receives rank r's parent, -1 for the root.  Channel c of a tree AllReduce
 * runs on tree c mod 2.  parents is a caller-owned host array of nranks
 * entries.  vcclInvalidArgument for an unknown handle, a null array or a
 * tree other than 0 or 1. */
vcclResult_t vcclCommGetTree(vcclComm_t comm, int tree, int* parents);

/* XCC (accelerator die) id of each of `n` workgroups of a plain launch,
 * written to the host array ids[n] (caller-owned).  Synchronises the device.
 * vcclInvalidArgument for n <= 0 or a null ids; vcclUnhandledHipError if a
 * HIP call failed. */
vcclResult_t vcclProbeXccIds(int n, int* ids);

/* ---------------------------------------------------------------- serving
 * Continuous batching over one persistent kernel: requests are admitted
 * while earlier ones still run, as lanes and the staging budget free up.
 * Admission takes the oldest request that fits; a request that does not fit
 * yet lets younger ones pass for at most VCCL_SERVE_BYPASS_US microseconds
 * (default 500), after which nothing overtakes it.  A request's plan is the
 * per-call planner's for the same arguments, with at most
 * VCCL_SERVE_MAX_LANES_PER_REQUEST lanes (default half the server's) unless
 * the request holds more than half the budget (then no request of its size
 * can run beside it and it keeps its plan's lanes, up to the server's).  The
 * plan depends only on the request, so a request gives the same result alone
 * and among others. */
typedef struct vcclServer* vcclServer_t;

typedef struct {
  int coll;                        /* 0 AllReduce, 1 Broadcast, 2 Reduce, 3 AllGather, 4 ReduceScatter */
  int datatype;                    /* vcclDataType_t */
  int op;                          /* vcclRedOp_t */
  int root;
  size_t count;                    /* as the per-call API's count / sendcount / recvcount */
  const void* send[VCCL_MAX_RANKS];/* per-rank device buffers, caller-owned */
  void* recv[VCCL_MAX_RANKS];
} vcclRequest_t;

/* budgetBytes: device bytes the in-flight requests may hold (their send and
 * receive buffers plus the FIFOs of the lanes they occupy); lanes: concurrent
 * lanes of the persistent kernel (each lane = one workgroup per rank).
 * comms: the set's handles, as vcclCommInitAll returned them (comms[0] names
 * the set).  Starts the persistent kernel on a stream of its own.  Errors:
 * vcclInvalidArgument for a null pointer, lanes < 1 or above the set's lane
 * limit, or a grid that cannot be resident at once; vcclInvalidUsage if the
 * set already serves or was aborted.  While a server runs, the set's per-call
 * API must not be used. */
vcclResult_t vcclServeCreate(vcclComm_t* comms, size_t budgetBytes, int lanes, vcclServer_t* server);
/* Non-blocking: queues the request; *id receives its identifier.  Errors,
 * before anything is queued: vcclInvalidArgument for an unknown collective,
 * datatype or op, a root outside 0..nranks-1 (Broadcast, Reduce), a zero
 * count, a missing or element-misaligned buffer that the collective uses,
 * or a request whose buffers and FIFOs exceed the budget (it could never be
 * admitted). */
vcclResult_t vcclServeSubmit(vcclServer_t server, const vcclRequest_t* req, uint64_t* id);
/* Makes progress (admits queued requests, retires finished ones) and
 * reports whether `id` has completed; status (may be NULL) receives the
 * request's result, vcclInProgress while it runs; t_done_ns (may be NULL)
 * the host monotonic time (ns) at which completion was observed.  Once
 * reported done, the id is retired and unknown from then on.
 * vcclInvalidArgument for a null server or done, or an unknown id. */
vcclResult_t vcclServeTest(vcclServer_t server, uint64_t id, int* done, vcclResult_t* status, uint64_t* t_done_ns);
/* Native request loop: submits reqs[i] when arrival_ns[i] nanoseconds have
 * passed since the call began (arrival_ns non-decreasing), keeps making
 * progress, and returns when all n requests completed.  latency_ns[i]
 * receives completion time - arrival time; statuses (may be NULL) the
 * per-request result.  Host arrays of n entries, caller-owned.  A submit
 * error (as vcclServeSubmit's) returns at once; requests already submitted
 * stay queued and are drained by vcclServeDestroy. */
vcclResult_t vcclServeReplay(vcclServer_t server, const vcclRequest_t* reqs, const uint64_t* arrival_ns, int n,
                             uint64_t* latency_ns, vcclResult_t* statuses);
/* The plain per-call path over the same kind of request stream, for
 * comparison with the server: submits nothing to a server; instead issues
 * reqs[i] when arrival_ns[i] nanoseconds have passed since the call began
 * (arrival_ns non-decreasing) as one ordinary per-rank call per rank of the
 * set (vcclAllReduce ... vcclReduceScatter with comms[r], so each request
 * is one launch of the per-call planner's plan, on `stream`, a hipStream_t
 * as void*), and returns when all n launches completed.  latency_ns[i]
 * receives the host monotonic time at which request i's completion was
 * observed minus its arrival time; statuses (may be NULL) the call's result,
 * or the set's asynchronous error after a device-side failure.  comms is the
 * set's nranks handles in rank order; reqs, arrival_ns, latency_ns and
 * statuses are caller-owned host arrays of n entries; the request buffers
 * follow the per-call API's rules.  The set must not be serving.  Errors:
 * vcclInvalidArgument for a null pointer, n < 0 or handles of another set
 * or out of order; the first failing call's result otherwise (requests
 * issued before it have completed when this returns). */
vcclResult_t vcclReplayPerCall(vcclComm_t* comms, const vcclRequest_t* reqs, const uint64_t* arrival_ns, int n,
                               void* stream, uint64_t* latency_ns, vcclResult_t* statuses);
/* The plan request `id` runs with, frozen at submission (it depends only on
 * the request): algorithm, protocol, channels (= lanes it occupies), chunk,
 * store policy; nthreads and grid are the persistent kernel's.  A request
 * whose size (larger per-rank buffer) is at least VCCL_SERVE_FULL_PLAN_BYTES
 * (default 16 MiB), and every floating-point sum AllReduce (whose bits
 * depend on the channel count), keeps the per-call plan's channels, up to
 * the server's lanes; any other request takes at most
 * VCCL_SERVE_MAX_LANES_PER_REQUEST.  A float sum's bits follow from this
 * plan exactly as for the same plan launched per call, so with the set's
 * lane limit as its lanes a server gives every request the per-call bits.  Valid from submission until vcclServeTest reports the
 * request done.  *info is caller-owned host memory.  vcclInvalidArgument
 * for a null server or info, or an unknown (or already retired) id. */
vcclResult_t vcclServeGetPlan(vcclServer_t server, uint64_t id, vcclPlanInfo_t* info);
/* Monitoring: for each of the first maxEntries (lane, rank) pairs,
 * VCCL_SERVE_DEBUG_WORDS words into out[]: requests posted to the lane (host),
 * the last posted count the workgroup observed (the lane's rank-0 workgroup
 * watches the host counter, the others its release counter), entries it
 * picked up, entries it completed, its poll iteration count, and the device
 * clock (100 MHz ticks) when it picked up and finished its last entry.
 * Reads host memory only. */
#define VCCL_SERVE_DEBUG_WORDS 7
vcclResult_t vcclServeDebugState(vcclServer_t server, uint64_t* out, int maxEntries);
/* Drains every request (waiting at most 60 s), stops the persistent kernel,
 * waits for it and frees the server; the set's per-call API is usable again.
 * vcclInvalidArgument for a null server. */
vcclResult_t vcclServeDestroy(vcclServer_t server);

#ifdef __cplusplus
}
#endif
#endif /* VCCL_H */
