// gfx950 kernels of the virtual-rank collectives.
//
// One workgroup runs one (lane, rank): it executes, for every work item of its
// lane, that rank's primitive sequence (Section V-E step tables) on the item's
// channel region.  Workgroups of the same lane exchange data through FIFOs in
// HBM under one of three protocols (Section III):
//
//  * Simple: a slot holds a whole chunk.  The sender waits for a free slot
//    (head counter), stores the chunk, drains the stores (every wave waits
//    for its stores, then a barrier) and publishes the tail counter; the
//    receiver waits on tail, reads the slot and returns it through head.
//    The receiver waits for the full chunk.
//  * LL: every 8-byte unit carries 4 bytes of data and a 4-byte flag and is
//    written by one 64-bit store and read by one 64-bit load, so no fence is
//    needed; the receiver polls each unit's flag.  A lane handles four pairs
//    of units per pass and issues all their loads before it polls.
//  * LL128: every 128-byte line carries 120 bytes of data and an 8-byte flag
//    and is written by one 16-byte store per lane across 8 lanes (one store
//    instruction) and read back the same way; the receiver checks the flag
//    word and re-reads the whole line until it is current.  A wave handles
//    four 8-line groups per pass.  This relies on 128-byte lines not being
//    torn (see the tear probe below).
// Loads are device-scope coherent; stores follow the work item's scope (see
// the memory policy below).
//
// Section V-D's mapping is kept where it holds on CDNA: a channel is a
// workgroup per rank, wave 0 stages the work descriptor in LDS, all waves of
// the workgroup move 16-byte vectors in an unrolled, wave-uniform loop.
// Values uniform over the workgroup (the context, the item, stream bases)
// are read once into scalar registers.
// "Direct" variants (Section IV-A, P2P_DIRECT) write straight into the peer's
// receive buffer instead of its FIFO while keeping the head/tail protocol.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vccl_dev.h"

namespace vccl {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ memory access

__device__ __forceinline__ uint64_t ldAgent(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void stAgent(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ldSystem32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void orSystem32(uint32_t* p, uint32_t v) {
  __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
// Drain this wave's outstanding vector memory operations (vmcnt(0)).  A bare
// workgroup barrier does not wait for them on gfx950.
__device__ __forceinline__ void drainVmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }
__device__ __forceinline__ uint64_t nowTicks() { return __builtin_amdgcn_s_memrealtime(); }

// Race-detection build (compiled with -DVCCL_JITTER, never the default):
// every publish -- a counter store, a batch of LL / LL128 line stores -- is
// preceded by a pause of a random 0..63 x 512 clocks, so that producers and
// consumers meet in orders the normal timing rarely gives, and every FIFO
// slot a receiver has consumed is overwritten with a poison pattern (and,
// under LL / LL128, a flag that is never current) before its credit is
// returned, so that a read of a slot before its data was published, or
// after its credit was returned, gives wrong results instead of stale
// right ones.
#ifdef VCCL_JITTER
constexpr bool kJitter = true;
__device__ __forceinline__ void jitterPause() {
  uint32_t h = (uint32_t)nowTicks() * 0x9E3779B1u ^ (uint32_t)(threadIdx.x >> 6) * 0x85EBCA77u ^
               (uint32_t)blockIdx.x * 0xC2B2AE3Du;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 13;
  for (uint32_t k = __builtin_amdgcn_readfirstlane(h & 63u); k; --k) __builtin_amdgcn_s_sleep(8);
}
#else
constexpr bool kJitter = false;
__device__ __forceinline__ void jitterPause() {}
#endif
constexpr uint32_t POISON = 0xDEADBEEFu;

// Workgroup-uniform values (stream bases, sizes, strides) often reach the
// code that uses them through LDS, memory or a call, where the compiler can
// no longer tell they are uniform: it keeps them in vector registers and
// wraps every buffer access in a loop over the distinct values of the wave.
// Taking lane 0's copy makes them scalar; callers pass only uniform values.
__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
  return ((uint64_t)uniform((uint32_t)(v >> 32)) << 32) | uniform((uint32_t)v);
}
template <class T>
__device__ __forceinline__ T* uniformPtr(T* p) { return (T*)uniform64((uint64_t)p); }

// Buffer resource over [base, base + bytes): accesses past the end read zero
// and write nothing.  base and bytes must be uniform over the wave.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t makeRsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(uniformPtr(base)), (short)0, (int)uniform(bytes),
                                           0x00020000);
}
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Memory policy of everything that passes between the workgroups of a lane:
// chunks and direct writes (Simple), counters, LL units and LL128 lines
// (WorkItem::scope, chosen per item by the planner; DevComm::scope forces
// device scope for the whole set).  Loads are always device-scope coherent
// (sc1): they skip
// the CU cache and read the XCD's L2, or memory when the line is not there.
//  SCOPE_DEVICE: stores are device-scope coherent too (sc1), so they reach
//    memory and a reader on any XCD sees them.
//  SCOPE_XCD: every workgroup of a lane runs on the same XCD (roles are
//    claimed per XCD at kernel start), so the XCD's L2 is the meeting point:
//    stores are plain (through the write-through CU cache into L2) and the
//    reader's sc1 loads hit the line there.  A flag round trip between two
//    workgroups of one XCD takes about half the time of the device-scope
//    pair (measured on the device with a ping-pong of flags).  Plain stores
//    are never read by another XCD within the launch; the end of the launch
//    writes the L2 back.
// In both, draining a wave's stores (vmcnt 0) before the counter or flag that
// announces them is the whole release, and the sc1 load of that counter or
// flag, followed by sc1 loads of the data, is the whole acquire.
constexpr int LOAD_AUX = 16;  // sc1
template <int SC> struct StoreAux { static constexpr int value = SC == SCOPE_XCD ? 0 : 16; };

__device__ __forceinline__ void stPlain64(uint64_t* p, uint64_t v) {
  __builtin_amdgcn_raw_buffer_store_b64(u32x2{(uint32_t)v, (uint32_t)(v >> 32)}, makeRsrc(p, 8), 0, 0, 0);
}

template <int SC>
__device__ __forceinline__ uint64_t ldCtr(const uint64_t* p) { return ldAgent(p); }
template <int SC>
__device__ __forceinline__ void stCtr(uint64_t* p, uint64_t v) {
  if constexpr (SC == SCOPE_XCD) stPlain64(p, v);
  else stAgent(p, v);
}
// After a tail was observed, before the chunk it announces is read: the sc1
// loads of the chunk need no cache invalidation.
template <int SC>
__device__ __forceinline__ void acquireData() {}
// 8-byte LL unit and 16-byte LL128 line access (one instruction each).
template <int SC>
__device__ __forceinline__ uint64_t ldUnit(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, LOAD_AUX);
  return (uint64_t)v.x | ((uint64_t)v.y << 32);
}
template <int SC>
__device__ __forceinline__ void stUnit(__amdgpu_buffer_rsrc_t r, uint32_t off, uint64_t v) {
  __builtin_amdgcn_raw_buffer_store_b64(u32x2{(uint32_t)v, (uint32_t)(v >> 32)}, r, off, 0, StoreAux<SC>::value);
}
template <int SC>
__device__ __forceinline__ u32x4 ldLine16(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, LOAD_AUX);
}
template <int SC>
__device__ __forceinline__ void stLine16(__amdgpu_buffer_rsrc_t r, uint32_t off, u32x4 v) {
  __builtin_amdgcn_raw_buffer_store_b128(v, r, off, 0, StoreAux<SC>::value);
}

// ------------------------------------------------------------------ element operators
// Words are 32-bit and hold one int32 / fp32 element or two bf16 elements.

__device__ __forceinline__ uint32_t bf16Round(float s) {
  // round to nearest even (inputs are NaN-free)
  uint32_t u = __float_as_uint(s);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float fmaxRule(float a, float b) {
  // a > b ? a : (b > a ? b : (signbit(a) ? b : a)) -- max preferring +0
  return a > b ? a : (b > a ? b : (__float_as_uint(a) >> 31 ? b : a));
}

template <int DT, int OP>
__device__ __forceinline__ uint32_t redWord(uint32_t a, uint32_t b) {
  if constexpr (DT == DT_I32) {
    if constexpr (OP == OP_SUM) return a + b;
    else return (int32_t)a > (int32_t)b ? a : b;
  } else if constexpr (DT == DT_F32) {
    float fa = __uint_as_float(a), fb = __uint_as_float(b);
    if constexpr (OP == OP_SUM) return __float_as_uint(fa + fb);
    else return __float_as_uint(fmaxRule(fa, fb));
  } else if constexpr (DT == DT_BF16) {
    float al = __uint_as_float(a << 16), bl = __uint_as_float(b << 16);
    float ah = __uint_as_float(a & 0xFFFF0000u), bh = __uint_as_float(b & 0xFFFF0000u);
    if constexpr (OP == OP_SUM) {
      return bf16Round(al + bl) | (bf16Round(ah + bh) << 16);
    } else {
      // the result is one of the inputs: pick it by the max rule on the widened values
      const bool pickLo = bl > al || (!(al > bl) && !(bl > al) && (__float_as_uint(al) >> 31));
      const bool pickHi = bh > ah || (!(ah > bh) && !(bh > ah) && (__float_as_uint(ah) >> 31));
      return (pickLo ? (b & 0xFFFFu) : (a & 0xFFFFu)) | (pickHi ? (b & 0xFFFF0000u) : (a & 0xFFFF0000u));
    }
  } else {
    return b;
  }
}

template <int DT, int OP>
__device__ __forceinline__ uint4 redVec(uint4 a, uint4 b) {
  return make_uint4(redWord<DT, OP>(a.x, b.x), redWord<DT, OP>(a.y, b.y), redWord<DT, OP>(a.z, b.z),
                    redWord<DT, OP>(a.w, b.w));
}

template <int DT, int OP>
__device__ __forceinline__ u32x4 redVec4(u32x4 a, u32x4 b) {
  return u32x4{redWord<DT, OP>(a.x, b.x), redWord<DT, OP>(a.y, b.y), redWord<DT, OP>(a.z, b.z),
               redWord<DT, OP>(a.w, b.w)};
}

template <int DT> struct ElemSize { static constexpr int value = (DT == DT_BF16) ? 2 : (DT == DT_U8 ? 1 : 4); };

// Partial (or misaligned) payload access: element by element, never touching
// bytes at or beyond `valid`.  Pointers are element-aligned.
template <int E, bool COH>
__device__ __forceinline__ uint32_t ldElem(const char* p) {
  if constexpr (COH) {
    if constexpr (E == 4) return __hip_atomic_load((const uint32_t*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else if constexpr (E == 2) return __hip_atomic_load((const uint16_t*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return __hip_atomic_load((const uint8_t*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    if constexpr (E == 4) return *(const uint32_t*)p;
    else if constexpr (E == 2) return *(const uint16_t*)p;
    else return *(const uint8_t*)p;
  }
}
template <int E, bool COH>
__device__ __forceinline__ void stElem(char* p, uint32_t v) {
  if constexpr (COH) {
    if constexpr (E == 4) __hip_atomic_store((uint32_t*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else if constexpr (E == 2) __hip_atomic_store((uint16_t*)p, (uint16_t)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else __hip_atomic_store((uint8_t*)p, (uint8_t)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    if constexpr (E == 4) *(uint32_t*)p = v;
    else if constexpr (E == 2) *(uint16_t*)p = (uint16_t)v;
    else *(uint8_t*)p = (uint8_t)v;
  }
}

// Partial (or misaligned) payload access: element by element, never touching
// bytes at or beyond `valid`.  Pointers are element-aligned.  COH: device-
// scope coherent accesses.
template <int E, int NW, bool COH = false>
__device__ __forceinline__ void loadPart(const char* p, int valid, uint32_t (&w)[NW]) {
#pragma unroll
  for (int k = 0; k < NW; ++k) w[k] = 0;
#pragma unroll
  for (int i = 0; i < NW * 4 / E; ++i) {
    if (i * E < valid) w[(i * E) / 4] |= ldElem<E, COH>(p + i * E) << (8 * ((i * E) % 4));
  }
}
template <int E, int NW, bool COH = false>
__device__ __forceinline__ void storePart(char* p, int valid, const uint32_t (&w)[NW]) {
#pragma unroll
  for (int i = 0; i < NW * 4 / E; ++i) {
    if (i * E < valid) stElem<E, COH>(p + i * E, w[(i * E) / 4] >> (8 * ((i * E) % 4)));
  }
}

// ------------------------------------------------------------------ context

struct Ctx {
  const DevComm* comm;
  int rank, lane, nranks;
  int tid, nthreads, wave, nwaves, lid;
  int* sAbort;  // LDS flag: set when any wait of this workgroup failed
  uint32_t slotB;   // FIFO slot bytes of the running item's connections (ring or tree) and protocol
  uint64_t* sWait;  // LDS: ticks this workgroup spent in counter waits (profiling launches only), or null
};

// LDS words through LDS pointers: LDS instructions wait only on LDS, where a
// generic pointer's access would also wait on every outstanding memory access
// of the wave.
typedef __attribute__((address_space(3))) uint64_t LdsU64;
typedef volatile __attribute__((address_space(3))) int LdsFlag;
__device__ __forceinline__ LdsFlag* abortWord(const Ctx& c) { return (LdsFlag*)c.sAbort; }

// Scalar copies of the workgroup-uniform state a work item runs on (the
// context, the item's words, read from LDS or through a call): every pointer,
// size and loop bound derived from them then stays in scalar registers.
__device__ __forceinline__ Ctx uniformCtx(const Ctx& c0) {
  Ctx c;
  c.comm = uniformPtr(c0.comm);
  c.rank = (int)uniform((uint32_t)c0.rank);
  c.lane = (int)uniform((uint32_t)c0.lane);
  c.nranks = (int)uniform((uint32_t)c0.nranks);
  c.nthreads = (int)uniform((uint32_t)c0.nthreads);
  c.nwaves = (int)uniform((uint32_t)c0.nwaves);
  c.wave = (int)uniform((uint32_t)c0.wave);
  c.tid = c0.tid;
  c.lid = c0.lid;
  c.sAbort = uniformPtr(c0.sAbort);
  c.slotB = uniform(c0.slotB);
  c.sWait = uniformPtr(c0.sWait);
  return c;
}
__device__ __forceinline__ WorkItem uniformItem(const WorkItem& w0) {
  uint32_t words[sizeof(WorkItem) / 4];
  __builtin_memcpy(words, &w0, sizeof(WorkItem));
#pragma unroll
  for (int i = 0; i < (int)(sizeof(WorkItem) / 4); ++i) words[i] = uniform(words[i]);
  WorkItem w;
  __builtin_memcpy(&w, words, sizeof(WorkItem));
  return w;
}

struct Conn {
  char* fifo = nullptr;       // this connection's FIFO for the current protocol
  uint64_t* tail = nullptr;   // counter record; head() is in the same record
  uint64_t step = 0;
  __device__ __forceinline__ uint64_t* head() const { return tail + CTR_HEAD_U64; }
};

// Slot (step % NSLOTS) may be overwritten once the receiver has consumed step
// step - NSLOTS, i.e. once head >= step + 1 - NSLOTS.
__device__ __forceinline__ uint64_t creditTarget(uint64_t step) { return step + 1 > NSLOTS ? step + 1 - NSLOTS : 0; }

// Bounded wait for *ctr >= target, one lane.  Returns false (and records the
// error) on timeout or abort.
template <int SC>
__device__ __forceinline__ bool waitCounter(const Ctx& c, const uint64_t* ctr, uint64_t target) {
  if (ldCtr<SC>(ctr) >= target) return true;
  uint64_t t0 = nowTicks();
  uint32_t it = 0;
  for (;;) {
    __builtin_amdgcn_s_sleep(1);
    if (ldCtr<SC>(ctr) >= target) return true;
    if ((++it & 63u) == 0) {
      if (ldSystem32(c.comm->abortFlag)) { orSystem32(c.comm->errorWord, ERR_ABORT); return false; }
      if (nowTicks() - t0 > c.comm->timeoutTicks) { orSystem32(c.comm->errorWord, ERR_TIMEOUT); return false; }
    }
  }
}

// Before a step: every send in smask needs its slot's credit (head >=
// creditTarget(step)) and every receive in rmask its chunk (tail >= step + 1).
// One lane waits; the barrier hands the outcome to every thread.
template <int SC>
__device__ __forceinline__ bool syncConns(const Ctx& c, Conn* r, int rmask, Conn* s, int smask) {
  if (c.tid == 0) {
    const uint64_t t0 = c.sWait ? nowTicks() : 0;
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 3; ++j)
      if (ok && (smask & (1 << j))) ok = waitCounter<SC>(c, s[j].head(), creditTarget(s[j].step));
#pragma unroll
    for (int i = 0; i < 3; ++i)
      if (ok && (rmask & (1 << i))) ok = waitCounter<SC>(c, r[i].tail, r[i].step + 1);
    if (!ok) *abortWord(c) = 1;
    if (c.sWait) *(LdsU64*)c.sWait += nowTicks() - t0;
  }
  __syncthreads();
  return !*abortWord(c);
}

// Per-lane poll helper for flag-based protocols: counts spins and checks the
// abort word / timeout now and then.
struct Spinner {
  uint64_t t0 = 0;
  uint32_t it = 0;
  __device__ __forceinline__ bool tick(const Ctx& c) {
    if ((++it & 255u) == 0) {
      if (*abortWord(c)) return false;
      if (t0 == 0) t0 = nowTicks();
      if (ldSystem32(c.comm->abortFlag)) { orSystem32(c.comm->errorWord, ERR_ABORT); atomicOr(c.sAbort, 1); return false; }
      if (nowTicks() - t0 > c.comm->timeoutTicks) {
        orSystem32(c.comm->errorWord, ERR_TIMEOUT);
        atomicOr(c.sAbort, 1);
        return false;
      }
    }
    return true;
  }
};

// ------------------------------------------------------------------ Simple datapath

// Up to three pointers filled in order; every access uses a constant index so
// the list stays in registers.
struct PtrList {
  const char* p0 = nullptr;
  const char* p1 = nullptr;
  const char* p2 = nullptr;
  int n = 0;
  __device__ __forceinline__ void add(const char* v) {
    if (n == 0) p0 = v;
    else if (n == 1) p1 = v;
    else p2 = v;
    ++n;
  }
  __device__ __forceinline__ const char* get(int k) const { return k == 0 ? p0 : (k == 1 ? p1 : p2); }
};

// out[o] = in[0] (+) in[1] (+) in[2] over 16-byte vectors.  Pointers need only
// be element-aligned: the GPU runs in unaligned-access mode, so a 16-byte
// buffer access at any byte address moves exactly those 16 bytes (checked on
// the device for every misalignment 0..15, loads and stores, with and without
// sc1).  Buffer instructions: one lane offset register shared by every stream, the
// unroll stride in a scalar offset, and hardware range checks (an access past
// the stream's end reads zero and writes nothing), so the loop needs no
// per-vector bounds test.
template <int DT, int OP, int NIN, int NOUT, int LP, int SP>
__device__ __forceinline__ void reduceCopyVec(const Ctx& c, const PtrList& in, const PtrList& out, uint32_t nvec) {
  constexpr int U = 4;
  const uint32_t nb = nvec * 16;
  const uint32_t stride = uniform((uint32_t)c.nthreads * 16);
  const __amdgpu_buffer_rsrc_t i0 = makeRsrc(in.p0, nb);
  const __amdgpu_buffer_rsrc_t i1 = makeRsrc(in.p1, nb);
  const __amdgpu_buffer_rsrc_t i2 = makeRsrc(in.p2, nb);
  const __amdgpu_buffer_rsrc_t o0 = makeRsrc(out.p0, nb);
  const __amdgpu_buffer_rsrc_t o1 = makeRsrc(out.p1, nb);
  const __amdgpu_buffer_rsrc_t o2 = makeRsrc(out.p2, nb);
  for (uint32_t base = (uint32_t)c.tid * 16; base < nb; base += stride * U) {
    u32x4 v0[U], v1[U], v2[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      v0[u] = __builtin_amdgcn_raw_buffer_load_b128(i0, base, u * stride, LP);
      if constexpr (NIN > 1) v1[u] = __builtin_amdgcn_raw_buffer_load_b128(i1, base, u * stride, LP);
      if constexpr (NIN > 2) v2[u] = __builtin_amdgcn_raw_buffer_load_b128(i2, base, u * stride, LP);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      u32x4 acc = v0[u];
      if constexpr (NIN > 1) acc = redVec4<DT, OP>(acc, v1[u]);
      if constexpr (NIN > 2) acc = redVec4<DT, OP>(acc, v2[u]);
      __builtin_amdgcn_raw_buffer_store_b128(acc, o0, base, u * stride, SP);
      if constexpr (NOUT > 1) __builtin_amdgcn_raw_buffer_store_b128(acc, o1, base, u * stride, SP);
      if constexpr (NOUT > 2) __builtin_amdgcn_raw_buffer_store_b128(acc, o2, base, u * stride, SP);
    }
  }
}

// Same operation through element-wise accesses, 16 bytes (or the tail) per
// lane: the last nbytes % 16 bytes of a step.
template <int DT, int OP, int NIN, int NOUT, bool SCOH>
__device__ __forceinline__ void reduceCopyPart(const Ctx& c, const PtrList& in, const PtrList& out, uint64_t begin,
                                               uint64_t nbytes) {
  constexpr int E = ElemSize<DT>::value;
  for (uint64_t off = begin + (uint64_t)c.tid * 16; off < nbytes; off += (uint64_t)c.nthreads * 16) {
    const int valid = (int)((nbytes - off) < 16 ? (nbytes - off) : 16);
    uint32_t acc[4], w[4];
    loadPart<E, 4, true>(in.p0 + off, valid, acc);
    if constexpr (NIN > 1) {
      loadPart<E, 4, true>(in.p1 + off, valid, w);
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = redWord<DT, OP>(acc[q], w[q]);
    }
    if constexpr (NIN > 2) {
      loadPart<E, 4, true>(in.p2 + off, valid, w);
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = redWord<DT, OP>(acc[q], w[q]);
    }
    storePart<E, 4, SCOH>((char*)out.p0 + off, valid, acc);
    if constexpr (NOUT > 1) storePart<E, 4, SCOH>((char*)out.p1 + off, valid, acc);
    if constexpr (NOUT > 2) storePart<E, 4, SCOH>((char*)out.p2 + off, valid, acc);
  }
}

// Loads of every stream are sc1; stores follow the scope (sc1 for
// SCOPE_DEVICE, plain for SCOPE_XCD).
// Arguments by value: they travel in registers, where a reference would make
// the caller store the lists to its stack for every step.
template <int DT, int OP, int NIN, int NOUT, int SC>
__device__ __noinline__ void reduceCopy(int tid, int nthreads, const char* i0, const char* i1, const char* i2,
                                        const char* o0, const char* o1, const char* o2, uint64_t nbytes) {
  Ctx c{};
  c.tid = tid;
  c.nthreads = nthreads;
  PtrList in, out;
  in.p0 = i0;
  in.p1 = i1;
  in.p2 = i2;
  in.n = NIN;
  out.p0 = o0;
  out.p1 = o1;
  out.p2 = o2;
  out.n = NOUT;
  const uint32_t nvec = (uint32_t)(nbytes / 16);
  reduceCopyVec<DT, OP, NIN, NOUT, LOAD_AUX, StoreAux<SC>::value>(c, in, out, nvec);
  if (nbytes % 16) reduceCopyPart<DT, OP, NIN, NOUT, SC == SCOPE_DEVICE>(c, in, out, (uint64_t)nvec * 16, nbytes);
}

template <int DT, int OP, int SC>
__device__ void reduceCopyN(const Ctx& c, const PtrList& in, const PtrList& out, uint64_t nbytes) {
  if (nbytes == 0 || in.n == 0 || out.n == 0) return;
#define VCCL_RC(I, O) \
  if (in.n == I && out.n == O) {                                                                        \
    reduceCopy<DT, OP, I, O, SC>(c.tid, c.nthreads, in.p0, in.p1, in.p2, out.p0, out.p1, out.p2, nbytes); \
    return;                                                                                               \
  }
  VCCL_RC(1, 1) VCCL_RC(1, 2) VCCL_RC(1, 3) VCCL_RC(2, 1) VCCL_RC(2, 2) VCCL_RC(2, 3) VCCL_RC(3, 1) VCCL_RC(3, 2)
  VCCL_RC(3, 3)
#undef VCCL_RC
}

// ------------------------------------------------------------------ one elementary step
//
// Receives from the connections in rmask, sends to those in smask.  The data
// combined is: src (if any) first, then each received slot in connection
// order; it is stored to dst (if any) and to every send target.
//  recvDirect: the data of the receive is already in dst (a peer wrote it
//              there directly); only synchronise, and forward dst's content.
//  sendDirect[j]: non-null -> send j stores into that buffer instead of the
//              peer's FIFO slot.

struct StepArgs {
  const char* src;
  char* dst;
  char* sendDirect[3];
  uint64_t nbytes;
  int rmask, smask;
  bool recvDirect;
};

template <int SC, int DT, int OP>
__device__ bool stepSimple(const Ctx& c, Conn* r, Conn* s, const StepArgs& a) {
  if (!syncConns<SC>(c, r, a.rmask, s, a.smask)) return false;
  if (a.rmask) acquireData<SC>();

  PtrList in, out;
  const uint64_t slotB = c.slotB;
  if (a.src) in.add(a.src);
  if (a.recvDirect) {
    if (a.smask) in.add(a.dst);  // forward what the peer stored into our buffer
  } else {
#pragma unroll
    for (int i = 0; i < 3; ++i)
      if (a.rmask & (1 << i)) in.add(r[i].fifo + (r[i].step % NSLOTS) * slotB);
    if (a.dst && !(a.src == a.dst && in.n == 1)) out.add(a.dst);
  }
#pragma unroll
  for (int j = 0; j < 3; ++j)
    if (a.smask & (1 << j)) out.add(a.sendDirect[j] ? a.sendDirect[j] : s[j].fifo + (s[j].step % NSLOTS) * slotB);
  reduceCopyN<DT, OP, SC>(c, in, out, a.nbytes);

  drainVmem();
  __syncthreads();
  if constexpr (kJitter) {
    // every wave has read the received slots: poison them before their
    // credit goes back
    if (!a.recvDirect) {
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        if (!(a.rmask & (1 << i))) continue;
        const __amdgpu_buffer_rsrc_t rs = makeRsrc(r[i].fifo + (r[i].step % NSLOTS) * slotB, (uint32_t)slotB);
        for (uint32_t off = (uint32_t)c.tid * 16; off < a.nbytes; off += (uint32_t)c.nthreads * 16)
          __builtin_amdgcn_raw_buffer_store_b128(u32x4{POISON, POISON, POISON, POISON}, rs, off, 0,
                                                 StoreAux<SC>::value);
      }
      drainVmem();
      __syncthreads();
    }
    if (c.tid == 0) jitterPause();
  }
  if (c.tid == 0) {
    // every wave drained its stores before the barrier: the chunk is
    // visible at the traffic's scope before the tail that announces it
#pragma unroll
    for (int j = 0; j < 3; ++j)
      if (a.smask & (1 << j)) stCtr<SC>(s[j].tail, s[j].step + 1);
#pragma unroll
    for (int i = 0; i < 3; ++i)
      if (a.rmask & (1 << i)) stCtr<SC>(r[i].head(), r[i].step + 1);
  }
#pragma unroll
  for (int j = 0; j < 3; ++j)
    if (a.smask & (1 << j)) s[j].step++;
#pragma unroll
  for (int i = 0; i < 3; ++i)
    if (a.rmask & (1 << i)) r[i].step++;
  return true;
}

// Credit wait shared by LL and LL128: the slot about to be written must have
// been consumed NSLOTS steps ago.  Receives wait on their lines' flags, not
// on a counter.
template <int SC>
__device__ __forceinline__ bool waitCredits(const Ctx& c, Conn* s, int smask) {
  return syncConns<SC>(c, s, 0, s, smask);
}

// End of an LL / LL128 step.  The lines carry their own flags, so the data
// stores need not be drained before the counters; the barrier only makes sure
// every wave has read the received slot (its loads returned: their values
// were used) before the head store frees it.
template <int SC>
__device__ __forceinline__ bool finishFlagStep(const Ctx& c, Conn* r, Conn* s, int rmask, int smask,
                                               uint32_t consumedBytes = 0, bool ll128 = false) {
  __syncthreads();
  bool ok = !*abortWord(c);
  if constexpr (kJitter) {
    // poison the consumed lines: payload POISON, flag 0 (never current: the
    // first flag of a connection is 1); LL units are 8 bytes (data, flag),
    // LL128 lines carry their flag in bytes 120..127
    if (ok && rmask) {
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        if (!(rmask & (1 << i))) continue;
        const __amdgpu_buffer_rsrc_t rs = makeRsrc(r[i].fifo + (r[i].step % NSLOTS) * (uint64_t)c.slotB, c.slotB);
        for (uint32_t off = (uint32_t)c.tid * 16; off < consumedBytes; off += (uint32_t)c.nthreads * 16) {
          const bool flagWords = ll128 ? ((off / 16) % 8 == 7) : false;
          const u32x4 v = ll128 ? (flagWords ? u32x4{POISON, POISON, 0u, 0u} : u32x4{POISON, POISON, POISON, POISON})
                                : u32x4{POISON, 0u, POISON, 0u};
          __builtin_amdgcn_raw_buffer_store_b128(v, rs, off, 0, StoreAux<SC>::value);
        }
      }
      drainVmem();
      __syncthreads();
    }
    if (c.tid == 0) jitterPause();
  }
  if (c.tid == 0 && ok) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
      if (rmask & (1 << i)) stCtr<SC>(r[i].head(), r[i].step + 1);
#pragma unroll
    for (int j = 0; j < 3; ++j)
      if (smask & (1 << j)) stCtr<SC>(s[j].tail, s[j].step + 1);
  }
#pragma unroll
  for (int j = 0; j < 3; ++j)
    if (smask & (1 << j)) s[j].step++;
#pragma unroll
  for (int i = 0; i < 3; ++i)
    if (rmask & (1 << i)) r[i].step++;
  return ok;
}

// ------------------------------------------------------------------ LL datapath
// A lane handles LL_UNROLL pairs of 8-byte units (8 payload bytes, 16 FIFO
// bytes each) per pass, nthreads pairs apart so that a wave's accesses stay
// contiguous.  All loads of a pass are issued before any flag is checked: a
// receive is a round trip to memory, and one pair in flight per lane leaves
// the step latency-bound.

constexpr int LL_UNROLL = 4;

template <int SC, int DT, int OP>
__device__ bool stepLL(const Ctx& c, Conn* r, Conn* s, const StepArgs& a) {
  constexpr int E = ElemSize<DT>::value;
  constexpr int U = LL_UNROLL;
  if (!waitCredits<SC>(c, s, a.smask)) return false;
  const uint32_t slotB = c.slotB;
  const uint64_t npairs = (a.nbytes + 7) / 8;
  __amdgpu_buffer_rsrc_t rin[3], sout[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    rin[i] = makeRsrc(r[i].fifo + (r[i].step % NSLOTS) * (uint64_t)slotB, slotB);
    sout[i] = makeRsrc(s[i].fifo + (s[i].step % NSLOTS) * (uint64_t)slotB, slotB);
  }
  // user buffers: full 8-byte pieces through buffer accesses at any element
  // alignment, the short last piece element by element; reads are sc1 like
  // every other read of data another workgroup may have written
  const __amdgpu_buffer_rsrc_t bsrc = makeRsrc(a.src, (uint32_t)a.nbytes);
  const __amdgpu_buffer_rsrc_t bdst = makeRsrc(a.dst, (uint32_t)a.nbytes);
  const bool writeDst = a.dst && !(a.src == a.dst && a.rmask == 0);
  const uint64_t stride = (uint64_t)c.nthreads;
  bool alive = true;
  for (uint64_t p0 = c.tid; p0 < npairs; p0 += stride * U) {
    uint32_t acc[U][2];
    int valid[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t p = p0 + stride * u;
      const uint64_t off = p * 8;
      valid[u] = p < npairs ? (int)((a.nbytes - off) < 8 ? (a.nbytes - off) : 8) : 0;
      acc[u][0] = acc[u][1] = 0;
      if (a.src) {
        if (valid[u] == 8) {
          const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(bsrc, (uint32_t)off, 0, LOAD_AUX);
          acc[u][0] = v.x;
          acc[u][1] = v.y;
        } else if (valid[u] > 0) {
          loadPart<E, 2, true>(a.src + off, valid[u], acc[u]);
        }
      }
    }
    bool have = a.src != nullptr;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      if (alive && (a.rmask & (1 << i))) {
        const uint32_t flag = (uint32_t)(r[i].step + 1);
        uint64_t u0[U], u1[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const uint32_t uoff = (uint32_t)(p0 + stride * u) * 16;
          u0[u] = valid[u] ? ldUnit<SC>(rin[i], uoff) : ((uint64_t)flag << 32);
          u1[u] = valid[u] ? ldUnit<SC>(rin[i], uoff + 8) : ((uint64_t)flag << 32);
        }
        Spinner sp;
        for (;;) {
          uint32_t pend = 0;
#pragma unroll
          for (int u = 0; u < U; ++u)
            if ((uint32_t)(u0[u] >> 32) != flag || (uint32_t)(u1[u] >> 32) != flag) pend |= 1u << u;
          if (pend == 0) break;
          if (!sp.tick(c)) { alive = false; break; }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            if (pend & (1u << u)) {
              const uint32_t uoff = (uint32_t)(p0 + stride * u) * 16;
              u0[u] = ldUnit<SC>(rin[i], uoff);
              u1[u] = ldUnit<SC>(rin[i], uoff + 8);
            }
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (have) {
            acc[u][0] = redWord<DT, OP>(acc[u][0], (uint32_t)u0[u]);
            acc[u][1] = redWord<DT, OP>(acc[u][1], (uint32_t)u1[u]);
          } else {
            acc[u][0] = (uint32_t)u0[u];
            acc[u][1] = (uint32_t)u1[u];
          }
        }
        have = true;
      }
    }
    if (!alive) break;
    if constexpr (kJitter) jitterPause();  // a wave's line stores of this pass
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (valid[u] == 0) continue;
      const uint64_t p = p0 + stride * u;
      const uint64_t off = p * 8;
      if (writeDst) {
        if (valid[u] == 8) __builtin_amdgcn_raw_buffer_store_b64(u32x2{acc[u][0], acc[u][1]}, bdst, (uint32_t)off, 0, 0);
        else storePart<E, 2>(a.dst + off, valid[u], acc[u]);
      }
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        if (a.smask & (1 << j)) {
          const uint64_t flag = (uint64_t)(uint32_t)(s[j].step + 1) << 32;
          stUnit<SC>(sout[j], (uint32_t)p * 16, (uint64_t)acc[u][0] | flag);
          stUnit<SC>(sout[j], (uint32_t)p * 16 + 8, (uint64_t)acc[u][1] | flag);
        }
      }
    }
  }
  return finishFlagStep<SC>(c, r, s, a.rmask, a.smask, (uint32_t)(npairs * 16), false);
}

// ------------------------------------------------------------------ LL128 datapath
// Lane l of a wave handles 16 bytes (word pair l % 8) of line l / 8 of an
// 8-line group; lane 7 of each line carries 8 payload bytes and the 8-byte
// flag.  A pass covers nwaves * LL128_UNROLL groups, wave-major (group
// wave + nwaves * u), so a short step spreads over the waves and a long one
// keeps LL128_UNROLL groups in flight per wave.  Every line load of a pass is
// issued before any flag is checked, and only lines whose flag is still
// stale are read again.

constexpr int LL128_UNROLL = 4;

template <int SC, int DT, int OP>
__device__ bool stepLL128(const Ctx& c, Conn* r, Conn* s, const StepArgs& a) {
  constexpr int E = ElemSize<DT>::value;
  constexpr int U = LL128_UNROLL;
  if (!waitCredits<SC>(c, s, a.smask)) return false;
  const uint32_t slotB = c.slotB;
  const uint32_t nlines = (uint32_t)((a.nbytes + LL128_DATA - 1) / LL128_DATA);
  __amdgpu_buffer_rsrc_t rin[3], sout[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    rin[i] = makeRsrc(r[i].fifo + (r[i].step % NSLOTS) * (uint64_t)slotB, slotB);
    sout[i] = makeRsrc(s[i].fifo + (s[i].step % NSLOTS) * (uint64_t)slotB, slotB);
  }
  const __amdgpu_buffer_rsrc_t bsrc = makeRsrc(a.src, (uint32_t)a.nbytes);
  const __amdgpu_buffer_rsrc_t bdst = makeRsrc(a.dst, (uint32_t)a.nbytes);
  const bool writeDst = a.dst && !(a.src == a.dst && a.rmask == 0);
  const int g = c.lid >> 3, j = c.lid & 7;
  const int plen = (j < 7) ? 16 : 8;
  bool alive = true;
  for (uint32_t L0 = 0; L0 < nlines; L0 += (uint32_t)c.nwaves * 8 * U) {
    uint32_t acc[U][4];
    uint32_t lineOf[U];
    int valid[U];
    bool act[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t line = L0 + 8 * ((uint32_t)c.wave + (uint32_t)c.nwaves * u) + g;
      lineOf[u] = line;
      act[u] = line < nlines;
      const uint64_t payOff = (uint64_t)line * LL128_DATA + 16u * j;
      valid[u] = 0;
      if (act[u] && payOff < a.nbytes)
        valid[u] = (int)((a.nbytes - payOff) < (uint64_t)plen ? (a.nbytes - payOff) : plen);
      acc[u][0] = acc[u][1] = acc[u][2] = acc[u][3] = 0;
      if (a.src) {
        if (valid[u] == plen) {
          // user buffers: full pieces through buffer accesses at any element
          // alignment, a short piece element by element
          if (plen == 16) {
            const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(bsrc, (uint32_t)payOff, 0, LOAD_AUX);
            acc[u][0] = v.x;
            acc[u][1] = v.y;
            acc[u][2] = v.z;
            acc[u][3] = v.w;
          } else {
            const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(bsrc, (uint32_t)payOff, 0, LOAD_AUX);
            acc[u][0] = v.x;
            acc[u][1] = v.y;
          }
        } else if (valid[u] > 0) {
          loadPart<E, 4, true>(a.src + payOff, valid[u], acc[u]);
        }
      }
    }
    bool have = a.src != nullptr;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      if (alive && (a.rmask & (1 << i))) {
        const uint64_t flag = r[i].step + 1;
        u32x4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
          v[u] = act[u] ? ldLine16<SC>(rin[i], lineOf[u] * LL128_LINE + 16u * j) : u32x4{0, 0, 0, 0};
        Spinner sp;
        const uint64_t live = __ballot(1);
        for (;;) {
          // lane 7 of each line holds the flag; a line is re-read whole (one
          // 8-lane load) until its flag is current.  One ballot per group of
          // lines tells every lane its line's state and the wave whether all
          // lines are current.
          uint32_t pend = 0;
          bool allOk = true;
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const bool flagOk = !act[u] || j != 7 || ((((uint64_t)v[u].w << 32) | v[u].z) == flag);
            const uint64_t okMask = __ballot(flagOk);
            allOk = allOk && okMask == live;
            if (!((okMask >> (c.lid | 7)) & 1ull)) pend |= 1u << u;
          }
          if (allOk) break;
          if (__any(!sp.tick(c))) { alive = false; break; }
#pragma unroll
          for (int u = 0; u < U; ++u)
            if (pend & (1u << u)) v[u] = ldLine16<SC>(rin[i], lineOf[u] * LL128_LINE + 16u * j);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const uint32_t pw0 = v[u].x, pw1 = v[u].y, pw2 = (j < 7) ? v[u].z : 0u, pw3 = (j < 7) ? v[u].w : 0u;
          if (have) {
            acc[u][0] = redWord<DT, OP>(acc[u][0], pw0);
            acc[u][1] = redWord<DT, OP>(acc[u][1], pw1);
            acc[u][2] = redWord<DT, OP>(acc[u][2], pw2);
            acc[u][3] = redWord<DT, OP>(acc[u][3], pw3);
          } else {
            acc[u][0] = pw0;
            acc[u][1] = pw1;
            acc[u][2] = pw2;
            acc[u][3] = pw3;
          }
        }
        have = true;
      }
    }
    if (!alive) break;
    if constexpr (kJitter) jitterPause();  // a wave's line stores of this pass
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t line = lineOf[u];
      const uint64_t payOff = (uint64_t)line * LL128_DATA + 16u * j;
      if (writeDst && valid[u] > 0) {
        if (valid[u] == plen) {
          if (plen == 16)
            __builtin_amdgcn_raw_buffer_store_b128(u32x4{acc[u][0], acc[u][1], acc[u][2], acc[u][3]}, bdst, (uint32_t)payOff, 0, 0);
          else
            __builtin_amdgcn_raw_buffer_store_b64(u32x2{acc[u][0], acc[u][1]}, bdst, (uint32_t)payOff, 0, 0);
        } else {
          storePart<E, 4>(a.dst + payOff, valid[u], acc[u]);
        }
      }
      if (act[u]) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          if (a.smask & (1 << q)) {
            const uint64_t flag = s[q].step + 1;
            u32x4 w = {acc[u][0], acc[u][1], acc[u][2], acc[u][3]};
            if (j == 7) {
              w.z = (uint32_t)flag;
              w.w = (uint32_t)(flag >> 32);
            }
            stLine16<SC>(sout[q], line * LL128_LINE + 16u * j, w);
          }
        }
      }
    }
  }
  if (!alive) atomicOr(c.sAbort, 1);
  return finishFlagStep<SC>(c, r, s, a.rmask, a.smask, nlines * LL128_LINE, true);
}

template <int PROTO, int SC, int DT, int OP>
__device__ __forceinline__ bool step(const Ctx& c, Conn* r, Conn* s, const StepArgs& a) {
  if constexpr (PROTO == PROTO_SIMPLE) return stepSimple<SC, DT, OP>(c, r, s, a);
  else if constexpr (PROTO == PROTO_LL) return stepLL<SC, DT, OP>(c, r, s, a);
  else return stepLL128<SC, DT, OP>(c, r, s, a);
}

// ------------------------------------------------------------------ connections

__device__ __forceinline__ uint64_t connId(const Ctx& c, int receiver, int kind) {
  return ((uint64_t)c.lane * c.nranks + receiver) * NCONN + kind;
}

__device__ __forceinline__ char* fifoOf(const Ctx& c, int proto, int receiver, int kind, uint64_t fifoBytes) {
  const uint64_t lr = (uint64_t)c.lane * c.nranks + receiver;
  if (kind == 0) return c.comm->fifo[proto] + lr * fifoBytes;
  if (kind > NTREE_CONN) {  // ring k >= 1: its own block of lanes x ranks connections
    const uint64_t k = (uint64_t)(kind - NTREE_CONN);
    return c.comm->fifo[proto] + (k * (uint64_t)c.comm->maxLanes * c.nranks + lr) * fifoBytes;
  }
  return c.comm->treeFifo[proto] + (lr * NTREE_CONN + (kind - 1)) * fifoBytes;
}

// A channel's ring order (Section II-C): position of a rank, rank at a
// position (any integer, taken mod R).
struct RingView {
  const int8_t* rank;
  int q;     // this rank's position
  int R;
  int kind;  // connection kind of the ring's connections
  __device__ __forceinline__ int at(int k) const { return (int)rank[((k % R) + R) % R]; }
};
__device__ __forceinline__ RingView ringOf(const Ctx& c, const WorkItem& w) {
  RingView v;
  v.rank = c.comm->ringRank[w.ring];
  v.q = (int)uniform((uint32_t)(int32_t)c.comm->ringPos[w.ring][c.rank]);
  v.R = c.nranks;
  v.kind = ringKind(w.ring);
  return v;
}

// Thread 0 reads the step counters (a receiver's own head, a sender's own
// tail) and all threads pick them up from LDS.
template <int SC>
__device__ void setupConns(const Ctx& c, int proto, Conn* r, const int* rkind, Conn* s, const int* speer,
                           const int* skind, uint64_t* sStepsGeneric) {
  const uint64_t fifoBytes = (uint64_t)NSLOTS * c.slotB;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    if (rkind[i] >= 0) {
      uint64_t id = connId(c, c.rank, rkind[i]);
      r[i].fifo = fifoOf(c, proto, c.rank, rkind[i], fifoBytes);
      r[i].tail = c.comm->ctr + id * CTR_RECORD_U64;
    }
    if (speer[i] >= 0) {
      uint64_t id = connId(c, speer[i], skind[i]);
      s[i].fifo = fifoOf(c, proto, speer[i], skind[i], fifoBytes);
      s[i].tail = c.comm->ctr + id * CTR_RECORD_U64;
    }
  }
  // a receive end starts at the steps it consumed (head), a send end at the
  // steps it produced (tail)
  LdsU64* sSteps = (LdsU64*)sStepsGeneric;
  if (c.tid == 0) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      sSteps[i] = rkind[i] >= 0 ? ldCtr<SC>(r[i].head()) : 0;
      sSteps[3 + i] = speer[i] >= 0 ? ldCtr<SC>(s[i].tail) : 0;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    r[i].step = uniform64(sSteps[i]);
    s[i].step = uniform64(sSteps[3 + i]);
  }
  __syncthreads();
}

__device__ __forceinline__ uint64_t ceilDiv(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
__device__ __forceinline__ uint64_t umin(uint64_t a, uint64_t b) { return a < b ? a : b; }
__device__ __forceinline__ uint64_t roundUp(uint64_t a, uint64_t b) { return ceilDiv(a, b) * b; }

// ------------------------------------------------------------------ algorithms

// Ring AllReduce, Section V-E table: step 0 send, 1..k-2 recvReduceSend,
// k-1 recvReduceCopySend, k..2k-3 recvCopySend, 2k-2 recv.  At step t the
// rank at ring position q works on segment (q - 1 - t) mod k of the loop.
template <int PROTO, int SC, int DT, int OP>
__device__ void ringAllReduce(const Ctx& c, const WorkItem& w, const CollArgs& args, uint64_t* sSteps) {
  const RingView ring = ringOf(c, w);
  const int R = c.nranks, me = c.rank, q = ring.q, nxt = ring.at(q + 1);
  Conn r[3], s[3];
  const int rk[3] = {ring.kind, -1, -1}, sp[3] = {nxt, -1, -1}, sk[3] = {ring.kind, -1, -1};
  setupConns<SC>(c, PROTO, r, rk, s, sp, sk, sSteps);
  const uint64_t E = w.elemBytes, A = 16 / E, K = w.chunk;
  const uint64_t loopCount = (uint64_t)R * K;
  const uint64_t full = w.chCount / loopCount, rem = w.chCount - full * loopCount;
  const uint64_t nloops = full + (rem ? 1 : 0);
  const bool direct = (PROTO == PROTO_SIMPLE) && w.direct;
  const char* sendb = uniformPtr(args.send[me]);
  char* recvb = uniformPtr(args.recv[me]);
  char* nextRecv = uniformPtr(args.recv[nxt]);
  for (uint64_t l = 0; l < nloops; ++l) {
    const uint64_t base = l * loopCount;
    const uint64_t Kl = (l < full) ? K : roundUp(ceilDiv(rem, R), A);
    const uint64_t lim = (l < full) ? loopCount : rem;
    for (int t = 0; t < 2 * R - 1; ++t) {
      const int sidx = ((q - 1 - t) % R + 2 * R) % R;
      const uint64_t a0 = umin(lim, (uint64_t)sidx * Kl), b0 = umin(lim, (uint64_t)(sidx + 1) * Kl);
      const uint64_t off = (w.chOffset + base + a0) * E;
      StepArgs a{};
      a.nbytes = (b0 - a0) * E;
      if (t == 0) {                         // send
        a.src = sendb + off;
        a.smask = 1;
      } else if (t <= R - 2) {              // recvReduceSend
        a.src = sendb + off;
        a.rmask = 1;
        a.smask = 1;
      } else if (t == R - 1) {              // recvReduceCopySend
        a.src = sendb + off;
        a.dst = recvb + off;
        a.rmask = 1;
        a.smask = 1;
        if (direct) a.sendDirect[0] = nextRecv + off;
      } else if (t <= 2 * R - 3) {          // recvCopySend / directRecvCopySend
        a.dst = recvb + off;
        a.rmask = 1;
        a.smask = 1;
        if (direct) {
          a.recvDirect = true;
          a.sendDirect[0] = nextRecv + off;
        }
      } else {                              // recv / directRecv
        a.dst = recvb + off;
        a.rmask = 1;
        a.recvDirect = direct;
      }
      if (!step<PROTO, SC, DT, OP>(c, r, s, a)) return;
    }
  }
}

// Ring ReduceScatter, Section V-E table: step 0 send, 1..k-2 recvReduceSend,
// k-1 recvReduceCopy; at step t the rank at ring position q works on the
// block of the rank at position (q - 1 - t) mod k.
template <int PROTO, int SC, int DT, int OP>
__device__ void ringReduceScatter(const Ctx& c, const WorkItem& w, const CollArgs& args, uint64_t* sSteps) {
  const RingView ring = ringOf(c, w);
  const int R = c.nranks, me = c.rank, q = ring.q, nxt = ring.at(q + 1);
  Conn r[3], s[3];
  const int rk[3] = {ring.kind, -1, -1}, sp[3] = {nxt, -1, -1}, sk[3] = {ring.kind, -1, -1};
  setupConns<SC>(c, PROTO, r, rk, s, sp, sk, sSteps);
  const uint64_t E = w.elemBytes, n = w.count, K = w.chunk;
  const char* sendb = uniformPtr(args.send[me]);
  char* recvb = uniformPtr(args.recv[me]);
  for (uint64_t a0 = 0; a0 < w.chCount; a0 += K) {
    const uint64_t len = umin(K, w.chCount - a0);
    for (int t = 0; t < R; ++t) {
      const int blk = ring.at(q - 1 - t);
      StepArgs a{};
      a.nbytes = len * E;
      a.src = sendb + ((uint64_t)blk * n + w.chOffset + a0) * E;
      a.rmask = t > 0 ? 1 : 0;
      a.smask = t < R - 1 ? 1 : 0;
      if (t == R - 1) a.dst = recvb + (w.chOffset + a0) * E;
      if (!step<PROTO, SC, DT, OP>(c, r, s, a)) return;
    }
  }
}

// Ring AllGather, Section V-E table: step 0 copySend (send in place),
// 1..k-2 recvCopySend, k-1 recv; at step t rank p handles block (p - t) mod k.
// Units are bytes.
template <int PROTO, int SC, int DT, int OP>
__device__ void ringAllGather(const Ctx& c, const WorkItem& w, const CollArgs& args, uint64_t* sSteps) {
  const RingView ring = ringOf(c, w);
  const int R = c.nranks, me = c.rank, q = ring.q, nxt = ring.at(q + 1);
  Conn r[3], s[3];
  const int rk[3] = {ring.kind, -1, -1}, sp[3] = {nxt, -1, -1}, sk[3] = {ring.kind, -1, -1};
  setupConns<SC>(c, PROTO, r, rk, s, sp, sk, sSteps);
  const uint64_t n = w.count, K = w.chunk;
  const bool direct = (PROTO == PROTO_SIMPLE) && w.direct;
  const char* sendb = uniformPtr(args.send[me]);
  char* recvb = uniformPtr(args.recv[me]);
  char* nextRecv = uniformPtr(args.recv[nxt]);
  for (uint64_t a0 = 0; a0 < w.chCount; a0 += K) {
    const uint64_t len = umin(K, w.chCount - a0);
    for (int t = 0; t < R; ++t) {
      const int blk = ring.at(q - t);
      const uint64_t off = (uint64_t)blk * n + w.chOffset + a0;
      StepArgs a{};
      a.nbytes = len;
      a.dst = recvb + off;
      if (t == 0) {
        a.src = sendb + w.chOffset + a0;
        a.smask = 1;
        if (direct) a.sendDirect[0] = nextRecv + off;
      } else if (t <= R - 2) {
        a.rmask = 1;
        a.smask = 1;
        if (direct) {
          a.recvDirect = true;
          a.sendDirect[0] = nextRecv + off;
        }
      } else {
        a.rmask = 1;
        a.recvDirect = direct;
      }
      if (!step<PROTO, SC, DT, OP>(c, r, s, a)) return;
    }
  }
}

// Ring Broadcast, Section V-E table: a chain along the ring from the root;
// root copySend (send in place), middle recvCopySend, last recv.  Bytes.
// With direct sends the root's copySend would be the chain's slowest stage
// (a read and two writes per byte, against a read and a write for a middle
// rank and none for the last): the root's copy into its own receive buffer
// needs no synchronisation, since the input is there from the start, so the
// last rank, which otherwise only waits, makes it.
template <int PROTO, int SC, int DT, int OP>
__device__ void ringBroadcast(const Ctx& c, const WorkItem& w, const CollArgs& args, uint64_t* sSteps) {
  const RingView ring = ringOf(c, w);
  const int R = c.nranks, me = c.rank, nxt = ring.at(ring.q + 1);
  const int pos = ((ring.q - (int)c.comm->ringPos[w.ring][w.root]) % R + R) % R;
  Conn r[3], s[3];
  const int rk[3] = {pos > 0 ? ring.kind : -1, -1, -1}, sp[3] = {pos < R - 1 ? nxt : -1, -1, -1},
            sk[3] = {ring.kind, -1, -1};
  setupConns<SC>(c, PROTO, r, rk, s, sp, sk, sSteps);
  const uint64_t K = w.chunk;
  const bool direct = (PROTO == PROTO_SIMPLE) && w.direct;
  const char* rootSend = uniformPtr(args.send[w.root]);
  char* rootRecv = uniformPtr(args.recv[w.root]);
  const bool lastCopiesRoot = direct && rootSend != rootRecv;
  for (uint64_t a0 = 0; a0 < w.chCount; a0 += K) {
    const uint64_t len = umin(K, w.chCount - a0);
    const uint64_t off = w.chOffset + a0;
    StepArgs a{};
    a.nbytes = len;
    a.dst = uniformPtr(args.recv[me]) + off;
    if (lastCopiesRoot && pos == R - 1) {
      PtrList in, out;
      in.add(rootSend + off);
      out.add(rootRecv + off);
      reduceCopyN<DT_U8, OP_COPY, SC>(c, in, out, len);
    }
    if (pos == 0) {
      a.src = uniformPtr(args.send[me]) + off;
      a.smask = 1;
      if (lastCopiesRoot) a.dst = nullptr;
    } else {
      a.rmask = 1;
      a.recvDirect = direct;
      if (pos < R - 1) a.smask = 1;
    }
    if (direct && a.smask) a.sendDirect[0] = uniformPtr(args.recv[nxt]) + off;
    if (!step<PROTO, SC, DT, OP>(c, r, s, a)) return;
  }
}

// Ring Reduce, Section V-E table: a chain along the ring from the root's
// successor to the root; initiator send, middle recvReduceSend, root
// recvReduceCopy.
template <int PROTO, int SC, int DT, int OP>
__device__ void ringReduce(const Ctx& c, const WorkItem& w, const CollArgs& args, uint64_t* sSteps) {
  const RingView ring = ringOf(c, w);
  const int R = c.nranks, me = c.rank, nxt = ring.at(ring.q + 1);
  const int pos = ((ring.q - (int)c.comm->ringPos[w.ring][w.root] - 1) % R + 2 * R) % R;
  Conn r[3], s[3];
  const int rk[3] = {pos > 0 ? ring.kind : -1, -1, -1}, sp[3] = {pos < R - 1 ? nxt : -1, -1, -1},
            sk[3] = {ring.kind, -1, -1};
  setupConns<SC>(c, PROTO, r, rk, s, sp, sk, sSteps);
  const uint64_t E = w.elemBytes, K = w.chunk;
  for (uint64_t a0 = 0; a0 < w.chCount; a0 += K) {
    const uint64_t len = umin(K, w.chCount - a0);
    const uint64_t off = (w.chOffset + a0) * E;
    StepArgs a{};
    a.nbytes = len * E;
    a.src = uniformPtr(args.send[me]) + off;
    a.rmask = pos > 0 ? 1 : 0;
    a.smask = pos < R - 1 ? 1 : 0;
    if (pos == R - 1) a.dst = uniformPtr(args.recv[me]) + off;
    if (!step<PROTO, SC, DT, OP>(c, r, s, a)) return;
  }
}

// Tree AllReduce, Section V-E table: root recvReduceCopySend, middle
// recvReduceSend then recvCopySend, leaf send then recv.  The reduction at a
// node is op(op(local, first child), second child).  Chunk iterations are
// software-pipelined: the upward step of chunk j precedes the downward step
// of chunk j - (NSLOTS - 1), which cannot deadlock with NSLOTS slots.
template <int PROTO, int SC, int DT, int OP>
__device__ void treeAllReduce(const Ctx& c0, const WorkItem& w, const CollArgs& args, uint64_t* sSteps) {
  // A channel runs fused (one workgroup per rank takes both phases, the
  // downward step of iteration j - lag after the upward step of iteration j)
  // or split: the up half and the down half run on two lanes of one XCD at
  // once, both addressing the connections of the up half's lane.
  if (w.role == ROLE_IDLE) return;
  Ctx c = c0;
  if (w.role != ROLE_FUSED) c.lane = w.connLane;
  const bool up = w.role != ROLE_DOWN, down = w.role != ROLE_UP;
  const int me = c.rank, t = w.tree;
  const int par = c.comm->parent[t][me];
  const int nk = c.comm->nchild[t][me];
  const int k0 = c.comm->child[t][me][0], k1 = c.comm->child[t][me][1];
  if (!up && par < 0) return;  // the root's downward sends belong to its upward step
  // receive side: 0,1 up from children; 2 down from parent
  const int rk[3] = {up && nk > 0 ? 1 + 3 * t : -1, up && nk > 1 ? 2 + 3 * t : -1,
                     down && par >= 0 ? 3 + 3 * t : -1};
  // send side: 0 up to parent; 1,2 down to children (the root's in its upward step)
  const bool sendsDown = down || par < 0;
  const int sp[3] = {up ? par : -1, sendsDown && nk > 0 ? k0 : -1, sendsDown && nk > 1 ? k1 : -1};
  const int sk[3] = {up && par >= 0 ? 1 + 3 * t + c.comm->childIdx[t][me] : -1, 3 + 3 * t, 3 + 3 * t};
  Conn r[3], s[3];
  setupConns<SC>(c, PROTO, r, rk, s, sp, sk, sSteps);
  const int upR = (nk > 0 ? 1 : 0) | (nk > 1 ? 2 : 0);
  const int downS = (nk > 0 ? 2 : 0) | (nk > 1 ? 4 : 0);
  const uint64_t E = w.elemBytes, K = w.chunk;
  const uint64_t nch = ceilDiv(w.chCount, K);
  const uint64_t lag = (up && down) ? NSLOTS - 1 : 0;
  const char* sendb = uniformPtr(args.send[me]);
  char* recvb = uniformPtr(args.recv[me]);
  for (uint64_t j = 0; j < nch + lag; ++j) {
    if (up && j < nch) {
      const uint64_t a0 = j * K, len = umin(K, w.chCount - a0);
      const uint64_t off = (w.chOffset + a0) * E;
      StepArgs a{};
      a.nbytes = len * E;
      a.src = sendb + off;
      a.rmask = upR;
      if (par < 0) {             // root: recvReduceCopySend
        a.dst = recvb + off;
        a.smask = downS;
      } else {                   // middle: recvReduceSend; leaf: send
        a.smask = 1;
      }
      if (!step<PROTO, SC, DT, OP>(c, r, s, a)) return;
    }
    if (down && j >= lag && par >= 0) {
      const uint64_t jd = j - lag, a0 = jd * K, len = umin(K, w.chCount - a0);
      const uint64_t off = (w.chOffset + a0) * E;
      StepArgs a{};
      a.nbytes = len * E;
      a.dst = recvb + off;
      a.rmask = 4;
      a.smask = downS;           // middle: recvCopySend; leaf: recv
      if (!step<PROTO, SC, DT, OP>(c, r, s, a)) return;
    }
  }
}

// Point-to-point transfer (Section II-A Send/Recv) in the spirit of
// P2P_DIRECT (Section IV-A): the bytes go straight from the sender's buffer
// into the receiver's, with no intermediate FIFO.  Both buffers belong to the
// same launch, whose start and end order them against every other operation,
// so no workgroup has to wait for another: every workgroup of the lane copies
// a 1/R share of the item's range, in slot-sized pieces.  Units are bytes.
template <int SC>
__device__ void p2pTransfer(const Ctx& c, const WorkItem& w, const CollArgs& args) {
  const uint64_t n = w.chCount, R = (uint64_t)c.nranks;
  const uint64_t per = (n + R - 1) / R;
  const uint64_t share = (per + 15) / 16 * 16;
  const uint64_t b0 = umin(n, (uint64_t)c.rank * share), b1 = umin(n, ((uint64_t)c.rank + 1) * share);
  const char* src = uniformPtr(args.send[w.root]) + w.chOffset;
  char* dst = uniformPtr(args.recv[w.peer]) + w.chOffset;
  for (uint64_t a0 = b0; a0 < b1; a0 += w.chunk) {
    PtrList in, out;
    in.add(src + a0);
    out.add(dst + a0);
    reduceCopyN<DT_U8, OP_COPY, SC>(c, in, out, umin(w.chunk, b1 - a0));
  }
}

template <int PROTO, int SC, int DT, int OP>
__device__ __noinline__ void runItem(const Ctx& c0, const WorkItem& w0, const CollArgs& args, uint64_t* sSteps) {
  Ctx c = uniformCtx(c0);
  const WorkItem w = uniformItem(w0);
  // an item uses ring connections or tree connections, never both
  c.slotB = uniform((uint32_t)(w.algo == ALGO_TREE ? c.comm->treeSlotBytes[PROTO] : c.comm->slotBytes[PROTO]));
  if constexpr (OP == OP_COPY) {
    if (w.coll == COLL_ALLGATHER) ringAllGather<PROTO, SC, DT, OP>(c, w, args, sSteps);
    else if (w.coll == COLL_BROADCAST) ringBroadcast<PROTO, SC, DT, OP>(c, w, args, sSteps);
    else if constexpr (PROTO == PROTO_SIMPLE) {
      if (w.coll == COLL_SENDRECV) p2pTransfer<SC>(c, w, args);
    }
  } else {
    if (w.coll == COLL_ALLREDUCE) {
      if (w.algo == ALGO_TREE) treeAllReduce<PROTO, SC, DT, OP>(c, w, args, sSteps);
      else ringAllReduce<PROTO, SC, DT, OP>(c, w, args, sSteps);
    } else if (w.coll == COLL_REDUCESCATTER) {
      ringReduceScatter<PROTO, SC, DT, OP>(c, w, args, sSteps);
    } else if (w.coll == COLL_REDUCE) {
      ringReduce<PROTO, SC, DT, OP>(c, w, args, sSteps);
    }
  }
}

template <int PROTO, int SC>
__device__ void dispatchType(const Ctx& c, const WorkItem& w, const CollArgs& args, uint64_t* sSteps) {
  const int key = w.dtype * 4 + w.op;
  switch (key) {
    case DT_I32 * 4 + OP_SUM: runItem<PROTO, SC, DT_I32, OP_SUM>(c, w, args, sSteps); break;
    case DT_I32 * 4 + OP_MAX: runItem<PROTO, SC, DT_I32, OP_MAX>(c, w, args, sSteps); break;
    case DT_F32 * 4 + OP_SUM: runItem<PROTO, SC, DT_F32, OP_SUM>(c, w, args, sSteps); break;
    case DT_F32 * 4 + OP_MAX: runItem<PROTO, SC, DT_F32, OP_MAX>(c, w, args, sSteps); break;
    case DT_BF16 * 4 + OP_SUM: runItem<PROTO, SC, DT_BF16, OP_SUM>(c, w, args, sSteps); break;
    case DT_BF16 * 4 + OP_MAX: runItem<PROTO, SC, DT_BF16, OP_MAX>(c, w, args, sSteps); break;
    case DT_U8 * 4 + OP_COPY: runItem<PROTO, SC, DT_U8, OP_COPY>(c, w, args, sSteps); break;
    default: break;
  }
}

__device__ __forceinline__ void dispatchItem(const Ctx& c, const WorkItem& w, const CollArgs& args, uint64_t* sSteps) {
  // XCD scope only where the set runs with the lane map (every lane's
  // workgroups on one XCD) and the plan chose it for this item
  if (c.comm->scope == SCOPE_XCD && w.scope == SCOPE_XCD) {
    switch (w.proto) {
      case PROTO_SIMPLE: dispatchType<PROTO_SIMPLE, SCOPE_XCD>(c, w, args, sSteps); break;
      case PROTO_LL: dispatchType<PROTO_LL, SCOPE_XCD>(c, w, args, sSteps); break;
      default: dispatchType<PROTO_LL128, SCOPE_XCD>(c, w, args, sSteps); break;
    }
  } else {
    switch (w.proto) {
      case PROTO_SIMPLE: dispatchType<PROTO_SIMPLE, SCOPE_DEVICE>(c, w, args, sSteps); break;
      case PROTO_LL: dispatchType<PROTO_LL, SCOPE_DEVICE>(c, w, args, sSteps); break;
      default: dispatchType<PROTO_LL128, SCOPE_DEVICE>(c, w, args, sSteps); break;
    }
  }
}

// Lane map.  With the XCD map, lane l lives on XCD (l % 8): every workgroup
// reads the XCD it actually runs on and claims the next free (lane, rank)
// role of that XCD from a per-XCD counter, so a lane's workgroups share one L2
// by construction, whatever XCD the dispatcher starts from.  The counters
// only grow; `claimBase` (the claims of all earlier launches, equal for every
// XCD since launches are multiples of 8 workgroups dispatched round-robin) is
// subtracted.  A claim beyond the launch's `perXcd` roles means the
// workgroups were not spread evenly: that workgroup records an error and
// raises the abort word so no lane waits on a role nobody holds.
// Without the map, workgroup w is lane w / R, rank w % R.
__device__ __forceinline__ bool claimRole(const DevComm* comm, uint32_t xcdMap, uint64_t claimBase, uint32_t perXcd,
                                          uint32_t R, uint32_t* lane, uint32_t* rank, uint32_t* sRole) {
  if (!xcdMap) {
    *lane = blockIdx.x / R;
    *rank = blockIdx.x % R;
    return true;
  }
  if (threadIdx.x == 0) {
    uint32_t x;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(x));
    x &= 7u;
    const uint64_t old = atomicAdd((unsigned long long*)(comm->claim + (uint64_t)x * CLAIM_STRIDE_U64), 1ull);
    const uint64_t slot = old - claimBase;
    uint32_t role = 0xFFFFFFFFu;
    if (slot < perXcd) {
      role = ((x + 8u * (uint32_t)(slot / R)) << 8) | (uint32_t)(slot % R);
    } else {
      orSystem32(comm->errorWord, ERR_PLACEMENT);
      __hip_atomic_store(comm->abortFlag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    *sRole = role;
  }
  __syncthreads();
  const uint32_t role = *sRole;
  if (role == 0xFFFFFFFFu) return false;
  *lane = role >> 8;
  *rank = role & 0xFFu;
  return true;
}

// ------------------------------------------------------------------ kernel

__global__ void __launch_bounds__(1024) collKernel(const LaunchDesc d) {
  __shared__ WorkItem sItem;
  __shared__ CollArgs sArgs;
  __shared__ uint64_t sSteps[6];
  __shared__ int sAbort;
  __shared__ uint32_t sRole;
  __shared__ uint64_t sWait;

  const uint32_t R = d.nranks;
  const DevComm* comm = d.comm;
  uint32_t lane, rank;
  if (!claimRole(comm, d.xcdMap, d.claimBase, d.perXcd, R, &lane, &rank, &sRole)) return;
  if (lane >= d.nlanes) return;
  if ((comm->deadMask >> rank) & 1u) return;

  Ctx c;
  c.comm = comm;
  c.rank = (int)rank;
  c.lane = (int)lane;
  c.nranks = (int)R;
  c.tid = threadIdx.x;
  c.nthreads = blockDim.x;
  c.wave = threadIdx.x >> 6;
  c.nwaves = (blockDim.x + 63) >> 6;
  c.lid = threadIdx.x & 63;
  c.sAbort = &sAbort;
  c.sWait = d.profile ? &sWait : nullptr;
  if (threadIdx.x == 0) {
    sAbort = 0;
    sWait = 0;
  }
  const uint64_t tStart = d.profile ? nowTicks() : 0;
  uint32_t nrun = 0;

  const bool inl = d.items == nullptr;
  const uint32_t first = inl ? lane : d.laneStart[lane];
  const uint32_t last = inl ? lane + 1 : d.laneStart[lane + 1];
  for (uint32_t it = first; it < last; ++it) {
    __syncthreads();
    const WorkItem* src = inl ? &d.inlineItems[it] : &d.items[it];
    if (threadIdx.x < sizeof(WorkItem) / 4) ((uint32_t*)&sItem)[threadIdx.x] = ((const uint32_t*)src)[threadIdx.x];
    __syncthreads();
    const CollArgs* as = inl ? &d.inlineArgs : &d.args[sItem.argsIndex];
    if (threadIdx.x < sizeof(CollArgs) / 8) ((uint64_t*)&sArgs)[threadIdx.x] = ((const uint64_t*)as)[threadIdx.x];
    __syncthreads();
    dispatchItem(c, sItem, sArgs, sSteps);
    drainVmem();  // the item's stores complete before the next item reads counters
    __syncthreads();
    if (*(volatile int*)&sAbort) break;
    if (threadIdx.x == 0 && d.stamps && sItem.doneIndex != 0xFFFFFFFFu)
      d.stamps[(uint64_t)sItem.doneIndex * R + rank] = nowTicks();
    ++nrun;
  }
  if (d.profile && threadIdx.x == 0) {
    // this workgroup's span, the part of it spent waiting for counters, and
    // its item count
    uint64_t* rec = d.profile + ((uint64_t)lane * R + rank) * PROFILE_WORDS;
    rec[0] = tStart;
    rec[1] = nowTicks();
    rec[2] = sWait;
    rec[3] = nrun;
  }
}

// ------------------------------------------------------------------ serving kernel
// Persistent: every (lane, rank) workgroup waits for its lane's next posted
// entry, runs it like any work item, and publishes completion.  The lane's
// leader (rank 0) alone decides when the lane stops taking work: on the
// host's stop word, on the idle word (raised by the first leader that waited
// `idleTicks` without work: a lane whose workgroups left could not run what
// the host posts next, so the whole grid ends together and the host
// relaunches it), or on an abort or a failed wait; it then stores the exit
// marker into the lane's release counter.  The lane's other workgroups leave
// only on that marker, the host's stop word (raised once every request has
// completed) or a failure, so an entry the leader accepted always finds its
// whole lane.

__device__ __forceinline__ uint64_t ldSystem64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ void __launch_bounds__(1024) serveKernel(const ServeDesc d) {
  __shared__ WorkItem sItem;
  __shared__ CollArgs sArgs;
  __shared__ uint64_t sSteps[6];
  __shared__ int sAbort;
  __shared__ int sCmd;
  __shared__ uint32_t sRole;

  const uint32_t R = d.nranks;
  uint32_t lane, rank;
  if (!claimRole(d.comm, d.xcdMap, d.claimBase, d.perXcd, R, &lane, &rank, &sRole)) return;
  if (lane >= d.nlanes) return;
  if ((d.comm->deadMask >> rank) & 1u) return;  // test hook: a rank that never shows up
  Ctx c;
  c.comm = d.comm;
  c.rank = (int)rank;
  c.lane = (int)lane;
  c.nranks = (int)R;
  c.tid = threadIdx.x;
  c.nthreads = blockDim.x;
  c.wave = threadIdx.x >> 6;
  c.nwaves = (blockDim.x + 63) >> 6;
  c.lid = threadIdx.x & 63;
  c.sAbort = &sAbort;
  c.sWait = nullptr;
  if (threadIdx.x == 0) sAbort = 0;
  const bool leader = rank == 0;
  uint64_t* dbg = d.dbg + ((uint64_t)lane * R + rank) * SERVE_STRIDE_U64;
  uint64_t* laneSeq = d.laneSeq + (uint64_t)lane * SERVE_STRIDE_U64;
  uint64_t seq = d.startSeq[lane];
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) {
      // wait for entry `seq`: the leader watches the host's posted counter,
      // the others the leader's release counter in device memory
      int cmd = 0;
      const uint64_t t0 = nowTicks();
      for (uint32_t it = 0;; ++it) {
        const uint64_t p = leader ? ldSystem64(d.posted + (uint64_t)lane * SERVE_STRIDE_U64) : ldAgent(laneSeq);
        if ((it & 1023u) == 0) {
          __hip_atomic_store(dbg, p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
          __hip_atomic_store(dbg + 2, (uint64_t)it, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        if (!leader && (p & SERVE_EXIT)) break;  // the leader closed the lane
        if (p > seq) {
          cmd = 1;
          break;
        }
        // back off once the lane has been idle for a while (~100 us)
        if (it < 2048u) __builtin_amdgcn_s_sleep(2);
        else __builtin_amdgcn_s_sleep(16);
        if ((it & 63u) == 63u) {
          if (ldSystem32(d.stop)) break;
          // an abort, or a failed wait anywhere (timeout): the whole grid leaves
          if (ldSystem32(d.comm->abortFlag) || ldSystem32(d.comm->errorWord)) break;
          if (leader) {
            if (ldSystem32(d.idle)) break;
            if (nowTicks() - t0 > d.idleTicks) {
              __hip_atomic_store(d.idle, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
              break;
            }
          }
        }
      }
      if (cmd) {
        __hip_atomic_store(dbg + 1, seq + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(dbg + 3, nowTicks(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      } else if (leader) {
        stAgent(laneSeq, SERVE_EXIT | seq);  // release the lane's other workgroups for good
      }
      sCmd = cmd;
    }
    __syncthreads();
    if (sCmd != 1) break;
    const uint64_t slot = (uint64_t)lane * SERVE_QUEUE + seq % SERVE_QUEUE;
    constexpr uint32_t kItemWords = sizeof(WorkItem) / 4, kArgWords = sizeof(CollArgs) / 8;
    if (leader) {
      // host entry -> LDS and the device mirror, then release the lane
      const ServeEntry* e = d.queue + slot;
      ServeEntry* m = d.mirror + slot;
      if (threadIdx.x < kItemWords) {
        const uint32_t w = __hip_atomic_load(((const uint32_t*)&e->item) + threadIdx.x, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_SYSTEM);
        ((uint32_t*)&sItem)[threadIdx.x] = w;
        __hip_atomic_store(((uint32_t*)&m->item) + threadIdx.x, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      if (threadIdx.x < kArgWords) {
        const uint64_t w = ldSystem64(((const uint64_t*)&e->args) + threadIdx.x);
        ((uint64_t*)&sArgs)[threadIdx.x] = w;
        stAgent(((uint64_t*)&m->args) + threadIdx.x, w);
      }
      drainVmem();
      __syncthreads();
      if (threadIdx.x == 0) stAgent(laneSeq, seq + 1);
    } else {
      const ServeEntry* m = d.mirror + slot;
      if (threadIdx.x < kItemWords)
        ((uint32_t*)&sItem)[threadIdx.x] =
            __hip_atomic_load(((const uint32_t*)&m->item) + threadIdx.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (threadIdx.x < kArgWords) ((uint64_t*)&sArgs)[threadIdx.x] = ldAgent(((const uint64_t*)&m->args) + threadIdx.x);
    }
    __syncthreads();
    dispatchItem(c, sItem, sArgs, sSteps);
    drainVmem();
    __syncthreads();
    if (*(volatile int*)&sAbort) break;
    if (threadIdx.x == 0) {
      __hip_atomic_store(dbg + 4, nowTicks(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      // outputs visible to the host and to later kernels before completion
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
      __hip_atomic_store(d.done + ((uint64_t)lane * R + rank) * SERVE_STRIDE_U64, seq + 1, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_SYSTEM);
    }
    ++seq;
  }
}

// ------------------------------------------------------------------ probes

__global__ void xccProbeKernel(int* ids, int n) {
  uint32_t x;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(x));
  if (threadIdx.x == 0 && (int)blockIdx.x < n) ids[blockIdx.x] = (int)(x & 0xF);
}

// LL128 tear probe: workgroup w < pairs writes, workgroup pairs + w reads
// `lines` lines per round (workgroups are dispatched round-robin over the 8
// XCDs, so with pairs a multiple of 8 each pair shares an XCD, with pairs = 4
// it does not).  SC picks the store policy of the protocol's lines.  Payload word q of line i in
// round r is a hash of (r, i, q); a line whose flag is current but whose
// payload differs is a torn line.  The writer waits for the reader's ack
// before reusing the buffer.  Every wait is bounded by `maxTicks`.
__device__ __forceinline__ uint32_t tearHash(uint32_t r, uint32_t i, uint32_t q) {
  uint32_t h = r * 0x9E3779B1u ^ (i * 0x85EBCA77u) ^ (q * 0xC2B2AE3Du);
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 13;
  return h;
}

template <int SC>
__global__ void __launch_bounds__(256) tearProbeKernel(char* bufs, uint64_t* acks, int pairs, int lines, int rounds,
                                                        unsigned long long* counts, uint64_t maxTicks,
                                                        uint32_t* failed) {
  // pairing: writer w = blockIdx.x < pairs, reader = pairs + w
  const int w = blockIdx.x % pairs;
  const bool writer = (int)blockIdx.x < pairs;
  if ((int)blockIdx.x >= 2 * pairs) return;
  const uint32_t bytes = (uint32_t)lines * LL128_LINE;
  __amdgpu_buffer_rsrc_t rs = makeRsrc(bufs + (uint64_t)w * bytes, bytes);
  uint64_t* ack = acks + (uint64_t)w * 32;
  const int lid = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const int g = lid >> 3, j = lid & 7;
  __shared__ int sFail;
  if (threadIdx.x == 0) sFail = 0;
  __syncthreads();
  unsigned long long torn = 0, checked = 0;
  for (int r = 0; r < rounds; ++r) {
    const uint64_t flag = (uint64_t)r + 1;
    if (writer) {
      if (threadIdx.x == 0) {
        uint64_t t0 = nowTicks();
        while (ldAgent(ack) < (uint64_t)r) {
          __builtin_amdgcn_s_sleep(1);
          if (nowTicks() - t0 > maxTicks) { sFail = 1; break; }
        }
      }
      __syncthreads();
      if (sFail) break;
      for (int L0 = wave * 8; L0 < lines; L0 += nwaves * 8) {
        const int line = L0 + g;
        if (line < lines) {
          u32x4 v = {tearHash(r, line, 4 * j), tearHash(r, line, 4 * j + 1), tearHash(r, line, 4 * j + 2),
                     tearHash(r, line, 4 * j + 3)};
          if (j == 7) {
            v.z = (uint32_t)flag;
            v.w = (uint32_t)(flag >> 32);
          }
          stLine16<SC>(rs, line * LL128_LINE + 16 * j, v);
        }
      }
    } else {
      for (int L0 = wave * 8; L0 < lines; L0 += nwaves * 8) {
        const int line = L0 + g;
        const bool act = line < lines;
        const uint32_t loff = (uint32_t)line * LL128_LINE + 16u * j;
        u32x4 v = act ? ldLine16<SC>(rs, loff) : u32x4{0, 0, 0, 0};
        const uint64_t t0 = nowTicks();
        bool tornSeen = false;
        for (;;) {
          const int flagOk = (!act || j != 7 || ((((uint64_t)v.w << 32) | v.z) == flag)) ? 1 : 0;
          const bool lineOk = __shfl(flagOk, lid | 7) != 0;
          const bool dataOk = !act || (v.x == tearHash(r, line, 4 * j) && v.y == tearHash(r, line, 4 * j + 1) &&
                                       (j == 7 || (v.z == tearHash(r, line, 4 * j + 2) &&
                                                   v.w == tearHash(r, line, 4 * j + 3))));
          const unsigned long long okMask = __ballot(dataOk ? 1 : 0);
          const bool lineData = ((okMask >> (lid & ~7)) & 0xFFull) == 0xFFull;
          // a current flag with stale payload in any of the line's 8 lanes is a torn line
          if (lineOk && !lineData && act && !tornSeen) {
            tornSeen = true;
            if (j == 0) torn++;
          }
          const bool done = lineOk && lineData;
          if (__all(done)) break;
          if (__any(nowTicks() - t0 > maxTicks)) { atomicOr(&sFail, 1); break; }
          if (!done && act) v = ldLine16<SC>(rs, loff);
        }
        if (act && j == 0) checked++;
        if (*(volatile int*)&sFail) break;
      }
      drainVmem();
      __syncthreads();
      if (sFail) break;
      if (threadIdx.x == 0) stAgent(ack, (uint64_t)r + 1);
    }
  }
  atomicAdd(&counts[0], torn);
  atomicAdd(&counts[1], checked);
  if (threadIdx.x == 0 && sFail) atomicOr(failed, 1u);
}

// ------------------------------------------------------------------ allocation-free AllReduce
// The scratch of vcclAllReduceNoAlloc (layout in vccl_dev.h).  Each device the
// library runs on holds its own copy until the process ends.
static __device__ __align__(256) char scratch[NA_SCRATCH_BYTES];

// Before each allocation-free launch, on the same stream: writes the DevComm
// the collective runs with, and zeroes [NA_OFF_WORDS, NA_OFF_CTR + ctrBytes)
// (abort and error words, claim counters, the counters the launch uses) and
// the first llBytes of the LL FIFOs.  The host checks ctrBytes <= NA_CTR_BYTES
// and llBytes <= the LL region.
__global__ void __launch_bounds__(256) noAllocPrepKernel(char* base, const DevComm comm, uint64_t ctrBytes,
                                                           uint64_t llBytes) {
  const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t nthr = (uint64_t)gridDim.x * blockDim.x;
  const u32x4 zero = {0, 0, 0, 0};
  u32x4* r1 = (u32x4*)(base + NA_OFF_WORDS);
  const uint64_t n1 = (NA_OFF_CTR - NA_OFF_WORDS + ctrBytes) / 16;
  for (uint64_t i = tid; i < n1; i += nthr) r1[i] = zero;
  u32x4* r2 = (u32x4*)(base + NA_OFF_FIFO_LL);
  const uint64_t n2 = llBytes / 16;
  for (uint64_t i = tid; i < n2; i += nthr) r2[i] = zero;
  if (blockIdx.x == 0 && threadIdx.x < sizeof(DevComm) / 8)
    ((uint64_t*)(base + NA_OFF_COMM))[threadIdx.x] = ((const uint64_t*)&comm)[threadIdx.x];
}

}  // namespace vccl

// ------------------------------------------------------------------ host-side launchers
// (called by the host runtime; plain C++ linkage inside the library)

hipError_t vcclLaunchColl(const vccl::LaunchDesc& d, int grid, int block, hipStream_t stream, bool cooperative) {
  void* args[] = {(void*)&d};
  if (cooperative)
    return hipLaunchCooperativeKernel((const void*)vccl::collKernel, dim3(grid), dim3(block), args, 0, stream);
  return hipLaunchKernel((const void*)vccl::collKernel, dim3(grid), dim3(block), args, 0, stream);
}

hipError_t vcclCollOccupancy(int block, int* blocksPerCU) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocksPerCU, (const void*)vccl::collKernel, block, 0);
}

hipError_t vcclLaunchServe(const vccl::ServeDesc& d, int grid, int block, hipStream_t stream) {
  void* args[] = {(void*)&d};
  return hipLaunchKernel((const void*)vccl::serveKernel, dim3(grid), dim3(block), args, 0, stream);
}

hipError_t vcclServeOccupancy(int block, int* blocksPerCU) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocksPerCU, (const void*)vccl::serveKernel, block, 0);
}

// Device address of the allocation-free scratch on `device` (the current
// device): looked up once per device with that device current and kept; the
// array's name in host code is only a stand-in for the symbol, never an
// address to hand to a kernel or a copy.
hipError_t vcclScratchPtr(int device, char** ptr) {
  static char* ptrs[64] = {};
  if (device < 0 || device >= 64) return hipErrorInvalidDevice;
  if (!ptrs[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(vccl::scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    ptrs[device] = (char*)p;
  }
  *ptr = ptrs[device];
  return hipSuccess;
}

hipError_t vcclLaunchNoAllocPrep(char* base, const vccl::DevComm& comm, uint64_t ctrBytes, uint64_t llBytes,
                                 hipStream_t stream) {
  if (ctrBytes > vccl::NA_CTR_BYTES || llBytes > vccl::NA_CONNS * vccl::NSLOTS * vccl::NA_SLOT_LL || ctrBytes % 16 ||
      llBytes % 16)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(vccl::noAllocPrepKernel, dim3(64), dim3(256), 0, stream, base, comm, ctrBytes, llBytes);
  return hipGetLastError();
}

hipError_t vcclLaunchXccProbe(int* dIds, int n, hipStream_t stream) {
  hipLaunchKernelGGL(vccl::xccProbeKernel, dim3(n), dim3(64), 0, stream, dIds, n);
  return hipGetLastError();
}

hipError_t vcclLaunchTearProbe(char* bufs, uint64_t* acks, int pairs, int lines, int rounds, unsigned long long* counts,
                               uint64_t maxTicks, uint32_t* failed, int scope, hipStream_t stream) {
  void* args[] = {&bufs, &acks, &pairs, &lines, &rounds, &counts, &maxTicks, &failed};
  const void* k = scope == vccl::SCOPE_XCD ? (const void*)vccl::tearProbeKernel<vccl::SCOPE_XCD>
                                           : (const void*)vccl::tearProbeKernel<vccl::SCOPE_DEVICE>;
  return hipLaunchCooperativeKernel(k, dim3(2 * pairs), dim3(256), args, 0, stream);
}
