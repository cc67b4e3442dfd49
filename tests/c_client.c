/* A plain C program (no C++, no Python) using the library through its C ABI
 * (include/vccl.h) and the HIP runtime's C API: R virtual ranks on the
 * current device.
 *
 *   c_client [R [n [keep | rings]]]
 *
 * With "keep" the program exits without destroying its communicators or
 * freeing its buffers, leaving the set's device memory, pinned host words
 * and events to process exit.  With "rings" the set is created with two
 * ring orders (the reversed ring and a rotation of it by two), read back
 * with vcclCommGetRings; every check below then runs on them.
 *
 * Checks, on int32 data whose results are exact in any summation order:
 *   - AllReduce sum: recv_r[i] = sum over ranks q of x_q[i];
 *   - AllGather and ReduceScatter issued together in one group;
 *   - Broadcast from rank 1;
 *   - the allocation-free AllReduce (no communicator; int32 max) on the same
 *     buffers, twice, the second call smaller.
 * Then times an 8-byte AllReduce issued from C (R calls, then a stream
 * synchronisation) to show the per-call host cost without an interpreter.
 * Prints one JSON line; exits 0 only when every check passed. */
#define _POSIX_C_SOURCE 199309L /* clock_gettime */

#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#include "vccl.h"

#define MAXR VCCL_MAX_RANKS

static int failures = 0;

#define HIP_OK(x)                                                              \
  do {                                                                         \
    hipError_t e_ = (x);                                                       \
    if (e_ != hipSuccess) {                                                    \
      fprintf(stderr, "%s:%d %s: %s\n", __FILE__, __LINE__, #x,                \
              hipGetErrorString(e_));                                          \
      exit(2);                                                                 \
    }                                                                          \
  } while (0)

#define V_OK(x)                                                                \
  do {                                                                         \
    vcclResult_t r_ = (x);                                                     \
    if (r_ != vcclSuccess) {                                                   \
      fprintf(stderr, "%s:%d %s: %s\n", __FILE__, __LINE__, #x,                \
              vcclGetErrorString(r_));                                         \
      exit(3);                                                                 \
    }                                                                          \
  } while (0)

/* rank q's value at index i: small, so sums over 16 ranks stay far from
 * int32 overflow */
static int32_t value(int q, size_t i) { return (int32_t)((i * 7919u + (size_t)q * 104729u) % 2001u) - 1000; }

static double nowUs(void) {
  struct timespec t;
  clock_gettime(CLOCK_MONOTONIC, &t);
  return (double)t.tv_sec * 1e6 + (double)t.tv_nsec / 1e3;
}

static int cmpDouble(const void* a, const void* b) {
  const double x = *(const double*)a, y = *(const double*)b;
  return (x > y) - (x < y);
}

static void expectEqual(const char* what, const int32_t* got, const int32_t* want, size_t n) {
  for (size_t i = 0; i < n; ++i) {
    if (got[i] != want[i]) {
      fprintf(stderr, "%s: element %zu is %d, expected %d\n", what, i, got[i], want[i]);
      ++failures;
      return;
    }
  }
}

int main(int argc, char** argv) {
  const int R = argc > 1 ? atoi(argv[1]) : 4;
  const size_t n = argc > 2 ? (size_t)strtoull(argv[2], NULL, 10) : 100003;
  const int keep = argc > 3 && strcmp(argv[3], "keep") == 0;
  const int useRings = argc > 3 && strcmp(argv[3], "rings") == 0;
  if (R < 2 || R > MAXR || n == 0) {
    fprintf(stderr, "usage: c_client [R in 2..%d [n > 0]]\n", MAXR);
    return 1;
  }
  vcclComm_t comms[MAXR];
  if (useRings) {
    int rings[2 * MAXR], back[2 * MAXR], nr = 0;
    for (int q = 0; q < R; ++q) {
      rings[q] = R - 1 - q;                   /* reversed */
      rings[R + q] = (R - 1 - q + 2) % R;     /* the reversed ring rotated by two */
    }
    V_OK(vcclCommInitAllRings(comms, R, NULL, 2, rings));
    V_OK(vcclCommGetRings(comms[R - 1], &nr, NULL));
    V_OK(vcclCommGetRings(comms[R - 1], &nr, back));
    if (nr != 2 || memcmp(rings, back, (size_t)(2 * R) * sizeof(int)) != 0) {
      fprintf(stderr, "vcclCommGetRings does not return the rings given\n");
      ++failures;
    }
  } else {
    V_OK(vcclCommInitAll(comms, R, NULL));
  }
  hipStream_t st;
  HIP_OK(hipStreamCreate(&st));

  /* every buffer holds R * n elements: enough for the AllGather output and
   * the ReduceScatter input */
  const size_t big = (size_t)R * n;
  int32_t* host = (int32_t*)malloc(big * sizeof(int32_t));
  int32_t* want = (int32_t*)malloc(big * sizeof(int32_t));
  int32_t* send[MAXR];
  int32_t* recv[MAXR];
  for (int q = 0; q < R; ++q) {
    HIP_OK(hipMalloc((void**)&send[q], big * sizeof(int32_t)));
    HIP_OK(hipMalloc((void**)&recv[q], big * sizeof(int32_t)));
    for (size_t i = 0; i < big; ++i) host[i] = value(q, i);
    HIP_OK(hipMemcpy(send[q], host, big * sizeof(int32_t), hipMemcpyHostToDevice));
  }

  /* AllReduce over the first n elements */
  for (int q = 0; q < R; ++q) V_OK(vcclAllReduce(send[q], recv[q], n, vcclInt32, vcclSum, comms[q], st));
  HIP_OK(hipStreamSynchronize(st));
  for (size_t i = 0; i < n; ++i) {
    int64_t s = 0;
    for (int q = 0; q < R; ++q) s += value(q, i);
    want[i] = (int32_t)s;
  }
  for (int q = 0; q < R; ++q) {
    HIP_OK(hipMemcpy(host, recv[q], n * sizeof(int32_t), hipMemcpyDeviceToHost));
    expectEqual("allreduce", host, want, n);
  }

  /* AllGather and ReduceScatter in one group, on disjoint outputs:
   * AllGather reads send[q][0, n) and writes recv[q][0, R n);
   * ReduceScatter reads send[q][0, R n) and writes rs[q][0, n). */
  int32_t* rs[MAXR];
  for (int q = 0; q < R; ++q) HIP_OK(hipMalloc((void**)&rs[q], n * sizeof(int32_t)));
  V_OK(vcclGroupStart());
  for (int q = 0; q < R; ++q) {
    V_OK(vcclAllGather(send[q], recv[q], n, vcclInt32, comms[q], st));
    V_OK(vcclReduceScatter(send[q], rs[q], n, vcclInt32, vcclSum, comms[q], st));
  }
  V_OK(vcclGroupEnd());
  HIP_OK(hipStreamSynchronize(st));
  for (int p = 0; p < R; ++p)
    for (size_t i = 0; i < n; ++i) want[(size_t)p * n + i] = value(p, i);
  for (int q = 0; q < R; ++q) {
    HIP_OK(hipMemcpy(host, recv[q], big * sizeof(int32_t), hipMemcpyDeviceToHost));
    expectEqual("allgather", host, want, big);
  }
  for (int q = 0; q < R; ++q) {
    for (size_t i = 0; i < n; ++i) {
      int64_t s = 0;
      for (int p = 0; p < R; ++p) s += value(p, (size_t)q * n + i);
      want[i] = (int32_t)s;
    }
    HIP_OK(hipMemcpy(host, rs[q], n * sizeof(int32_t), hipMemcpyDeviceToHost));
    expectEqual("reducescatter", host, want, n);
  }

  /* Broadcast from rank 1 */
  for (int q = 0; q < R; ++q) V_OK(vcclBroadcast(send[q], recv[q], n, vcclInt32, 1, comms[q], st));
  HIP_OK(hipStreamSynchronize(st));
  for (size_t i = 0; i < n; ++i) want[i] = value(1, i);
  for (int q = 0; q < R; ++q) {
    HIP_OK(hipMemcpy(host, recv[q], n * sizeof(int32_t), hipMemcpyDeviceToHost));
    expectEqual("broadcast", host, want, n);
  }

  /* the allocation-free AllReduce: rank arrays of the same buffers */
  {
    const void* sb[MAXR];
    void* rb[MAXR];
    for (int q = 0; q < R; ++q) {
      sb[q] = send[q];
      rb[q] = recv[q];
    }
    const size_t counts[2] = {n, n / 3 + 1};
    for (int k = 0; k < 2; ++k) {
      vcclPlanInfo_t plan;
      V_OK(vcclAllReduceNoAlloc(sb, rb, R, counts[k], vcclInt32, vcclMax, (void*)st, &plan));
      HIP_OK(hipStreamSynchronize(st));
      for (size_t i = 0; i < counts[k]; ++i) {
        int32_t m = value(0, i);
        for (int q = 1; q < R; ++q)
          if (value(q, i) > m) m = value(q, i);
        want[i] = m;
      }
      for (int q = 0; q < R; ++q) {
        HIP_OK(hipMemcpy(host, recv[q], counts[k] * sizeof(int32_t), hipMemcpyDeviceToHost));
        expectEqual(k ? "allreduce without allocation, second call" : "allreduce without allocation", host, want,
                    counts[k]);
      }
    }
  }

  vcclResult_t async = vcclSuccess;
  V_OK(vcclCommGetAsyncError(comms[0], &async));
  if (async != vcclSuccess) {
    fprintf(stderr, "asynchronous error: %s\n", vcclGetErrorString(async));
    ++failures;
  }

  /* per-call cost of an 8-byte AllReduce issued from C */
  enum { REPS = 200 };
  static double rt[REPS], issue[REPS];
  for (int k = 0; k < 20; ++k) {
    for (int q = 0; q < R; ++q) V_OK(vcclAllReduce(send[q], recv[q], 2, vcclInt32, vcclSum, comms[q], st));
    HIP_OK(hipStreamSynchronize(st));
  }
  for (int k = 0; k < REPS; ++k) {
    const double t0 = nowUs();
    for (int q = 0; q < R; ++q) V_OK(vcclAllReduce(send[q], recv[q], 2, vcclInt32, vcclSum, comms[q], st));
    const double t1 = nowUs();
    HIP_OK(hipStreamSynchronize(st));
    rt[k] = nowUs() - t0;
    issue[k] = t1 - t0;
  }
  qsort(rt, REPS, sizeof(double), cmpDouble);
  qsort(issue, REPS, sizeof(double), cmpDouble);

  printf("{\"ok\": %d, \"nranks\": %d, \"count\": %zu, \"allreduce_8B_roundtrip_us_p50\": %.1f, "
         "\"allreduce_8B_issue_us_p50\": %.1f}\n",
         failures == 0, R, n, rt[REPS / 2], issue[REPS / 2]);

  fflush(stdout);
  if (keep) return failures == 0 ? 0 : 4;
  for (int q = 0; q < R; ++q) {
    HIP_OK(hipFree(send[q]));
    HIP_OK(hipFree(recv[q]));
    HIP_OK(hipFree(rs[q]));
  }
  for (int q = 0; q < R; ++q) V_OK(vcclCommDestroy(comms[q]));
  HIP_OK(hipStreamDestroy(st));
  free(host);
  free(want);
  return failures == 0 ? 0 : 4;
}
