// Serving: continuous batching over a persistent kernel.
#include "host_internal.h"

extern "C" {
vcclResult_t vcclServeCreate(vcclComm_t*, size_t, int, vcclServer_t*) { return vcclInvalidUsage; }
vcclResult_t vcclServeSubmit(vcclServer_t, const vcclRequest_t*, uint64_t*) { return vcclInvalidUsage; }
vcclResult_t vcclServeTest(vcclServer_t, uint64_t, int*, vcclResult_t*, uint64_t*) { return vcclInvalidUsage; }
vcclResult_t vcclServeDestroy(vcclServer_t) { return vcclInvalidUsage; }
}
