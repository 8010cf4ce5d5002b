// Serving loop (continuous batching).
#include <hip/hip_runtime.h>

#include "fpe_internal.h"

using namespace fpe;

extern "C" {
fpe_status fpe_server_create(size_t, int32_t, void*, fpe_server** out) {
  if (out) *out = nullptr;
  return fail(FPE_EUNSUPPORTED, "server is not built yet");
}
fpe_status fpe_server_submit(fpe_server*, const fpe_request*, uint64_t*) { return fail(FPE_EINVAL, "no server"); }
fpe_status fpe_server_poll(fpe_server*, uint64_t, int32_t*) { return fail(FPE_EINVAL, "no server"); }
fpe_status fpe_server_wait(fpe_server*, uint64_t) { return fail(FPE_EINVAL, "no server"); }
fpe_status fpe_server_drain(fpe_server*) { return fail(FPE_EINVAL, "no server"); }
fpe_status fpe_server_stats(fpe_server*, fpe_stats*) { return fail(FPE_EINVAL, "no server"); }
void fpe_server_destroy(fpe_server*) {}
}
