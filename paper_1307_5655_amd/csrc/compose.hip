// Composition p(q(x)) over Z/(2^31 - 1) through the evaluation tree of p.
#include <hip/hip_runtime.h>

#include "fpe_internal.h"

namespace fpe {

size_t compose_workspace_bytes(const fpe_tree*, int32_t) { return 0; }

fpe_status launch_compose(const fpe_tree*, const uint32_t*, int32_t, uint32_t*, void*, size_t, void*) {
  return fail(FPE_EUNSUPPORTED, "composition is not built yet");
}

}  // namespace fpe
