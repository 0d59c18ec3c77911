// Serving entry points (continuous batching); filled in by the scheduler.
#include <hip/hip_runtime.h>

#include "za.h"

extern "C" {
za_status za_server_create(size_t, int32_t, int32_t, za_server** out) {
  if (out) *out = nullptr;
  return ZA_ERR_UNSUPPORTED;
}
za_status za_server_submit(za_server*, const za_problem*, const double*, int64_t, za_req_id*) {
  return ZA_ERR_UNSUPPORTED;
}
za_status za_server_poll(za_server*, za_req_id, int32_t*, double*, za_req_stats*) { return ZA_ERR_UNSUPPORTED; }
za_status za_server_drain(za_server*) { return ZA_ERR_UNSUPPORTED; }
za_status za_server_destroy(za_server*) { return ZA_ERR_UNSUPPORTED; }
}
