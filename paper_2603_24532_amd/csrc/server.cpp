// Continuous-batching server (see include/mbpt_vegas.h).
#include <hip/hip_runtime.h>

#include "mbpt_vegas.h"
#include "runtime.hpp"

extern "C" int mbpt_server_workspace_query(const mbpt_context *, int, uint64_t, size_t *) {
  return MBPT_ESTATE;
}
extern "C" int mbpt_server_create(mbpt_context *ctx, int, uint64_t, int, void *, size_t,
                                  mbpt_server **) {
  mbpt::set_err(ctx, "server not available in this build");
  return MBPT_ESTATE;
}
extern "C" void mbpt_server_destroy(mbpt_server *) {}
extern "C" int mbpt_server_submit(mbpt_server *, const mbpt_request *, uint64_t *) {
  return MBPT_ESTATE;
}
extern "C" int mbpt_server_step(mbpt_server *, int *, int *) { return MBPT_ESTATE; }
extern "C" int mbpt_server_poll(mbpt_server *, uint64_t, mbpt_result *, int *, double *, double *,
                                double *) {
  return MBPT_ESTATE;
}
