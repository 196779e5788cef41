// Entry points whose device code is not in this build yet: they fail loudly.
#include "rlu_device.h"
#include "rlu_internal.h"

namespace rlu {

void serve_shutdown(rlu_ctx_impl &) {}

}  // namespace rlu

extern "C" {
rlu_status rlu_serve_start(rlu_ctx *, size_t, int) { return rlu::fail(RLU_ERR_INVALID_ARG, "serving is not available in this build"); }
rlu_status rlu_submit(rlu_ctx *, const rlu_matrix *, const rlu_params *, const rlu_factors *, uint64_t *) {
  return rlu::fail(RLU_ERR_INVALID_ARG, "serving is not available in this build");
}
rlu_status rlu_poll(rlu_ctx *, uint64_t) { return rlu::fail(RLU_ERR_UNKNOWN_TICKET, "serving is not available in this build"); }
rlu_status rlu_serve_stop(rlu_ctx *) { return RLU_OK; }
}
