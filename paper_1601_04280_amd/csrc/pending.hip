// Entry points whose device code is not in this build yet: they fail loudly.
#include "rlu_device.h"
#include "rlu_internal.h"

namespace rlu {

hipError_t launch_csr_check(const rlu_matrix *, int, rlu_info *, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_sketch_csr(int64_t, int64_t, const int32_t *, const int32_t *, const double *, int, int,
                             const uint32_t *, const int32_t *, const double2 *, const double2 *, double *,
                             int64_t, int32_t *, int, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t contraction_csr(int64_t, int64_t, int, const int32_t *, const int32_t *, const double *,
                           const double *, double *, hipStream_t) {
  return hipErrorNotSupported;
}
struct FactorPlan;
size_t precision_scratch_bytes(int64_t, int64_t, int, int, int) { return 0; }
rlu_status run_precision_contraction(const rlu_ctx_impl &, const FactorPlan &, const rlu_matrix *,
                                     const rlu_params *, void *, hipStream_t) {
  return fail(RLU_ERR_INVALID_ARG, "reduced-precision contraction is not available in this build");
}
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
