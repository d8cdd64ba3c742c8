// Entry points whose kernels are not built yet: they fail with UNSUPPORTED.
#include "common.h"

using namespace spmv;

extern "C" {

spmv_status_t spmv_spmm(spmv_mat_t, const void*, int64_t, void*, int64_t, int32_t, spmv_stream_t) {
  return fail(SPMV_ERR_UNSUPPORTED, "spmm not built");
}
spmv_status_t spmv_batch_create(const spmv_mat_t*, int32_t, spmv_batch_t*) {
  return fail(SPMV_ERR_UNSUPPORTED, "batch not built");
}
spmv_status_t spmv_batch_run(spmv_batch_t, const void* const*, void* const*, spmv_stream_t) {
  return fail(SPMV_ERR_UNSUPPORTED, "batch not built");
}
void spmv_batch_free(spmv_batch_t) {}
spmv_status_t spmv_autotune(spmv_mat_t, spmv_fmt_t, const void*, void*, int64_t, int, spmv_params_t*, double*,
                            spmv_stream_t) {
  return fail(SPMV_ERR_UNSUPPORTED, "autotune not built");
}
}  // extern "C"
