// Randomized SVD and least-squares drivers (filled in below).
#include "common.hpp"
#include "ops.hpp"

extern "C" {

int rmm_rsvd_workspace(rmm_handle, rmm_dtype, rmm_precision, int64_t, int64_t, int64_t, int64_t,
                       size_t*) {
  return RMM_ERR_UNSUPPORTED;
}
int rmm_rsvd(rmm_handle, rmm_dtype, rmm_precision, int64_t, int64_t, const void*, int64_t,
             int64_t, int64_t, int64_t, uint64_t, void*, int64_t, void*, void*, int64_t,
             int32_t*) {
  return RMM_ERR_UNSUPPORTED;
}
int rmm_lsr_workspace(rmm_handle, rmm_dtype, rmm_sketch_kind, int64_t, int64_t, int64_t,
                      size_t*) {
  return RMM_ERR_UNSUPPORTED;
}
int rmm_sketched_lsr(rmm_handle, rmm_dtype, rmm_sketch_kind, int64_t, int64_t, const void*,
                     int64_t, const void*, int64_t, uint64_t, double*, double*, int32_t*) {
  return RMM_ERR_UNSUPPORTED;
}
int rmm_plain_lsr_workspace(rmm_handle, rmm_dtype, int64_t, int64_t, size_t*) {
  return RMM_ERR_UNSUPPORTED;
}
int rmm_plain_lsr(rmm_handle, rmm_dtype, int64_t, int64_t, const void*, int64_t, const void*,
                  double*, double*, int32_t*) {
  return RMM_ERR_UNSUPPORTED;
}
}
