// Sketch-and-solve least squares without a caller workspace.
//
// rmm_sketched_lsr_noalloc runs exactly the kernels of rmm_sketched_lsr, with
// their scratch (the sketch, its FP64 copy, the CholeskyQR2 factors and the
// sketch kernels' partial slots) carved from `scratch`, a file-scope device
// array of RMM_NOALLOC_SCRATCH_BYTES that every device the library runs on
// holds until the process ends.  The array's name is a host-side stand-in in
// host code: its device address is looked up once per device (with that
// device current) by rmm_create and kept in `g_scratch`, and only that
// address is handed to kernels.  No kernel of the path needs zeroed scratch.
#include <mutex>

#include "common.hpp"

static __device__ __align__(256) char scratch[RMM_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::once_flag g_once[kMaxDevices];
void* g_scratch[kMaxDevices] = {};
hipError_t g_err[kMaxDevices] = {};

}  // namespace

namespace rmm {

// Device address of `scratch` on `device` (looked up on the first call for
// that device, with the device current); null when the lookup failed.
void* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::call_once(g_once[device], [device] {
    int prev = 0;
    hipError_t e = hipGetDevice(&prev);
    if (e == hipSuccess) e = hipSetDevice(device);
    void* p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_err[device] = e;
    g_scratch[device] = e == hipSuccess ? p : nullptr;
    (void)hipSetDevice(prev);
  });
  return g_scratch[device];
}

}  // namespace rmm

using namespace rmm;

extern "C" {

int rmm_sketched_lsr_noalloc(rmm_handle h, rmm_dtype dt, rmm_sketch_kind kind, int64_t m,
                             int64_t d, const void* A, int64_t lda, const void* b, int64_t s,
                             uint64_t seed, double* x, double* resid, int32_t* status) {
  if (!h) return RMM_ERR_INVALID_ARG;
  size_t need = 0;
  RMM_TRY(rmm_lsr_workspace(h, dt, kind, m, d, s, &need));
  if (need > (size_t)RMM_NOALLOC_SCRATCH_BYTES) return RMM_ERR_SCRATCH_LIMIT;
  void* p = noalloc_scratch(h->device);
  if (!p) return RMM_ERR_HIP;
  char* ws = h->ws;
  const size_t wb = h->ws_bytes;
  h->ws = static_cast<char*>(p);
  h->ws_bytes = (size_t)RMM_NOALLOC_SCRATCH_BYTES;
  const int rc = rmm_sketched_lsr(h, dt, kind, m, d, A, lda, b, s, seed, x, resid, status);
  h->ws = ws;
  h->ws_bytes = wb;
  return rc;
}

}  // extern "C"
