// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/rmm.h"

#include <map>
#include <string>
#include <vector>

struct rmm_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  int cus = 256;
  size_t lds_bytes = 65536;  // usable LDS per workgroup
  std::vector<unsigned char> table_host;  // staging of the last batch descriptor table
  bool autotune = false;                  // time the candidate plans of new shapes
  std::map<std::string, int> plans;       // tuned plan per kernel shape key
  // rmm_set_kernel_timing: events around the main kernel of each sketch
  bool ktime = false;
  mutable bool kmarked = false;  // both events recorded since timing was enabled
  hipEvent_t kev[2] = {nullptr, nullptr};
  // pinned host words through which iterative solvers report convergence
  // to the host (null if the allocation failed)
  int* hflag = nullptr;
  ~rmm_ctx() {
    for (hipEvent_t e : kev)
      if (e) (void)hipEventDestroy(e);
    if (hflag) (void)hipHostFree(hflag);
  }
};

namespace rmm {

constexpr size_t kAlign = 256;

// Event k (0 before, 1 after) around a sketch's main kernel when kernel
// timing is on; recorded on the handle's stream.
inline void ktime_mark(const rmm_ctx* h, int k) {
  if (!h->ktime) return;
  (void)hipEventRecord(h->kev[k], h->stream);
  if (k == 1) h->kmarked = true;
}

// Bump allocator over the caller's workspace.  The size queries run the
// same carving sequence with a null base, so a query and the call that
// follows always agree on the layout.
struct Carver {
  char* base;
  size_t off = 0;
  size_t cap;
  Carver(char* b, size_t c) : base(b), cap(c) {}
  template <typename T>
  T* take(size_t count) {
    off = (off + kAlign - 1) / kAlign * kAlign;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
  bool fits() const { return off <= cap; }
};

inline int hip_status(hipError_t e) { return e == hipSuccess ? RMM_OK : RMM_ERR_HIP; }

// Check the launch that was just enqueued.
inline int launch_status() { return hip_status(hipGetLastError()); }

#define RMM_TRY(expr)               \
  do {                              \
    int rmm_rc_ = (expr);           \
    if (rmm_rc_ != RMM_OK) return rmm_rc_; \
  } while (0)

#define RMM_HIP(expr)                           \
  do {                                          \
    if ((expr) != hipSuccess) return RMM_ERR_HIP; \
  } while (0)

// Workgroup barrier that orders LDS accesses only: global stores issued
// before it are not waited for (they are consumed by later kernels).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// 16-byte loads of data a kernel reads once (A in the streaming passes) carry
// the nontemporal hint: the lines do not displace reused data in the caches,
// and on MI355X a plain streaming read of 1 GB goes from 5.9 to 6.7 TB/s
// with it (measured with rmm_stream_read).
typedef float stream_f4_t __attribute__((ext_vector_type(4)));
typedef double stream_d2_t __attribute__((ext_vector_type(2)));
typedef unsigned stream_u4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ld_stream(const float4* p) {
  const stream_f4_t v = __builtin_nontemporal_load(reinterpret_cast<const stream_f4_t*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ double2 ld_stream(const double2* p) {
  const stream_d2_t v = __builtin_nontemporal_load(reinterpret_cast<const stream_d2_t*>(p));
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ uint4 ld_stream(const uint4* p) {
  const stream_u4_t v = __builtin_nontemporal_load(reinterpret_cast<const stream_u4_t*>(p));
  return make_uint4(v.x, v.y, v.z, v.w);
}

// Orders the LDS accesses of one wave (no workgroup barrier).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

inline bool dt_ok(rmm_dtype dt) { return dt == RMM_F32 || dt == RMM_F64; }
inline size_t dt_size(rmm_dtype dt) { return dt == RMM_F64 ? 8 : 4; }

// ---- column-panel streaming plan ---------------------------------------------
//
// The sketch kernels stream A as (column panel, row chunk) work units.  A
// panel is a run of at most `width` consecutive columns; units are ordered
// panel-major and split into G contiguous, equally sized ranges, one per
// workgroup (or per wave).  A worker flushes its accumulators whenever its
// panel changes, so each panel receives partial results from a contiguous
// run of workers; partial slot = worker + panel is unique.
struct PanelPlan {
  int64_t m;        // rows of A
  int64_t nchunks;  // row chunks
  int64_t chunk;    // rows per chunk
  int64_t units;    // P * BT * nchunks
  int ncols;        // columns including the optional b column
  int P;            // column panels
  int width;        // max columns per panel
  int BT;           // bucket tiles (CountSketch only; 1 otherwise)
  int ST;           // buckets per tile
  int s;            // sketch size
  int G;            // workers
  int slot_elems;   // elements per partial slot = width * ST
};

__host__ __device__ __forceinline__ int64_t plan_col0(const PanelPlan& p, int panel) {
  return (int64_t)panel * p.ncols / p.P;
}
__host__ __device__ __forceinline__ int64_t plan_start(const PanelPlan& p, int64_t w) {
  return w * p.units / p.G;
}
// Worker whose range holds unit u.
__host__ __device__ __forceinline__ int64_t plan_worker(const PanelPlan& p, int64_t u) {
  return ((u + 1) * p.G - 1) / p.units;
}

PanelPlan make_plan(int64_t m, int ncols, int width, int s, int ST, int64_t chunk, int G);
inline int64_t plan_slots(const PanelPlan& p) { return (int64_t)p.G + (int64_t)p.P * p.BT; }

// Output column j of the fixed-order reduction: C[r, j] = scale * (sum of
// the slots of the contiguous run of workers that touched (panel, tile) of
// row r, in increasing worker order, in fp64).
template <typename T>
__device__ __forceinline__ void panel_reduce_body(const PanelPlan& plan, const T* __restrict__ partials,
                                                  double scale, T* __restrict__ C, int64_t ldc,
                                                  int64_t j) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= plan.s || j >= plan.ncols) return;
  const int p = (int)(((j + 1) * plan.P - 1) / plan.ncols);
  const int bt = (int)(r / plan.ST);
  const int64_t vp = (int64_t)p * plan.BT + bt;
  const int64_t w = j - plan_col0(plan, p);
  const int64_t rr = r - (int64_t)bt * plan.ST;
  const int64_t lo = plan_worker(plan, vp * plan.nchunks);
  const int64_t hi = plan_worker(plan, (vp + 1) * plan.nchunks - 1);
  double acc = 0.0;
  for (int64_t b = lo; b <= hi; ++b)
    acc += (double)partials[(b + vp) * plan.slot_elems + w * plan.ST + rr];
  C[r + j * ldc] = (T)(acc * scale);
}

// Fixed-order reduction of partial slots into C (scaled), see reduce.hip.
template <typename T>
int launch_panel_reduce(const PanelPlan& plan, const T* partials, double scale, T* C,
                        int64_t ldc, hipStream_t st);

// Zero an s x n column-major block of C.
template <typename T>
int launch_fill_zero(T* C, int64_t rows, int64_t cols, int64_t ldc, hipStream_t st);

}  // namespace rmm
