// C ABI: argument validation, workspace carving and dispatch.
#include <math.h>
#include <new>

#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "common.hpp"
#include "ops.hpp"
#include "rng.hpp"

using namespace rmm;

namespace {

bool bad_ld(int64_t ld, int64_t rows) { return ld < (rows > 1 ? rows : 1); }

// the sketch kernels index columns as int and rows as int64
bool sketch_dims_ok(int64_t m, int64_t n, int64_t s) {
  return m >= 0 && n >= 0 && s >= 1 && n < (1ll << 30) && s < (1ll << 30);
}

template <typename T>
size_t sketch_ws(const rmm_ctx* h, rmm_sketch_kind kind, int64_t m, int ncols, int64_t s) {
  switch (kind) {
    case RMM_COUNTSKETCH: return countsketch_workspace<T>(h, m, ncols, s);
    case RMM_SRHT: return srht_workspace<T>(h, m, ncols, s);
    default: return gauss_sketch_workspace<T>(h, m, ncols, s);
  }
}

template <typename T>
int sketch_dispatch(rmm_ctx* h, rmm_sketch_kind kind, int64_t m, int n, const T* A, int64_t lda,
                    const T* b, int64_t s, uint64_t seed, T* C, int64_t ldc, Carver& ws) {
  switch (kind) {
    case RMM_COUNTSKETCH: return countsketch_run<T>(h, m, n, A, lda, b, s, seed, C, ldc, ws);
    case RMM_SRHT: return srht_run<T>(h, m, n, A, lda, b, s, seed, C, ldc, ws);
    case RMM_GAUSSIAN: return gauss_sketch_run<T>(h, m, n, A, lda, b, s, seed, C, ldc, ws);
  }
  return RMM_ERR_INVALID_ARG;
}

bool kind_ok(rmm_sketch_kind k) {
  return k == RMM_GAUSSIAN || k == RMM_SRHT || k == RMM_COUNTSKETCH;
}

}  // namespace

namespace {

int batch_args(rmm_handle h, rmm_dtype dt, rmm_sketch_kind kind, int64_t count,
               const rmm_sketch_desc* d) {
  if (!h || !dt_ok(dt) || !kind_ok(kind) || count < 0 || (count > 0 && !d) || count >= (1 << 24))
    return RMM_ERR_INVALID_ARG;
  for (int64_t i = 0; i < count; ++i) {
    const rmm_sketch_desc& q = d[i];
    if (!sketch_dims_ok(q.m, q.n + 1, q.s)) return RMM_ERR_INVALID_ARG;
    if ((q.n > 0 && q.m > 0 && !q.A) || !q.C || bad_ld(q.lda, q.m) || bad_ld(q.ldc, q.s))
      return RMM_ERR_INVALID_ARG;
    if (kind == RMM_SRHT && q.s > (1ll << ceil_log2((uint64_t)(q.m > 0 ? q.m : 1))))
      return RMM_ERR_INVALID_ARG;
  }
  return RMM_OK;
}

template <typename T>
size_t batch_ws(const rmm_ctx* h, rmm_sketch_kind kind, int count, const rmm_sketch_desc* d) {
  if (kind == RMM_COUNTSKETCH && countsketch_batch_grouped<T>(count, d))
    return countsketch_batch_workspace<T>(h, count, d);
  size_t w = 0;
  for (int i = 0; i < count; ++i) {
    const size_t x = sketch_ws<T>(h, kind, d[i].m, (int)d[i].n + (d[i].b ? 1 : 0), d[i].s);
    if (x > w) w = x;
  }
  return w;
}

template <typename T>
int batch_run(rmm_ctx* h, rmm_sketch_kind kind, int count, const rmm_sketch_desc* d) {
  Carver ws(h->ws, h->ws_bytes);
  if (kind == RMM_COUNTSKETCH && countsketch_batch_grouped<T>(count, d))
    return countsketch_batch_run<T>(h, count, d, ws);
  for (int i = 0; i < count; ++i) {
    Carver w1(h->ws, h->ws_bytes);
    RMM_TRY(sketch_dispatch<T>(h, kind, d[i].m, (int)d[i].n, (const T*)d[i].A, d[i].lda,
                               (const T*)d[i].b, d[i].s, d[i].seed, (T*)d[i].C, d[i].ldc, w1));
  }
  return RMM_OK;
}

}  // namespace

namespace {

template <typename T>
size_t composite_ws(const rmm_ctx* h, rmm_sketch_kind kind2, int64_t m, int ncols, int64_t s1,
                    int64_t s) {
  Carver c(nullptr, 0);
  c.take<T>((size_t)s1 * (ncols > 0 ? ncols : 1));
  const size_t w1 = countsketch_workspace<T>(h, m, ncols, s1);
  const size_t w2 = sketch_ws<T>(h, kind2, s1, ncols, s);
  return c.off + (w1 > w2 ? w1 : w2) + 2 * kAlign;
}

// Sec. 3.2.4: Y = S_cs^T [A | b] (s1 x n') in the workspace, then C = S_2^T Y
template <typename T>
int composite_run(rmm_ctx* h, rmm_sketch_kind kind2, int64_t m, int n, const T* A, int64_t lda,
                  const T* b, int64_t s1, int64_t s, uint64_t seed, T* C, int64_t ldc) {
  const int ncols = n + (b ? 1 : 0);
  Carver ws(h->ws, h->ws_bytes);
  if (ws.cap < composite_ws<T>(h, kind2, m, ncols, s1, s)) return RMM_ERR_WORKSPACE_TOO_SMALL;
  T* Y = ws.take<T>((size_t)s1 * (ncols > 0 ? ncols : 1));
  const size_t mark = ws.off;
  RMM_TRY(countsketch_run<T>(h, m, n, A, lda, b, s1, seed, Y, s1, ws));
  ws.off = mark;
  return sketch_dispatch<T>(h, kind2, s1, ncols, Y, s1, nullptr, s, seed, C, ldc, ws);
}

int composite_args(rmm_handle h, rmm_dtype dt, rmm_sketch_kind kind2, int64_t m, int64_t n_total,
                   int64_t s1, int64_t s) {
  if (!h || !dt_ok(dt) || !kind_ok(kind2) || !sketch_dims_ok(m, n_total, s1) ||
      !sketch_dims_ok(s1, n_total, s))
    return RMM_ERR_INVALID_ARG;
  if (kind2 == RMM_COUNTSKETCH) return RMM_ERR_UNSUPPORTED;
  if (kind2 == RMM_SRHT && s > (1ll << ceil_log2((uint64_t)s1))) return RMM_ERR_INVALID_ARG;
  return RMM_OK;
}

}  // namespace

extern "C" {

int rmm_create(rmm_handle* h, int device) {
  if (!h) return RMM_ERR_INVALID_ARG;
  *h = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
    return RMM_ERR_INVALID_ARG;
  rmm_ctx* c = new (std::nothrow) rmm_ctx();
  if (!c) return RMM_ERR_HIP;
  c->device = device;
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && v > 0)
    c->cus = v;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess &&
      v > 0)
    c->lds_bytes = (size_t)v;
  if (const char* path = getenv("RMM_TUNE_CACHE")) (void)rmm_autotune_load(c, path);
  (void)noalloc_scratch(device);  // rmm_sketched_lsr_noalloc reports a failed lookup
  void* flag = nullptr;
  if (hipHostMalloc(&flag, 64, hipHostMallocDefault) == hipSuccess) c->hflag = static_cast<int*>(flag);
  *h = c;
  return RMM_OK;
}

int rmm_set_autotune(rmm_handle h, int on) {
  if (!h) return RMM_ERR_INVALID_ARG;
  h->autotune = on != 0;
  return RMM_OK;
}

int rmm_set_kernel_timing(rmm_handle h, int on) {
  if (!h) return RMM_ERR_INVALID_ARG;
  if (on) {
    for (hipEvent_t& e : h->kev)
      if (!e) RMM_HIP(hipEventCreate(&e));
  }
  h->ktime = on != 0;
  h->kmarked = false;
  return RMM_OK;
}

int rmm_kernel_time(rmm_handle h, float* ms) {
  if (!h || !ms || !h->ktime || !h->kmarked) return RMM_ERR_INVALID_ARG;
  RMM_HIP(hipEventSynchronize(h->kev[1]));
  RMM_HIP(hipEventElapsedTime(ms, h->kev[0], h->kev[1]));
  return RMM_OK;
}

int rmm_autotune_count(rmm_handle h, int64_t* count) {
  if (!h || !count) return RMM_ERR_INVALID_ARG;
  *count = (int64_t)h->plans.size();
  return RMM_OK;
}

int rmm_autotune_save(rmm_handle h, const char* path) {
  if (!h || !path) return RMM_ERR_INVALID_ARG;
  FILE* f = fopen(path, "w");
  if (!f) return RMM_ERR_INVALID_ARG;
  for (const auto& kv : h->plans) fprintf(f, "%s\t%d\n", kv.first.c_str(), kv.second);
  return fclose(f) == 0 ? RMM_OK : RMM_ERR_INVALID_ARG;
}

int rmm_autotune_load(rmm_handle h, const char* path) {
  if (!h || !path) return RMM_ERR_INVALID_ARG;
  FILE* f = fopen(path, "r");
  if (!f) return RMM_ERR_INVALID_ARG;
  char line[512];
  while (fgets(line, sizeof(line), f)) {
    char* tab = strchr(line, '\t');
    if (!tab) continue;
    *tab = '\0';
    const int plan = atoi(tab + 1);
    if (plan >= 0) h->plans[std::string(line)] = plan;
  }
  fclose(f);
  return RMM_OK;
}

int rmm_destroy(rmm_handle h) {
  delete h;
  return RMM_OK;
}

int rmm_set_stream(rmm_handle h, void* stream) {
  if (!h) return RMM_ERR_INVALID_ARG;
  h->stream = reinterpret_cast<hipStream_t>(stream);
  return RMM_OK;
}

int rmm_set_workspace(rmm_handle h, void* dptr, size_t bytes) {
  if (!h || (bytes > 0 && !dptr) || ((uintptr_t)dptr % kAlign) != 0) return RMM_ERR_INVALID_ARG;
  h->ws = reinterpret_cast<char*>(dptr);
  h->ws_bytes = bytes;
  return RMM_OK;
}

int rmm_device_cus(rmm_handle h, int* cus) {
  if (!h || !cus) return RMM_ERR_INVALID_ARG;
  *cus = h->cus;
  return RMM_OK;
}

const char* rmm_strerror(int code) {
  switch (code) {
    case RMM_OK: return "ok";
    case RMM_ERR_INVALID_ARG: return "invalid argument";
    case RMM_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case RMM_ERR_HIP: return "HIP runtime error";
    case RMM_ERR_UNSUPPORTED: return "unsupported combination";
    case RMM_ERR_SCRATCH_LIMIT: return "problem needs more than the static scratch of the no-alloc entry point";
  }
  return "unknown error";
}

int rmm_sketch_workspace(rmm_handle h, rmm_dtype dt, rmm_sketch_kind kind, int64_t m,
                         int64_t n_total, int64_t s, size_t* bytes) {
  if (!h || !bytes || !dt_ok(dt) || !kind_ok(kind) || !sketch_dims_ok(m, n_total, s))
    return RMM_ERR_INVALID_ARG;
  *bytes = dt == RMM_F32 ? sketch_ws<float>(h, kind, m, (int)n_total, s)
                         : sketch_ws<double>(h, kind, m, (int)n_total, s);
  return RMM_OK;
}

int rmm_sketch(rmm_handle h, rmm_dtype dt, rmm_sketch_kind kind, int64_t m, int64_t n,
               const void* A, int64_t lda, const void* b, int64_t s, uint64_t seed, void* C,
               int64_t ldc) {
  if (!h || !dt_ok(dt) || !kind_ok(kind) || !sketch_dims_ok(m, n + 1, s)) return RMM_ERR_INVALID_ARG;
  if ((n > 0 && m > 0 && !A) || !C || bad_ld(lda, m) || bad_ld(ldc, s)) return RMM_ERR_INVALID_ARG;
  if (kind == RMM_SRHT) {
    const int k = ceil_log2((uint64_t)(m > 0 ? m : 1));
    if (s > (1ll << k)) return RMM_ERR_INVALID_ARG;
  }
  Carver ws(h->ws, h->ws_bytes);
  if (dt == RMM_F32)
    return sketch_dispatch<float>(h, kind, m, (int)n, (const float*)A, lda, (const float*)b, s,
                                  seed, (float*)C, ldc, ws);
  return sketch_dispatch<double>(h, kind, m, (int)n, (const double*)A, lda, (const double*)b, s,
                                 seed, (double*)C, ldc, ws);
}

int rmm_sketch_composite_workspace(rmm_handle h, rmm_dtype dt, rmm_sketch_kind kind2, int64_t m,
                                   int64_t n_total, int64_t s1, int64_t s, size_t* bytes) {
  RMM_TRY(composite_args(h, dt, kind2, m, n_total, s1, s));
  if (!bytes) return RMM_ERR_INVALID_ARG;
  *bytes = dt == RMM_F32 ? composite_ws<float>(h, kind2, m, (int)n_total, s1, s)
                         : composite_ws<double>(h, kind2, m, (int)n_total, s1, s);
  return RMM_OK;
}

int rmm_sketch_composite(rmm_handle h, rmm_dtype dt, rmm_sketch_kind kind2, int64_t m, int64_t n,
                         const void* A, int64_t lda, const void* b, int64_t s1, int64_t s,
                         uint64_t seed, void* C, int64_t ldc) {
  RMM_TRY(composite_args(h, dt, kind2, m, n + 1, s1, s));
  if ((n > 0 && m > 0 && !A) || !C || bad_ld(lda, m) || bad_ld(ldc, s)) return RMM_ERR_INVALID_ARG;
  if (dt == RMM_F32)
    return composite_run<float>(h, kind2, m, (int)n, (const float*)A, lda, (const float*)b, s1, s,
                                seed, (float*)C, ldc);
  return composite_run<double>(h, kind2, m, (int)n, (const double*)A, lda, (const double*)b, s1,
                               s, seed, (double*)C, ldc);
}

int rmm_sketch_batch_workspace(rmm_handle h, rmm_dtype dt, rmm_sketch_kind kind, int64_t count,
                               const rmm_sketch_desc* descs, size_t* bytes) {
  RMM_TRY(batch_args(h, dt, kind, count, descs));
  if (!bytes) return RMM_ERR_INVALID_ARG;
  *bytes = dt == RMM_F32 ? batch_ws<float>(h, kind, (int)count, descs)
                         : batch_ws<double>(h, kind, (int)count, descs);
  return RMM_OK;
}

int rmm_sketch_batch(rmm_handle h, rmm_dtype dt, rmm_sketch_kind kind, int64_t count,
                     const rmm_sketch_desc* descs) {
  RMM_TRY(batch_args(h, dt, kind, count, descs));
  return dt == RMM_F32 ? batch_run<float>(h, kind, (int)count, descs)
                       : batch_run<double>(h, kind, (int)count, descs);
}

int rmm_sketch_hashes(rmm_handle h, int64_t m, int64_t s, uint64_t seed, int32_t* out) {
  if (!h || m < 0 || s < 1 || s >= (1ll << 31) || (m > 0 && !out)) return RMM_ERR_INVALID_ARG;
  return launch_cs_hashes(h, m, s, seed, out);
}

int rmm_sketch_signs(rmm_handle h, rmm_sketch_kind kind, int64_t m, uint64_t seed, int8_t* out) {
  if (!h || m < 0 || (m > 0 && !out) || (kind != RMM_COUNTSKETCH && kind != RMM_SRHT))
    return RMM_ERR_INVALID_ARG;
  return launch_signs(h, (int)kind, m, seed, out);
}

int rmm_srht_indices(rmm_handle h, int64_t m, int64_t s, uint64_t seed, int64_t* out) {
  if (!h || m < 0 || !out) return RMM_ERR_INVALID_ARG;
  const int k = ceil_log2((uint64_t)(m > 0 ? m : 1));
  if (s < 1 || s > (1ll << k)) return RMM_ERR_INVALID_ARG;
  if (s > 8192 || k > 32) return RMM_ERR_UNSUPPORTED;
  return launch_sample_indices_i64(h, 1ull << k, k, s, TAG_SRHT_SAMPLE, seed, out);
}

int rmm_gaussian(rmm_handle h, rmm_dtype dt, int stream, int64_t rows, int64_t cols, uint64_t seed,
                 void* out, int64_t ld) {
  static const uint32_t tags[3] = {TAG_GAUSS_SKETCH, TAG_GAUSS_RSVD, TAG_GAUSS_NYSTROM};
  if (!h || !dt_ok(dt) || stream < 0 || stream > 2 || rows < 0 || cols < 0 ||
      cols >= (1ll << 32) || bad_ld(ld, rows) || (rows * cols > 0 && !out))
    return RMM_ERR_INVALID_ARG;
  if (dt == RMM_F32) return launch_gaussian<float>(h, tags[stream], rows, cols, seed, (float*)out, ld);
  return launch_gaussian<double>(h, tags[stream], rows, cols, seed, (double*)out, ld);
}

}  // extern "C"
