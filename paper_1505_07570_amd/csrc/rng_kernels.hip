// Kernels that materialize the random quantities of the sketches:
// sorted sample indices (SRHT row sampling, Sec. 3.2.2; uniform column
// selection, Sec. 6.4), CountSketch buckets / signs (Alg. 3.1), SRHT signs
// and Gaussian matrices (Sec. 3.2.1).  The sketch kernels generate these in
// registers; the materializing kernels serve the workspace-held index list
// and the test hooks of the C ABI.
#include "common.hpp"
#include "rng.hpp"

namespace rmm {

constexpr int kSortThreads = 1024;
constexpr int kMaxSample = 8192;

// One workgroup: images of 0..s-1 under the (cycle-walked) Feistel map of
// [0, domain), then a bitonic sort in LDS.
template <typename OUT>
__global__ __launch_bounds__(kSortThreads) void sample_kernel(uint64_t domain, int k, int s,
                                                              int p2, uint32_t tag,
                                                              uint64_t seed, OUT* __restrict__ out) {
  __shared__ uint32_t v[kMaxSample];
  const int tid = threadIdx.x;
  for (int t = tid; t < p2; t += kSortThreads)
    v[t] = t < s ? (uint32_t)permute_domain((uint64_t)t, domain, k, tag, seed) : 0xFFFFFFFFu;
  for (int size = 2; size <= p2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      for (int i = tid; i < (p2 >> 1); i += kSortThreads) {
        const int lo = 2 * i - (i & (stride - 1));
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;
        const uint32_t a = v[lo], b = v[hi];
        if ((a > b) == up) {
          v[lo] = b;
          v[hi] = a;
        }
      }
    }
  }
  __syncthreads();
  for (int t = tid; t < s; t += kSortThreads) out[t] = (OUT)v[t];
}

template <typename OUT>
int launch_sample(const rmm_ctx* h, uint64_t domain, int k, int64_t s, uint32_t tag,
                  uint64_t seed, OUT* out) {
  if (s < 1 || s > kMaxSample || (uint64_t)s > domain || domain > 0xFFFFFFFFull)
    return RMM_ERR_INVALID_ARG;
  int p2 = 1;
  while (p2 < s) p2 <<= 1;
  hipLaunchKernelGGL(sample_kernel<OUT>, dim3(1), dim3(kSortThreads), 0, h->stream, domain, k,
                     (int)s, p2, tag, seed, out);
  return launch_status();
}

int launch_sample_indices_u32(const rmm_ctx* h, uint64_t domain, int k, int64_t s,
                              uint32_t tag, uint64_t seed, uint32_t* out) {
  return launch_sample<uint32_t>(h, domain, k, s, tag, seed, out);
}

int launch_sample_indices_i64(const rmm_ctx* h, uint64_t domain, int k, int64_t s,
                              uint32_t tag, uint64_t seed, int64_t* out) {
  return launch_sample<int64_t>(h, domain, k, s, tag, seed, out);
}

__global__ void cs_hash_kernel(int64_t m, uint32_t s, uint64_t seed, int32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) out[i] = (int32_t)cs_bucket(cs_word((uint64_t)i, seed), s);
}

__global__ void sign_kernel(int64_t m, int kind, uint64_t seed, int8_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const uint32_t bit = kind == RMM_COUNTSKETCH ? (cs_word((uint64_t)i, seed) & 1u)
                                               : srht_sign_bit((uint64_t)i, seed);
  out[i] = bit ? -1 : 1;
}

template <typename T>
__global__ void gaussian_kernel(int64_t rows, int64_t cols, uint32_t tag, uint64_t seed,
                                T* __restrict__ out, int64_t ld) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t q = blockIdx.y;
  if (i >= rows) return;
  if constexpr (sizeof(T) == 4) {
    float z[4];
    gauss4_f32((uint64_t)i, (uint32_t)q, tag, seed, z);
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (4 * q + t < cols) out[i + (4 * q + t) * ld] = z[t];
  } else {
    double z[2];
    gauss2_f64((uint64_t)i, (uint32_t)q, tag, seed, z);
#pragma unroll
    for (int t = 0; t < 2; ++t)
      if (2 * q + t < cols) out[i + (2 * q + t) * ld] = z[t];
  }
}

int launch_cs_hashes(const rmm_ctx* h, int64_t m, int64_t s, uint64_t seed, int32_t* out) {
  if (m == 0) return RMM_OK;
  hipLaunchKernelGGL(cs_hash_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, h->stream,
                     m, (uint32_t)s, seed, out);
  return launch_status();
}

int launch_signs(const rmm_ctx* h, int kind, int64_t m, uint64_t seed, int8_t* out) {
  if (m == 0) return RMM_OK;
  hipLaunchKernelGGL(sign_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, h->stream, m,
                     kind, seed, out);
  return launch_status();
}

template <typename T>
int launch_gaussian(const rmm_ctx* h, uint32_t tag, int64_t rows, int64_t cols, uint64_t seed,
                    T* out, int64_t ld) {
  if (rows == 0 || cols == 0) return RMM_OK;
  const int per = sizeof(T) == 4 ? 4 : 2;
  dim3 grid((unsigned)((rows + 255) / 256), (unsigned)((cols + per - 1) / per));
  hipLaunchKernelGGL(gaussian_kernel<T>, grid, dim3(256), 0, h->stream, rows, cols, tag, seed,
                     out, ld);
  return launch_status();
}

template int launch_gaussian<float>(const rmm_ctx*, uint32_t, int64_t, int64_t, uint64_t, float*,
                                    int64_t);
template int launch_gaussian<double>(const rmm_ctx*, uint32_t, int64_t, int64_t, uint64_t,
                                     double*, int64_t);

}  // namespace rmm
