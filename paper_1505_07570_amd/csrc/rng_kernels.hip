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

// The sample is the set of images of 0..s-1 under the (cycle-walked)
// Feistel map of [0, domain), in increasing order.  The images are computed
// one per thread across the device (sample_gen_kernel, into out), then one
// workgroup sorts them in place.
template <typename OUT>
__global__ __launch_bounds__(256) void sample_gen_kernel(uint64_t domain, int k, int s,
                                                         uint32_t tag, uint64_t seed,
                                                         OUT* __restrict__ out) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t < s) out[t] = (OUT)permute_domain((uint64_t)t, domain, k, tag, seed);
}

// Bitonic sort in LDS (any domain below 2^32).
template <typename OUT>
__global__ __launch_bounds__(kSortThreads) void sample_kernel(uint64_t domain, int k, int s,
                                                              int p2, uint32_t tag,
                                                              uint64_t seed, OUT* __restrict__ out) {
  __shared__ uint32_t v[kMaxSample];
  const int tid = threadIdx.x;
  for (int t = tid; t < p2; t += kSortThreads) v[t] = t < s ? (uint32_t)out[t] : 0xFFFFFFFFu;
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

// Domains up to kBitmapDomain: the same images marked in an LDS bitmap of
// the domain, then read out in increasing order (a counting sort).  Thread t
// owns a run of consecutive bitmap words; an exclusive scan of the per-thread
// bit counts gives each thread its first output position.  Word w is stored
// at w + w / 32, so the 64 lanes of a wave walking their runs in step hit
// distinct banks.
constexpr uint64_t kBitmapDomain = 1ull << 20;
__device__ __forceinline__ int bm_slot(int w) { return w + (w >> 5); }
inline size_t bm_lds_words(uint64_t domain) {
  const size_t nw = (size_t)((domain + 31) / 32);
  return nw + nw / 32 + 1;
}

template <typename OUT>
__global__ __launch_bounds__(kSortThreads) void sample_bitmap_kernel(uint64_t domain, int k, int s,
                                                                     uint32_t tag, uint64_t seed,
                                                                     OUT* __restrict__ out) {
  extern __shared__ uint32_t bits[];
  __shared__ uint32_t wave_tot[kSortThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nw = (int)((domain + 31) / 32);
  const int per = (nw + kSortThreads - 1) / kSortThreads;
  for (int w = tid; w < bm_slot(nw); w += kSortThreads) bits[w] = 0u;
  __syncthreads();
  for (int t = tid; t < s; t += kSortThreads) {
    const uint32_t v = (uint32_t)out[t];
    atomicOr(bits + bm_slot((int)(v >> 5)), 1u << (v & 31u));
  }
  __syncthreads();
  // this thread's run of words, in registers (per <= 32)
  const int w0 = tid * per;
  uint32_t word[32];
  uint32_t cnt = 0;
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    word[i] = (i < per && w0 + i < nw) ? bits[bm_slot(w0 + i)] : 0u;
    cnt += __popc(word[i]);
  }
  // inclusive scan within the wave, then across the waves
  uint32_t inc = cnt;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t o = __shfl_up(inc, off);
    if (lane >= off) inc += o;
  }
  if (lane == 63) wave_tot[wave] = inc;
  __syncthreads();
  uint32_t base = 0;
  for (int i = 0; i < wave; ++i) base += wave_tot[i];
  uint32_t pos = base + inc - cnt;
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    uint32_t wd = word[i];
    while (wd) {
      const int b = __builtin_ctz(wd);
      out[pos++] = (OUT)(32u * (uint32_t)(w0 + i) + (uint32_t)b);
      wd &= wd - 1u;
    }
  }
}

template <typename OUT>
int launch_sample(const rmm_ctx* h, uint64_t domain, int k, int64_t s, uint32_t tag,
                  uint64_t seed, OUT* out) {
  if (s < 1 || s > kMaxSample || (uint64_t)s > domain || domain > 0xFFFFFFFFull)
    return RMM_ERR_INVALID_ARG;
  hipLaunchKernelGGL(sample_gen_kernel<OUT>, dim3((unsigned)((s + 255) / 256)), dim3(256), 0,
                     h->stream, domain, k, (int)s, tag, seed, out);
  RMM_TRY(launch_status());
  if (domain <= kBitmapDomain) {
    const size_t lds = bm_lds_words(domain) * sizeof(uint32_t);
    RMM_HIP(hipFuncSetAttribute((const void*)sample_bitmap_kernel<OUT>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(sample_bitmap_kernel<OUT>, dim3(1), dim3(kSortThreads), lds, h->stream,
                       domain, k, (int)s, tag, seed, out);
    return launch_status();
  }
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
