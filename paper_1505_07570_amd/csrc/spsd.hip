// Kernels of the faster SPSD sketching (Alg. 6.1), leverage-score sampling
// (Sec. 3.3.2) and the faster CUR decomposition (Sec. 6.6.3):
//
// * leverage scores q_i = ||Q[i, :]||^2 of an orthonormal basis, one row per
//   thread (coalesced along the rows of the column-major Q);
// * weighted sampling with replacement by the inverse integer CDF: weights
//   w_i = floor(q_i 2^32 + 1/2), their inclusive prefix sums (exact in
//   uint64, so any summation order gives the same CDF), and per draw j the
//   target t_j = floor(r_j W / 2^64) of the 64-bit uniform r_j = (w0, w1) of
//   philox(j, tag, 0), answered by a binary search for the first CDF entry
//   above t_j;
// * the sorted union of two index lists (P = unique([draws; S])) through a
//   bitmap of the domain in LDS, compacted in index order; the output is
//   padded with -1 to its capacity and its length is written to the device;
// * row gathers X[P, :] with zero rows for the padding, and RBF kernel
//   blocks K[A, B] in FP64 with zeros outside the two index lists' lengths
//   (zero rows and columns leave the pseudo-inverse products unchanged);
// * RBF columns in FP64 (the FP32 path is the Nystrom kernel).
#include "common.hpp"
#include "ops.hpp"
#include "rng.hpp"

namespace rmm {

constexpr int kScanThreads = 1024;
constexpr int kUnionThreads = 1024;

__global__ void row_sqnorm_kernel(int64_t n, int k, const double* __restrict__ Q, int64_t ldq,
                                  double* __restrict__ q) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a = 0.0;
  for (int j = 0; j < k; ++j) {
    const double v = Q[i + (int64_t)j * ldq];
    a = fma(v, v, a);
  }
  q[i] = a;
}

// cdf[i] = w_0 + ... + w_i, w_i = floor(q_i 2^32 + 1/2); one workgroup, each
// thread a contiguous segment, segment totals scanned through LDS.
__global__ __launch_bounds__(kScanThreads) void weight_cdf_kernel(int64_t n, const double* __restrict__ q,
                                                                 uint64_t* __restrict__ cdf) {
  __shared__ uint64_t tot[kScanThreads];
  const int t = threadIdx.x;
  const int64_t seg = (n + kScanThreads - 1) / kScanThreads;
  const int64_t i0 = t * seg, i1 = (i0 + seg < n) ? i0 + seg : n;
  uint64_t s = 0;
  for (int64_t i = i0; i < i1; ++i) s += (uint64_t)floor(q[i] * 0x1p32 + 0.5);
  tot[t] = s;
  __syncthreads();
  // inclusive Hillis-Steele scan of the segment totals
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const uint64_t v = t >= off ? tot[t - off] : 0;
    __syncthreads();
    tot[t] += v;
    __syncthreads();
  }
  uint64_t run = t > 0 ? tot[t - 1] : 0;
  for (int64_t i = i0; i < i1; ++i) {
    run += (uint64_t)floor(q[i] * 0x1p32 + 0.5);
    cdf[i] = run;
  }
}

__global__ void weighted_draw_kernel(int64_t n, const uint64_t* __restrict__ cdf, int64_t p,
                                     uint32_t tag, uint64_t seed, int64_t* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= p) return;
  const uint64_t W = cdf[n - 1];
  const Words4 w = philox_at((uint64_t)j, tag, 0, seed);
  const uint64_t r = ((uint64_t)w.w[0] << 32) | (uint64_t)w.w[1];
  const uint64_t target = __umul64hi(r, W);  // < W
  int64_t lo = 0, hi = n - 1;                // first i with cdf[i] > target
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (cdf[mid] > target) hi = mid;
    else lo = mid + 1;
  }
  out[j] = lo;
}

// out = sorted unique(a[0:na] u b[0:nb]) over the domain [0, n), n <= 2^20;
// out[len:cap] = -1, *len_out = len.
__global__ __launch_bounds__(kUnionThreads) void union_sorted_kernel(int64_t n, const int64_t* __restrict__ a,
                                                                     int64_t na, const int64_t* __restrict__ b,
                                                                     int64_t nb, int64_t cap,
                                                                     int64_t* __restrict__ out,
                                                                     int64_t* __restrict__ len_out) {
  extern __shared__ uint32_t bits[];  // ceil(n / 32) words
  __shared__ int64_t pre[kUnionThreads];
  const int t = threadIdx.x;
  const int64_t words = (n + 31) / 32;
  for (int64_t w = t; w < words; w += kUnionThreads) bits[w] = 0u;
  __syncthreads();
  for (int64_t e = t; e < na + nb; e += kUnionThreads) {
    const int64_t v = e < na ? a[e] : b[e - na];
    if (v >= 0 && v < n) atomicOr(&bits[v >> 5], 1u << (v & 31));
  }
  __syncthreads();
  const int64_t seg = (words + kUnionThreads - 1) / kUnionThreads;
  const int64_t w0 = t * seg, w1 = (w0 + seg < words) ? w0 + seg : words;
  int64_t cnt = 0;
  for (int64_t w = w0; w < w1; ++w) cnt += __popc(bits[w]);
  pre[t] = cnt;
  __syncthreads();
  for (int off = 1; off < kUnionThreads; off <<= 1) {
    const int64_t v = t >= off ? pre[t - off] : 0;
    __syncthreads();
    pre[t] += v;
    __syncthreads();
  }
  int64_t pos = t > 0 ? pre[t - 1] : 0;
  for (int64_t w = w0; w < w1; ++w) {
    uint32_t m = bits[w];
    while (m) {
      const int bit = __ffs(m) - 1;
      m &= m - 1;
      if (pos < cap) out[pos] = w * 32 + bit;
      ++pos;
    }
  }
  const int64_t total = pre[kUnionThreads - 1];
  for (int64_t e = total + t; e < cap; e += kUnionThreads) out[e] = -1;
  if (t == 0) *len_out = total;
}

// G[a + j * pm] = X[P[a] + j * ldx] (a < *np), 0 for the padding rows
template <typename T>
__global__ void gather_rows_kernel(int64_t pm, int k, const int64_t* __restrict__ P,
                                   const int64_t* __restrict__ np, const T* __restrict__ X, int64_t ldx,
                                   double* __restrict__ G) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (a >= pm) return;
  const int64_t len = *np;
  G[a + (int64_t)j * pm] = a < len ? (double)X[P[a] + (int64_t)j * ldx] : 0.0;
}

// K[a + b * ma] = exp(-||x_{A_a} - y_{B_b}||^2 g) in FP64 for a < *na, b < *nb, else 0;
// points are rows of X (ld ldx) and Y (ld ldy)
template <typename T>
__global__ void rbf_block_f64_kernel(int d, const T* __restrict__ X, int64_t ldx,
                                     const int64_t* __restrict__ A, const int64_t* __restrict__ na,
                                     int64_t ma, const T* __restrict__ Y, int64_t ldy,
                                     const int64_t* __restrict__ B, const int64_t* __restrict__ nb,
                                     double g, double* __restrict__ K) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t b = blockIdx.y;
  if (a >= ma) return;
  double v = 0.0;
  if (a < *na && b < *nb) {
    const T* xa = X + A[a] * ldx;
    const T* yb = Y + B[b] * ldy;
    double acc = 0.0;
    for (int k = 0; k < d; ++k) {
      const double t = (double)xa[k] - (double)yb[k];
      acc = fma(t, t, acc);
    }
    v = exp(-acc * g);
  }
  K[a + b * ma] = v;
}

// C[i + j * ldc] = exp(-||x_i - y_{idx_j}||^2 g) in FP64 (rows of X, ld ldx;
// rows of Y, ld ldy); grid (rows / 256, columns)
__global__ void rbf_cols_f64_kernel(int64_t n, int d, const double* __restrict__ X, int64_t ldx,
                                    const int64_t* __restrict__ idx, const double* __restrict__ Y,
                                    int64_t ldy, double g, double* __restrict__ C, int64_t ldc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i >= n) return;
  const double* xi = X + i * ldx;
  const double* yj = Y + idx[j] * ldy;
  double acc = 0.0;
  for (int k = 0; k < d; ++k) {
    const double t = xi[k] - yj[k];
    acc = fma(t, t, acc);
  }
  C[i + j * ldc] = exp(-acc * g);
}

int leverage_scores(const rmm_ctx* h, int64_t n, int k, const double* Q, int64_t ldq, double* q) {
  hipLaunchKernelGGL(row_sqnorm_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, h->stream, n,
                     k, Q, ldq, q);
  return launch_status();
}

int weighted_sample(const rmm_ctx* h, int64_t n, const double* q, int64_t p, uint32_t tag,
                    uint64_t seed, uint64_t* cdf, int64_t* out) {
  hipLaunchKernelGGL(weight_cdf_kernel, dim3(1), dim3(kScanThreads), 0, h->stream, n, q, cdf);
  RMM_TRY(launch_status());
  if (p == 0) return RMM_OK;
  hipLaunchKernelGGL(weighted_draw_kernel, dim3((unsigned)((p + 255) / 256)), dim3(256), 0, h->stream,
                     n, cdf, p, tag, seed, out);
  return launch_status();
}

int union_sorted(const rmm_ctx* h, int64_t n, const int64_t* a, int64_t na, const int64_t* b,
                 int64_t nb, int64_t cap, int64_t* out, int64_t* len) {
  if (n > kUnionMaxDomain) return RMM_ERR_UNSUPPORTED;
  const size_t lds = (size_t)((n + 31) / 32) * sizeof(uint32_t);
  RMM_HIP(hipFuncSetAttribute((const void*)union_sorted_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(union_sorted_kernel, dim3(1), dim3(kUnionThreads), lds, h->stream, n, a, na, b, nb,
                     cap, out, len);
  return launch_status();
}

template <typename T>
int gather_rows(const rmm_ctx* h, int64_t pm, int k, const int64_t* P, const int64_t* np, const T* X,
                int64_t ldx, double* G) {
  if (pm == 0 || k == 0) return RMM_OK;
  hipLaunchKernelGGL((gather_rows_kernel<T>), dim3((unsigned)((pm + 255) / 256), (unsigned)k), dim3(256),
                     0, h->stream, pm, k, P, np, X, ldx, G);
  return launch_status();
}

template <typename T>
int rbf_block_f64(const rmm_ctx* h, int d, const T* X, int64_t ldx, const int64_t* A,
                  const int64_t* na, int64_t ma, const T* Y, int64_t ldy, const int64_t* B,
                  const int64_t* nb, int64_t mb, double g, double* K) {
  if (ma == 0 || mb == 0) return RMM_OK;
  hipLaunchKernelGGL((rbf_block_f64_kernel<T>), dim3((unsigned)((ma + 127) / 128), (unsigned)mb), dim3(128),
                     0, h->stream, d, X, ldx, A, na, ma, Y, ldy, B, nb, g, K);
  return launch_status();
}

int rbf_cols_f64(const rmm_ctx* h, int64_t n, int d, const double* X, int64_t ldx, int c,
                 const int64_t* idx, const double* Y, int64_t ldy, double g, double* C, int64_t ldc) {
  if (n == 0 || c == 0) return RMM_OK;
  hipLaunchKernelGGL(rbf_cols_f64_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)c), dim3(256), 0,
                     h->stream, n, d, X, ldx, idx, Y, ldy, g, C, ldc);
  return launch_status();
}

template int gather_rows<float>(const rmm_ctx*, int64_t, int, const int64_t*, const int64_t*,
                                const float*, int64_t, double*);
template int gather_rows<double>(const rmm_ctx*, int64_t, int, const int64_t*, const int64_t*,
                                 const double*, int64_t, double*);
template int rbf_block_f64<float>(const rmm_ctx*, int, const float*, int64_t, const int64_t*,
                                  const int64_t*, int64_t, const float*, int64_t, const int64_t*,
                                  const int64_t*, int64_t, double, double*);
template int rbf_block_f64<double>(const rmm_ctx*, int, const double*, int64_t, const int64_t*,
                                   const int64_t*, int64_t, const double*, int64_t, const int64_t*,
                                   const int64_t*, int64_t, double, double*);

}  // namespace rmm
