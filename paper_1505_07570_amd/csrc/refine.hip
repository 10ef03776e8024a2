// Machine-precision least squares (Alg. 4.1, Sec. 4.3): the iterations after
// the sketch.  The sketch supplies T = R_Y^{-1} and the start x0 (the
// sketch-and-solve solution); the iterations are conjugate gradients on the
// normal equations of A T, written in x = T z, i.e. preconditioned CG on
// A^T A x = A^T b with preconditioner M = T T^T (the reading of the unstated
// step size: the paper names CG as interchangeable with its gradient step).
//
// Each iteration needs A p and A^T (A p).  normal_pass_kernel produces both
// from one read of A: a workgroup stages RC rows x d columns of A in LDS,
// forms r = [b] - A p for those rows (FP64 products and sums), and adds
// A_chunk^T r to its per-column FP64 accumulators; the workgroup's partial
// A^T r and ||r||^2 are summed in a fixed order by the update kernel, which
// also does the d-dimensional CG algebra (one workgroup, FP64).
#include "common.hpp"

namespace rmm {

namespace {

constexpr int kPassThreads = 256;

__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
  return s;
}

// elements of A per thread and chunk: 64 fp32 / 32 fp64 values (64 VGPRs)
template <typename T>
constexpr int pass_per() {
  return sizeof(T) == 4 ? 64 : 32;
}

// part[g * (d + 1) + j] = sum over this workgroup's rows i of A_ij r_i,
// part[g * (d + 1) + d] = sum of r_i^2, with r_i = (b ? b_i : 0) - (A p)_i.
// The chunk is staged row-major (stride d + 1, odd for even d, so the
// transposing stores and the column reads of phase 2 hit distinct banks);
// the next chunk's loads are in registers while the current one is used.
template <typename T, int RC, bool VEC>
__global__ __launch_bounds__(kPassThreads) void normal_pass_kernel(
    int64_t m, int d, const T* __restrict__ A, int64_t lda, const T* __restrict__ b,
    const double* __restrict__ p, int64_t rows_per_group, double* __restrict__ part) {
  constexpr int NP = kPassThreads / RC;  // threads sharing one row in phase 1
  constexpr int PER = pass_per<T>();     // staged elements per thread (RC d <= PER * 256)
  extern __shared__ __align__(16) unsigned char smem[];
  double* pv = reinterpret_cast<double*>(smem);  // d (+ padding to a multiple of 2)
  double* qpart = pv + ((d + 1) & ~1);            // NP x RC
  double* qv = qpart + NP * RC;                   // RC
  double* red = qv + RC;                          // 4
  T* tile = reinterpret_cast<T*>(red + 4);        // RC x (d + 1), row-major
  const int ldt = d + 1;
  const int tid = threadIdx.x;
  for (int j = tid; j < d; j += kPassThreads) pv[j] = p[j];
  const int64_t row0 = (int64_t)blockIdx.x * rows_per_group;
  int64_t row1 = row0 + rows_per_group;
  if (row1 > m) row1 = m;
  double wacc[4] = {0.0, 0.0, 0.0, 0.0};  // columns tid + 256 c (d <= 1024)
  double qq = 0.0;
  const int prow = tid % RC, ppart = tid / RC;
  const int c0 = ppart * d / NP, c1 = (ppart + 1) * d / NP;
  const int total = RC * d;
  // vector v of a chunk: rows VW (v % (RC / VW)) .. + VW - 1 of column
  // v / (RC / VW); consecutive threads read consecutive rows of one column
  // with 16-byte loads (narrower loads measured at half the bandwidth)
  constexpr int VW = 16 / sizeof(T);
  constexpr int NV = PER / VW;
  constexpr int VPC = RC / VW;  // vectors per column of the chunk
  const int nvec = total / VW;
  T v[PER];
  auto load = [&](int64_t r0) {
    const bool full = VEC && r0 + RC <= row1;
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int e = tid + u * kPassThreads;
      const int rg = e % VPC, cc = e / VPC;
      const int64_t i = r0 + VW * rg;
      const T* src = A + i + (int64_t)cc * lda;
      if (full && e < nvec) {
        if constexpr (sizeof(T) == 4) {
          const float4 q = ld_stream(reinterpret_cast<const float4*>(src));
          v[4 * u] = q.x; v[4 * u + 1] = q.y; v[4 * u + 2] = q.z; v[4 * u + 3] = q.w;
        } else {
          const double2 q = ld_stream(reinterpret_cast<const double2*>(src));
          v[2 * u] = q.x; v[2 * u + 1] = q.y;
        }
      } else {
#pragma unroll
        for (int k = 0; k < VW; ++k)
          v[VW * u + k] = (e < nvec && i + k < row1) ? src[k] : T(0);
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int e = tid + u * kPassThreads;
      if (e < nvec) {
        const int rg = e % VPC, cc = e / VPC;
#pragma unroll
        for (int k = 0; k < VW; ++k) tile[(VW * rg + k) * ldt + cc] = v[VW * u + k];
      }
    }
  };
  if (row0 < row1) load(row0);
  for (int64_t r0 = row0; r0 < row1; r0 += RC) {
    lds_barrier();  // the previous chunk is no longer read (LDS-only barriers: the
                    // prefetch loads stay in flight across them)
    store();
    if (r0 + RC < row1) load(r0 + RC);
    lds_barrier();
    // phase 1: (A p) for the RC rows, NP threads per row over column ranges
    const T* trow = tile + prow * ldt;
    double sp = 0.0;
    for (int c = c0; c < c1; ++c) sp += (double)trow[c] * pv[c];
    qpart[ppart * RC + prow] = sp;
    lds_barrier();
    if (tid < RC) {
      const int64_t i = r0 + tid;
      double q = 0.0;
      if (i < row1) {
        double ap = 0.0;
        for (int k = 0; k < NP; ++k) ap += qpart[k * RC + tid];
        q = (b ? (double)b[i] : 0.0) - ap;
      }
      qv[tid] = q;
      qq += q * q;
    }
    lds_barrier();
    // phase 2: A_chunk^T r into the column accumulators
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int j = tid + c * kPassThreads;
      if (j < d) {
        double s = 0.0;
#pragma unroll 8
        for (int rr = 0; rr < RC; ++rr) s += (double)tile[rr * ldt + j] * qv[rr];
        wacc[c] += s;
      }
    }
  }
  double* out = part + (int64_t)blockIdx.x * (d + 1);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int j = tid + c * kPassThreads;
    if (j < d) out[j] = wacc[c];
  }
  const double tot = block_sum(qq, red);
  if (tid == 0) out[d] = tot;
}

// First level of the fixed-order sum of the partials: group k of kFold
// partial rows -> fold row k.
constexpr int kFold = 16;
__global__ __launch_bounds__(256) void fold_parts_kernel(const double* __restrict__ part, int G,
                                                         int n, double* __restrict__ fold) {
  const int k = blockIdx.x;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    double v[kFold];
#pragma unroll
    for (int u = 0; u < kFold; ++u) {
      const int g = k * kFold + u;
      v[u] = g < G ? part[(int64_t)g * n + j] : 0.0;
    }
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < kFold; ++u) s += v[u];
    fold[(int64_t)k * n + j] = s;
  }
}

// Second level: the F fold rows (F <= 64) into vec (d) and, if sq, the last entry.
__device__ __forceinline__ void reduce_folds(const double* __restrict__ fold, int F, int d,
                                             double* vec, double* sq) {
  for (int j = threadIdx.x; j <= d; j += blockDim.x) {
    double v[64];
#pragma unroll
    for (int u = 0; u < 64; ++u) v[u] = u < F ? fold[(int64_t)u * (d + 1) + j] : 0.0;
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < 64; ++u) s += v[u];
    if (j < d) vec[j] = s;
    else if (sq) *sq = s;
  }
}

// y = M g (M symmetric d x d, column-major; g staged in LDS) into y;
// returns g . y on every thread.
__device__ __forceinline__ double apply_m(int d, const double* __restrict__ M, const double* gl,
                                          double* y, double* red) {
  double dot = 0.0;
  for (int i = threadIdx.x; i < d; i += blockDim.x) {
    double s = 0.0;
    int k = 0;
    for (; k + 8 <= d; k += 8) {
      double mv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) mv[u] = M[i + (int64_t)(k + u) * d];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += mv[u] * gl[k + u];
    }
    for (; k < d; ++k) s += M[i + (int64_t)k * d] * gl[k];
    y[i] = s;
    dot += s * gl[i];
  }
  return block_sum(dot, red);
}

// state: g (gradient A^T (b - A x)), y, p (d each), sc[0] = gamma = g . y
__global__ __launch_bounds__(256) void pcg_init_kernel(int d, const double* __restrict__ fold, int F,
                                                       const double* __restrict__ M, double* g,
                                                       double* y, double* p, double* sc) {
  extern __shared__ double gl[];  // d
  __shared__ double red[4];
  reduce_folds(fold, F, d, gl, nullptr);
  __syncthreads();
  for (int i = threadIdx.x; i < d; i += blockDim.x) g[i] = gl[i];
  const double gam = apply_m(d, M, gl, y, red);
  for (int i = threadIdx.x; i < d; i += blockDim.x) p[i] = y[i];
  if (threadIdx.x == 0) sc[0] = gam;
}

// After the pass with r = -A p: w = -A^T A p, qq = ||A p||^2.
//   alpha = gamma / qq; x += alpha p; g += alpha w; y = M g; gamma' = g . y;
//   p = y + (gamma' / gamma) p.
__global__ __launch_bounds__(256) void pcg_step_kernel(int d, const double* __restrict__ fold, int F,
                                                       const double* __restrict__ M, double* x,
                                                       double* g, double* y, double* p,
                                                       double* sc) {
  extern __shared__ double gl[];  // d: w, then the new g
  __shared__ double red[4];
  __shared__ double qq;
  reduce_folds(fold, F, d, gl, &qq);
  __syncthreads();
  const double gam = sc[0];
  const double alpha = (qq > 0.0) ? gam / qq : 0.0;
  for (int i = threadIdx.x; i < d; i += blockDim.x) {
    x[i] += alpha * p[i];
    const double gi = g[i] + alpha * gl[i];
    g[i] = gi;
    gl[i] = gi;
  }
  __syncthreads();
  const double gnew = apply_m(d, M, gl, y, red);
  const double beta = (gam > 0.0) ? gnew / gam : 0.0;
  for (int i = threadIdx.x; i < d; i += blockDim.x) p[i] = y[i] + beta * p[i];
  if (threadIdx.x == 0) sc[0] = gnew;
}

__global__ void sqrt_last_kernel(const double* __restrict__ fold, int F, int d, double* out) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int k = 0; k < F; ++k) s += fold[(int64_t)k * (d + 1) + d];
  *out = sqrt(s);
}

// rows per chunk: the largest power of two <= 64 with RC d <= PER * 256
template <typename T>
int pass_rc(int d) {
  int rc = 64;
  while (rc > 1 && rc * d > pass_per<T>() * kPassThreads) rc /= 2;
  return rc;
}

template <typename T>
size_t pass_lds(int d, int rc) {
  return (size_t)(((d + 1) & ~1) + (kPassThreads / rc) * rc + rc + 4) * sizeof(double) +
         (size_t)rc * (d + 1) * sizeof(T);
}

int fold_count(int G) { return (G + kFold - 1) / kFold; }

}  // namespace

int refine_groups(const rmm_ctx* h) { return 2 * h->cus; }

size_t refine_part_elems(const rmm_ctx* h, int d) {
  const int G = refine_groups(h);
  return (size_t)(G + fold_count(G)) * (d + 1);
}

template <typename T>
int normal_pass(const rmm_ctx* h, int64_t m, int d, const T* A, int64_t lda, const T* b,
                const double* p, double* part) {
  if (d > 1024) return RMM_ERR_UNSUPPORTED;
  const int G = refine_groups(h);
  const int rc = pass_rc<T>(d);
  int64_t per = (m + G - 1) / G;
  per = (per + rc - 1) / rc * rc;
  const size_t lds = pass_lds<T>(d, rc);
  const bool vec = ((uintptr_t)A % 16 == 0) && (lda % (16 / (int64_t)sizeof(T)) == 0);
#define RMM_PASS(RC)                                                                          \
  case RC: {                                                                                  \
    auto kern = vec ? normal_pass_kernel<T, RC, true> : normal_pass_kernel<T, RC, false>;     \
    RMM_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, \
                                (int)lds));                                                   \
    hipLaunchKernelGGL(kern, dim3(G), dim3(kPassThreads), lds, h->stream, m, d, A, lda, b, p,  \
                       per, part);                                                            \
    break;                                                                                    \
  }
  switch (rc) {
    RMM_PASS(64)
    RMM_PASS(32)
    RMM_PASS(16)
    RMM_PASS(8)
    default:
      return RMM_ERR_UNSUPPORTED;
  }
#undef RMM_PASS
  RMM_TRY(launch_status());
  hipLaunchKernelGGL(fold_parts_kernel, dim3(fold_count(G)), dim3(256), 0, h->stream, part, G, d + 1,
                     part + (size_t)G * (d + 1));
  return launch_status();
}

int pcg_init(const rmm_ctx* h, int d, const double* part, const double* M, double* g, double* y,
             double* p, double* sc) {
  const int G = refine_groups(h);
  hipLaunchKernelGGL(pcg_init_kernel, dim3(1), dim3(256), (size_t)d * sizeof(double), h->stream, d,
                     part + (size_t)G * (d + 1), fold_count(G), M, g, y, p, sc);
  return launch_status();
}

int pcg_step(const rmm_ctx* h, int d, const double* part, const double* M, double* x, double* g,
             double* y, double* p, double* sc) {
  const int G = refine_groups(h);
  hipLaunchKernelGGL(pcg_step_kernel, dim3(1), dim3(256), (size_t)d * sizeof(double), h->stream, d,
                     part + (size_t)G * (d + 1), fold_count(G), M, x, g, y, p, sc);
  return launch_status();
}

int pass_resid(const rmm_ctx* h, int d, const double* part, double* out) {
  const int G = refine_groups(h);
  hipLaunchKernelGGL(sqrt_last_kernel, dim3(1), dim3(64), 0, h->stream, part + (size_t)G * (d + 1),
                     fold_count(G), d, out);
  return launch_status();
}

template int normal_pass<float>(const rmm_ctx*, int64_t, int, const float*, int64_t, const float*,
                                const double*, double*);
template int normal_pass<double>(const rmm_ctx*, int64_t, int, const double*, int64_t,
                                 const double*, const double*, double*);

}  // namespace rmm
