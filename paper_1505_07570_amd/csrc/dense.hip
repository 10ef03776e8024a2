// Dense building blocks of the drivers: MFMA GEMMs with split-K, and the
// elementwise / GEMV helpers around them.
//
// gemm: C = alpha * op(A) * op(B), column-major, op = identity or transpose.
//  * workgroup tile BM x BN, 4 waves in a 2 x 2 grid, 16x16x4 MFMA in fp32 or
//    fp64 (the compute type TC); inputs of either precision are converted
//    to TC when they are staged into LDS;
//  * the K dimension is split over gridDim.z; each split writes a partial
//    tile and a fixed-order reduction adds them in fp64 and converts to the
//    output type, so results do not depend on scheduling.
#include <type_traits>

#include "common.hpp"
#include "dense.hpp"

namespace rmm {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename TC>
struct Mfma;
template <>
struct Mfma<float> {
  using acc = floatx4;
  static __device__ __forceinline__ acc run(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // row of D held in register v by lane group g = lane >> 4
  static __device__ __forceinline__ int row(int g, int v) { return 4 * g + v; }
};
template <>
struct Mfma<double> {
  using acc = doublex4;
  static __device__ __forceinline__ acc run(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g, int v) { return g + 4 * v; }
};

constexpr int kBK = 16;

// Epilogue: a partial tile of a split product is stored as is (alpha = 1,
// beta = 0); an unsplit product whose output type is the compute type is
// finished in place, with the arithmetic of gemm_reduce_kernel for one split.
template <typename TC>
__device__ __forceinline__ void gemm_store(TC* p, TC acc, double alpha, double beta) {
  double v = alpha * (double)acc;
  if (beta != 0.0) v += beta * (double)*p;
  *p = (TC)v;
}

// op(X)[i, k] for a column-major X: X[i + k*ld] or, transposed, X[k + i*ld]
template <typename T, bool TR>
__device__ __forceinline__ T opget(const T* __restrict__ X, int64_t ld, int64_t i, int64_t k) {
  return TR ? X[k + i * ld] : X[i + k * ld];
}

template <typename TAI, typename TBI, typename TC, bool TA, bool TB, int BM, int BN>
__global__ __launch_bounds__(256) void gemm_kernel(int M, int N, int64_t K, const TAI* __restrict__ A,
                                                   int64_t lda, const TBI* __restrict__ B, int64_t ldb,
                                                   TC* __restrict__ P, int64_t kchunk, int64_t ldp,
                                                   double alpha, double beta) {
  using F = Mfma<TC>;
  using acc_t = typename F::acc;
  constexpr int WM = BM / 2, WN = BN / 2;  // wave tile
  constexpr int TM = WM / 16, TN = WN / 16;
  __shared__ TC As[kBK][BM + 1];
  __shared__ TC Bs[kBK][BN + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  const int64_t k0 = (int64_t)blockIdx.z * kchunk;
  int64_t k1 = k0 + kchunk;
  if (k1 > K) k1 = K;
  acc_t acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

  const int g = lane >> 4, c16 = lane & 15;
  // operands of the next K stage are loaded into registers while the
  // current one is multiplied (one LDS buffer, two barriers per stage)
  constexpr int AE = BM * kBK / 256, BE = BN * kBK / 256;
  TC ra[AE], rb[BE];
  auto load = [&](int64_t kb) {
#pragma unroll
    for (int u = 0; u < AE; ++u) {
      const int e = tid + 256 * u;
      int i, kk;
      if (TA) { kk = e % kBK; i = e / kBK; } else { i = e % BM; kk = e / BM; }
      const int64_t gi = m0 + i, gk = kb + kk;
      ra[u] = (gi < M && gk < k1) ? (TC)opget<TAI, TA>(A, lda, gi, gk) : TC(0);
    }
#pragma unroll
    for (int u = 0; u < BE; ++u) {
      const int e = tid + 256 * u;
      int j, kk;
      // op(B)[k, j]: B[k + j*ldb] (k fastest) or, transposed, B[j + k*ldb]
      if (TB) { j = e % BN; kk = e / BN; } else { kk = e % kBK; j = e / kBK; }
      const int64_t gj = n0 + j, gk = kb + kk;
      TC v = TC(0);
      if (gj < N && gk < k1) v = (TC)(TB ? B[gj + gk * ldb] : B[gk + gj * ldb]);
      rb[u] = v;
    }
  };
  if (k0 < k1) load(k0);
  for (int64_t kb = k0; kb < k1; kb += kBK) {
#pragma unroll
    for (int u = 0; u < AE; ++u) {
      const int e = tid + 256 * u;
      int i, kk;
      if (TA) { kk = e % kBK; i = e / kBK; } else { i = e % BM; kk = e / BM; }
      As[kk][i] = ra[u];
    }
#pragma unroll
    for (int u = 0; u < BE; ++u) {
      const int e = tid + 256 * u;
      int j, kk;
      if (TB) { j = e % BN; kk = e / BN; } else { kk = e % kBK; j = e / kBK; }
      Bs[kk][j] = rb[u];
    }
    __syncthreads();
    if (kb + kBK < k1) load(kb + kBK);
#pragma unroll
    for (int ks = 0; ks < kBK; ks += 4) {
      TC av[TM], bv[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) av[a] = As[ks + g][wm * WM + a * 16 + c16];
#pragma unroll
      for (int b = 0; b < TN; ++b) bv[b] = Bs[ks + g][wn * WN + b * 16 + c16];
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = F::run(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
  TC* dst = P + (int64_t)blockIdx.z * M * N;
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      const int j = n0 + wn * WN + b * 16 + c16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = m0 + wm * WM + a * 16 + F::row(g, v);
        if (i < M && j < N) gemm_store(dst + i + (int64_t)j * ldp, acc[a][b][v], alpha, beta);
      }
    }
}

// Fast path for C = A B (no transposes, inputs already in the compute type,
// 16-byte aligned columns): 128 x 128 tiles, 4 waves of 64 x 64, operands
// staged with 16-byte loads (A along its columns, B along k) one stage ahead
// in registers, double-buffered LDS, one barrier per 16-wide K stage.
template <typename T>
__global__ __launch_bounds__(256) void gemm_nn_kernel(int M, int N, int64_t K, const T* __restrict__ A,
                                                      int64_t lda, const T* __restrict__ B, int64_t ldb,
                                                      T* __restrict__ P, int64_t kchunk, int64_t ldp,
                                                      double alpha, double beta) {
  using F = Mfma<T>;
  using acc_t = typename F::acc;
  constexpr int BM = 128, BN = 128, BK = sizeof(T) == 4 ? 2 * kBK : kBK;
  constexpr int V = 16 / (int)sizeof(T);        // elements per 16-byte load
  constexpr int AL = BM * BK / V / 256;          // A loads per thread per stage
  constexpr int BL = BN * BK / V / 256;          // B loads per thread per stage
  __shared__ __align__(16) T As[2][BK][BM + 4];
  __shared__ __align__(16) T Bs[2][BK][BN + 4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  const int64_t k0 = (int64_t)blockIdx.z * kchunk;
  int64_t k1 = k0 + kchunk;
  if (k1 > K) k1 = K;
  acc_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
  T ra[AL][V], rb[BL][V];
  auto load = [&](int64_t kb) {
    const bool fa = (m0 + BM <= M) && (kb + BK <= k1);
    const bool fb = (n0 + BN <= N) && (kb + BK <= k1);
#pragma unroll
    for (int u = 0; u < AL; ++u) {
      const int e = tid + 256 * u;             // (k, i-group)
      const int kk = e / (BM / V), ig = e % (BM / V);
      const int64_t gk = kb + kk;
      const int64_t gi = m0 + ig * V;
      if (fa) {
        const T* src = A + gi + gk * lda;
        if constexpr (sizeof(T) == 4) {
          const float4 x = *reinterpret_cast<const float4*>(src);
          ra[u][0] = x.x; ra[u][1] = x.y; ra[u][2] = x.z; ra[u][3] = x.w;
        } else {
          const double2 x = *reinterpret_cast<const double2*>(src);
          ra[u][0] = x.x; ra[u][1] = x.y;
        }
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v) ra[u][v] = (gi + v < M && gk < k1) ? A[gi + v + gk * lda] : T(0);
      }
    }
#pragma unroll
    for (int u = 0; u < BL; ++u) {
      const int e = tid + 256 * u;             // (j, k-group)
      const int j = e / (BK / V), kg = e % (BK / V);
      const int64_t gj = n0 + j;
      const int64_t gk = kb + kg * V;
      if (fb) {
        const T* src = B + gk + gj * ldb;
        if constexpr (sizeof(T) == 4) {
          const float4 x = *reinterpret_cast<const float4*>(src);
          rb[u][0] = x.x; rb[u][1] = x.y; rb[u][2] = x.z; rb[u][3] = x.w;
        } else {
          const double2 x = *reinterpret_cast<const double2*>(src);
          rb[u][0] = x.x; rb[u][1] = x.y;
        }
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v) rb[u][v] = (gj < N && gk + v < k1) ? B[gk + v + gj * ldb] : T(0);
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < AL; ++u) {
      const int e = tid + 256 * u;
      const int kk = e / (BM / V), ig = e % (BM / V);
#pragma unroll
      for (int v = 0; v < V; ++v) As[buf][kk][ig * V + v] = ra[u][v];
    }
#pragma unroll
    for (int u = 0; u < BL; ++u) {
      const int e = tid + 256 * u;
      const int j = e / (BK / V), kg = e % (BK / V);
#pragma unroll
      for (int v = 0; v < V; ++v) Bs[buf][kg * V + v][j] = rb[u][v];
    }
  };
  const int g = lane >> 4, c16 = lane & 15;
  const int64_t nst = (k1 - k0 + BK - 1) / BK;
  if (nst > 0) {
    load(k0);
    store(0);
  }
  __syncthreads();
  for (int64_t st = 0; st < nst; ++st) {
    const int buf = (int)(st & 1);
    const bool more = st + 1 < nst;
    if (more) load(k0 + (st + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      T av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[buf][ks + g][wm * 64 + a * 16 + c16];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Bs[buf][ks + g][wn * 64 + b * 16 + c16];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = F::run(av[a], bv[b], acc[a][b]);
    }
    if (more) store(buf ^ 1);
    __syncthreads();
  }
  T* dst = P + (int64_t)blockIdx.z * M * N;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int j = n0 + wn * 64 + b * 16 + c16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = m0 + wm * 64 + a * 16 + F::row(g, v);
        if (i < M && j < N) gemm_store(dst + i + (int64_t)j * ldp, acc[a][b][v], alpha, beta);
      }
    }
}

// y = op(A)^T x for one right-hand column (N = 1, A transposed): a wave
// per output, lanes striding along K with 16-byte loads when the columns
// allow them; the K range may be split over gridDim.y like the products.
// Lane sums are combined by a fixed butterfly, so results are reproducible.
template <typename TAI, typename TBI, typename TC, bool VEC>
__global__ __launch_bounds__(256) void gemv_tn_kernel(int M, int64_t K, const TAI* __restrict__ A,
                                                      int64_t lda, const TBI* __restrict__ x,
                                                      TC* __restrict__ P, int64_t kchunk,
                                                      double alpha, double beta) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= M) return;  // whole waves
  const int64_t k0 = (int64_t)blockIdx.y * kchunk;
  const int64_t k1 = k0 + kchunk < K ? k0 + kchunk : K;
  const TAI* a = A + (int64_t)i * lda;
  TC acc = TC(0);
  if constexpr (VEC && sizeof(TAI) == sizeof(TBI)) {
    constexpr int V = 16 / (int)sizeof(TAI);
    for (int64_t k = k0 + (int64_t)lane * V; k < k1; k += 64 * V) {
      TAI av[V];
      TBI xv[V];
      *reinterpret_cast<uint4*>(av) = *reinterpret_cast<const uint4*>(a + k);
      *reinterpret_cast<uint4*>(xv) = *reinterpret_cast<const uint4*>(x + k);
#pragma unroll
      for (int v = 0; v < V; ++v) acc = fma((TC)av[v], (TC)xv[v], acc);
    }
  } else {
    for (int64_t k = k0 + lane; k < k1; k += 64) acc = fma((TC)a[k], (TC)x[k], acc);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) gemm_store(P + (int64_t)blockIdx.y * M + i, acc, alpha, beta);
}

// K split of the one-column product: enough waves to cover the CUs a few
// times, at least 1024 elements per split, split boundaries on 256
static int64_t gemv_kchunk(const rmm_ctx* h, int M, int64_t K) {
  int64_t want = (4LL * h->cus + M - 1) / M;
  const int64_t most = (K + 1023) / 1024;
  if (want > most) want = most;
  if (want < 1) want = 1;
  int64_t kc = (K + want - 1) / want;
  kc = (kc + 255) / 256 * 256;
  return kc < 256 ? 256 : kc;
}

template <typename TC, typename TO>
__global__ void gemm_reduce_kernel(int M, int N, const TC* __restrict__ P, int splits, double alpha,
                                   double beta, TO* __restrict__ C, int64_t ldc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i >= M) return;
  double acc = 0.0;
  for (int z = 0; z < splits; ++z) acc += (double)P[(int64_t)z * M * N + i + j * M];
  double v = alpha * acc;
  if (beta != 0.0) v += beta * (double)C[i + j * ldc];
  C[i + j * ldc] = (TO)v;
}

// The same reduction for many splits (small outputs such as the l x l Gram
// matrices of tall panels): a workgroup takes 64 consecutive outputs, wave
// w sums the splits z = w, w + 4, ... with four loads in flight, and the four
// wave sums are added in a fixed order.
constexpr int kRedWide = 8;  // splits from which the wide reduction is used

template <typename TC, typename TO>
__global__ __launch_bounds__(256) void gemm_reduce_wide_kernel(int M, int N, const TC* __restrict__ P,
                                                               int splits, double alpha, double beta,
                                                               TO* __restrict__ C, int64_t ldc) {
  __shared__ double part[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t MN = (int64_t)M * N;
  const int64_t o = (int64_t)blockIdx.x * 64 + lane;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  if (o < MN) {
    int z = wave;
    for (; z + 12 < splits; z += 16) {
#pragma unroll
      for (int u = 0; u < 4; ++u) s[u] += (double)P[(int64_t)(z + 4 * u) * MN + o];
    }
    for (; z < splits; z += 4) s[0] += (double)P[(int64_t)z * MN + o];
  }
  part[wave][lane] = (s[0] + s[1]) + (s[2] + s[3]);
  __syncthreads();
  if (wave == 0 && o < MN) {
    const double acc = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
    const int64_t i = o % M, j = o / M;
    double v = alpha * acc;
    if (beta != 0.0) v += beta * (double)C[i + j * ldc];
    C[i + j * ldc] = (TO)v;
  }
}

template <typename TC, typename TO>
void launch_gemm_reduce(const rmm_ctx* h, int M, int N, const TC* P, int splits, double alpha, double beta,
                        TO* C, int64_t ldc) {
  if (splits >= kRedWide) {
    const int64_t blocks = ((int64_t)M * N + 63) / 64;
    hipLaunchKernelGGL((gemm_reduce_wide_kernel<TC, TO>), dim3((unsigned)blocks), dim3(256), 0, h->stream,
                       M, N, P, splits, alpha, beta, C, ldc);
  } else {
    dim3 grid((unsigned)((M + 255) / 256), (unsigned)N);
    hipLaunchKernelGGL((gemm_reduce_kernel<TC, TO>), grid, dim3(256), 0, h->stream, M, N, P, splits, alpha,
                       beta, C, ldc);
  }
}

namespace {

struct GemmShape {
  int BM, BN, splits;
  int64_t kchunk;
  bool nn;  // the 128 x 128 kernel may be used (untransposed, same types, aligned)
};

// Candidate launch plans of a product: column tile (0 = 128 above N = 64),
// workgroups per CU targeted by the K split, and whether the 128 x 128 fast
// path may be taken.  Plan 0 is the default; rmm_set_autotune times the
// others on the first call of a shape and keeps the fastest per handle.
struct GemmPlan {
  int bn, per_cu;
  bool nn;
};
constexpr GemmPlan kGemmPlans[] = {{0, 2, true}, {0, 1, true}, {0, 4, true}, {64, 2, true},
                                   {0, 2, false}, {64, 4, false}};
constexpr int kNumGemmPlans = sizeof(kGemmPlans) / sizeof(kGemmPlans[0]);
constexpr int kMaxPlanPerCu = 4;

GemmShape gemm_shape(const rmm_ctx* h, int M, int N, int64_t K, int plan = 0) {
  const GemmPlan& pl = kGemmPlans[plan];
  GemmShape g;
  g.BM = 64;
  g.BN = pl.bn ? pl.bn : (N > 64 ? 128 : 64);
  g.nn = pl.nn;
  const int64_t tiles = (int64_t)((M + g.BM - 1) / g.BM) * ((N + g.BN - 1) / g.BN);
  int64_t want = ((int64_t)pl.per_cu * h->cus + tiles - 1) / tiles;
  const int64_t maxsplit = (K + 255) / 256;  // at least 256 K per split
  if (want > maxsplit) want = maxsplit;
  if (want < 1) want = 1;
  int64_t kc = (K + want - 1) / want;
  kc = (kc + kBK - 1) / kBK * kBK;
  if (kc < kBK) kc = kBK;
  g.kchunk = kc;
  g.splits = K > 0 ? (int)((K + kc - 1) / kc) : 1;
  return g;
}

template <typename TAI, typename TBI, typename TC, bool TA, bool TB>
int launch_gemm_t(const rmm_ctx* h, const GemmShape& g, int M, int N, int64_t K, const TAI* A,
                  int64_t lda, const TBI* B, int64_t ldb, TC* P, int64_t ldp, double alpha,
                  double beta) {
  dim3 grid((unsigned)((M + g.BM - 1) / g.BM), (unsigned)((N + g.BN - 1) / g.BN),
            (unsigned)g.splits);
  if (g.BN == 128)
    hipLaunchKernelGGL((gemm_kernel<TAI, TBI, TC, TA, TB, 64, 128>), grid, dim3(256), 0, h->stream,
                       M, N, K, A, lda, B, ldb, P, g.kchunk, ldp, alpha, beta);
  else
    hipLaunchKernelGGL((gemm_kernel<TAI, TBI, TC, TA, TB, 64, 64>), grid, dim3(256), 0, h->stream,
                       M, N, K, A, lda, B, ldb, P, g.kchunk, ldp, alpha, beta);
  return launch_status();
}

}  // namespace

// the partials of every candidate plan fit (any tuned plan can run)
template <typename TC>
size_t gemm_workspace(const rmm_ctx* h, int M, int N, int64_t K) {
  size_t most = 0;
  for (int p = 0; p < kNumGemmPlans; ++p) {
    const GemmShape g = gemm_shape(h, M, N, K, p);
    const size_t e = (size_t)g.splits * M * N;
    if (e > most) most = e;
  }
  if (N == 1 && K > 0) {
    const int64_t kc = gemv_kchunk(h, M, K);
    const size_t e = (size_t)((K + kc - 1) / kc) * M;
    if (e > most) most = e;
  }
  Carver c(nullptr, 0);
  c.take<TC>(most);
  return c.off;
}

template <typename TAI, typename TBI, typename TC, typename TO>
int gemm_plan(rmm_ctx* h, int plan, bool ta, bool tb, int M, int N, int64_t K, const TAI* A,
              int64_t lda, const TBI* B, int64_t ldb, double alpha, TO* C, int64_t ldc,
              Carver& ws, double beta) {
  if (ta && !tb && N == 1 && K > 0) {
    const int64_t kc = gemv_kchunk(h, M, K);
    const int splits = (int)((K + kc - 1) / kc);
    const size_t mark = ws.off;
    bool direct = false;
    if constexpr (std::is_same<TO, TC>::value) direct = splits == 1;
    TC* P = direct ? (TC*)C : ws.take<TC>((size_t)splits * M);
    if (!ws.fits()) return RMM_ERR_WORKSPACE_TOO_SMALL;
    const double pa = direct ? alpha : 1.0, pb = direct ? beta : 0.0;
    constexpr int V = 16 / (int)sizeof(TAI);
    const bool vec = sizeof(TAI) == sizeof(TBI) && (uintptr_t)A % 16 == 0 &&
                     (uintptr_t)B % 16 == 0 && lda % V == 0 && K % V == 0;
    dim3 grid((unsigned)((M + 3) / 4), (unsigned)splits);
    if (vec && sizeof(TAI) == sizeof(TBI))
      hipLaunchKernelGGL((gemv_tn_kernel<TAI, TBI, TC, sizeof(TAI) == sizeof(TBI)>), grid, dim3(256),
                         0, h->stream, M, K, A, lda, B, P, kc, pa, pb);
    else
      hipLaunchKernelGGL((gemv_tn_kernel<TAI, TBI, TC, false>), grid, dim3(256), 0, h->stream, M, K,
                         A, lda, B, P, kc, pa, pb);
    RMM_TRY(launch_status());
    if (!direct) {
      dim3 rgrid((unsigned)((M + 255) / 256), 1u);
      hipLaunchKernelGGL((gemm_reduce_kernel<TC, TO>), rgrid, dim3(256), 0, h->stream, M, 1, P,
                         splits, alpha, beta, C, ldc);
    }
    ws.off = mark;
    return launch_status();
  }
  const GemmShape g = gemm_shape(h, M, N, K, plan);
  const size_t mark = ws.off;
  // one split with the output in the compute type: the product kernel
  // finishes C itself and no partials or reduction are needed
  bool direct = false;
  if constexpr (std::is_same<TO, TC>::value) direct = g.splits == 1;
  TC* P = direct ? (TC*)C : ws.take<TC>((size_t)g.splits * M * N);
  if (!ws.fits()) return RMM_ERR_WORKSPACE_TOO_SMALL;
  const int64_t ldp = direct ? ldc : M;
  const double pa = direct ? alpha : 1.0, pb = direct ? beta : 0.0;
  int rc;
  constexpr bool same = std::is_same<TAI, TC>::value && std::is_same<TBI, TC>::value;
  const int64_t va = 16 / sizeof(TC);
  bool fast = false;
  if constexpr (same) {
    if (g.nn && !ta && !tb && N > 64 && (uintptr_t)A % 16 == 0 && (uintptr_t)B % 16 == 0 &&
        lda % va == 0 && ldb % va == 0) {
      dim3 grid((unsigned)((M + 127) / 128), (unsigned)((N + 127) / 128), (unsigned)g.splits);
      hipLaunchKernelGGL((gemm_nn_kernel<TC>), grid, dim3(256), 0, h->stream, M, N, K,
                         (const TC*)A, lda, (const TC*)B, ldb, P, g.kchunk, ldp, pa, pb);
      RMM_TRY(launch_status());
      fast = true;
    }
  }
  if (!fast) {
    if (!ta && !tb)
      rc = launch_gemm_t<TAI, TBI, TC, false, false>(h, g, M, N, K, A, lda, B, ldb, P, ldp, pa, pb);
    else if (ta && !tb)
      rc = launch_gemm_t<TAI, TBI, TC, true, false>(h, g, M, N, K, A, lda, B, ldb, P, ldp, pa, pb);
    else if (!ta && tb)
      rc = launch_gemm_t<TAI, TBI, TC, false, true>(h, g, M, N, K, A, lda, B, ldb, P, ldp, pa, pb);
    else
      rc = launch_gemm_t<TAI, TBI, TC, true, true>(h, g, M, N, K, A, lda, B, ldb, P, ldp, pa, pb);
    RMM_TRY(rc);
  }
  if (direct) {
    ws.off = mark;
    return RMM_OK;
  }
  launch_gemm_reduce<TC, TO>(h, M, N, P, g.splits, alpha, beta, C, ldc);
  ws.off = mark;  // the partials are dead once the reduction is enqueued
  return launch_status();
}

// Tuning (rmm_set_autotune): each candidate plan runs twice on the caller's
// operands, timed with events on the handle's stream (this synchronizes, so
// it is off by default and not for graph capture); the fastest is kept for
// the shape.  Products that accumulate into C (beta != 0) are not tuned.
template <typename TAI, typename TBI, typename TC, typename TO>
int gemm(rmm_ctx* h, bool ta, bool tb, int M, int N, int64_t K, const TAI* A, int64_t lda,
         const TBI* B, int64_t ldb, double alpha, TO* C, int64_t ldc, Carver& ws, double beta) {
  if (M == 0 || N == 0) return RMM_OK;
  const std::string key = "gemm " + std::to_string(sizeof(TAI)) + std::to_string(sizeof(TBI)) +
                          std::to_string(sizeof(TC)) + std::to_string(sizeof(TO)) +
                          (ta ? "t" : "n") + (tb ? "t" : "n") + " " + std::to_string(M) + " " +
                          std::to_string(N) + " " + std::to_string(K);
  const auto it = h->plans.find(key);
  if (it != h->plans.end() && it->second >= 0 && it->second < kNumGemmPlans)
    return gemm_plan<TAI, TBI, TC, TO>(h, it->second, ta, tb, M, N, K, A, lda, B, ldb, alpha, C,
                                       ldc, ws, beta);
  if (!h->autotune || beta != 0.0)
    return gemm_plan<TAI, TBI, TC, TO>(h, 0, ta, tb, M, N, K, A, lda, B, ldb, alpha, C, ldc, ws,
                                       beta);
  hipEvent_t e0, e1;
  RMM_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return RMM_ERR_HIP;
  }
  int best = 0;
  float best_ms = 0.f;
  int rc = RMM_OK;
  for (int p = 0; p < kNumGemmPlans && rc == RMM_OK; ++p) {
    float ms = 0.f;
    for (int rep = 0; rep < 2 && rc == RMM_OK; ++rep) {
      (void)hipEventRecord(e0, h->stream);
      rc = gemm_plan<TAI, TBI, TC, TO>(h, p, ta, tb, M, N, K, A, lda, B, ldb, alpha, C, ldc, ws,
                                       beta);
      (void)hipEventRecord(e1, h->stream);
      if (hipEventSynchronize(e1) != hipSuccess) rc = RMM_ERR_HIP;
      (void)hipEventElapsedTime(&ms, e0, e1);
    }
    if (rc == RMM_OK && (p == 0 || ms < best_ms)) {
      best = p;
      best_ms = ms;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  RMM_TRY(rc);
  h->plans[key] = best;
  // C holds the last candidate's result; the kept plan writes it again so the
  // output always comes from the plan later calls will use
  return gemm_plan<TAI, TBI, TC, TO>(h, best, ta, tb, M, N, K, A, lda, B, ldb, alpha, C, ldc, ws,
                                     beta);
}

// ---- elementwise helpers ---------------------------------------------------------

template <typename TI, typename TO>
__global__ void copy_cast_kernel(int64_t rows, const TI* __restrict__ X, int64_t ldx,
                                 TO* __restrict__ Y, int64_t ldy) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i < rows) Y[i + j * ldy] = (TO)X[i + j * ldx];
}

template <typename TI, typename TO>
int copy_cast(const rmm_ctx* h, int64_t rows, int64_t cols, const TI* X, int64_t ldx, TO* Y,
              int64_t ldy) {
  if (rows == 0 || cols == 0) return RMM_OK;
  dim3 grid((unsigned)((rows + 255) / 256), (unsigned)cols);
  hipLaunchKernelGGL((copy_cast_kernel<TI, TO>), grid, dim3(256), 0, h->stream, rows, X, ldx, Y, ldy);
  return launch_status();
}

// partial sums of squares of r = A x - b (fp64), one per workgroup
template <typename T>
__global__ __launch_bounds__(256) void residual_kernel(int64_t m, int d, const T* __restrict__ A,
                                                       int64_t lda, const T* __restrict__ b,
                                                       const double* __restrict__ x,
                                                       double* __restrict__ part) {
  __shared__ double xs[1024];
  __shared__ double red[256];
  double acc = 0.0;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double r = 0.0;
  if (i < m) r = -(double)b[i];
  for (int j0 = 0; j0 < d; j0 += 1024) {
    const int nj = (d - j0) < 1024 ? (d - j0) : 1024;
    __syncthreads();
    for (int t = threadIdx.x; t < nj; t += 256) xs[t] = x[j0 + t];
    __syncthreads();
    if (i < m)
      for (int j = 0; j < nj; ++j) r += (double)A[i + (int64_t)(j0 + j) * lda] * xs[j];
  }
  acc = r * r;
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void sum_sqrt_kernel(const double* __restrict__ part, int64_t n, double* __restrict__ out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t t = threadIdx.x; t < n; t += 256) acc += part[t];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sqrt(red[0]);
}

template <typename T>
int residual_norm(const rmm_ctx* h, int64_t m, int d, const T* A, int64_t lda, const T* b,
                  const double* x, double* out, Carver& ws) {
  const int64_t blocks = m > 0 ? (m + 255) / 256 : 1;
  const size_t mark = ws.off;
  double* part = ws.take<double>((size_t)blocks);
  if (!ws.fits()) return RMM_ERR_WORKSPACE_TOO_SMALL;
  if (m > 0) {
    hipLaunchKernelGGL((residual_kernel<T>), dim3((unsigned)blocks), dim3(256), 0, h->stream, m, d, A,
                       lda, b, x, part);
    RMM_TRY(launch_status());
  }
  hipLaunchKernelGGL(sum_sqrt_kernel, dim3(1), dim3(256), 0, h->stream, part, m > 0 ? blocks : 0, out);
  ws.off = mark;
  return launch_status();
}

size_t residual_workspace(int64_t m) {
  Carver c(nullptr, 0);
  c.take<double>((size_t)(m > 0 ? (m + 255) / 256 : 1));
  return c.off;
}

#define RMM_GEMM_INST(TAI, TBI, TC, TO)                                                      \
  template int gemm<TAI, TBI, TC, TO>(rmm_ctx*, bool, bool, int, int, int64_t, const TAI*, \
                                      int64_t, const TBI*, int64_t, double, TO*, int64_t,  \
                                      Carver&, double);
RMM_GEMM_INST(double, double, double, double)
RMM_GEMM_INST(float, float, float, float)
RMM_GEMM_INST(float, float, double, double)
RMM_GEMM_INST(float, double, double, double)
RMM_GEMM_INST(double, float, double, double)
RMM_GEMM_INST(float, double, double, float)
RMM_GEMM_INST(double, double, double, float)
RMM_GEMM_INST(float, float, float, double)
#undef RMM_GEMM_INST

template size_t gemm_workspace<float>(const rmm_ctx*, int, int, int64_t);
template size_t gemm_workspace<double>(const rmm_ctx*, int, int, int64_t);
template int copy_cast<float, double>(const rmm_ctx*, int64_t, int64_t, const float*, int64_t, double*, int64_t);
template int copy_cast<double, float>(const rmm_ctx*, int64_t, int64_t, const double*, int64_t, float*, int64_t);
template int copy_cast<double, double>(const rmm_ctx*, int64_t, int64_t, const double*, int64_t, double*, int64_t);
template int copy_cast<float, float>(const rmm_ctx*, int64_t, int64_t, const float*, int64_t, float*, int64_t);
template int residual_norm<float>(const rmm_ctx*, int64_t, int, const float*, int64_t, const float*,
                                  const double*, double*, Carver&);
template int residual_norm<double>(const rmm_ctx*, int64_t, int, const double*, int64_t,
                                   const double*, const double*, double*, Carver&);

}  // namespace rmm
