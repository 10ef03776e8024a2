// Gaussian-projection sketch C = (Omega / sqrt(s))^T A  (Sec. 3.2.1).
//
// A GEMM with the long dimension m as its reduction:  C (s x n') =
// Omega^T (s x m) * A (m x n').  Omega is never stored: each wave generates
// the entries its MFMA operand needs in registers from the counter-based
// generator, so the only HBM traffic is one read of A and the split-K
// partials.
//
// Tiling (gfx950, 16x16x4 MFMA, fp32 or fp64):
//  * workgroup = 4 waves = 128 sketch rows x (16 NT) columns x one K range;
//  * wave w covers 32 sketch rows as two 16-row MFMA tiles; MFMA row mi of
//    tile t is sketch row m0 + 2 mi + t, so one Box-Muller pair of the
//    generator (the cos / sin entries of columns 2j, 2j+1) feeds both tiles;
//  * A is staged through a double-buffered LDS tile stored column-major
//    with a padded stride that keeps the MFMA operand reads conflict free;
//  * fp32 partial sums are folded into a second accumulator set every
//    4096 rows, so no fp32 running sum spans more than 1024 MFMA steps;
//  * the K ranges are reduced in a fixed order in fp64.
#include "common.hpp"
#include "rng.hpp"

namespace rmm {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename T>
struct GaussCfg;
template <>
struct GaussCfg<float> {
  static constexpr int KS = 32;   // rows per LDS stage
  static constexpr int LDT = 34;  // padded stride (elements) of a tile column
  using acc_t = floatx4;
};
template <>
struct GaussCfg<double> {
  static constexpr int KS = 16;
  static constexpr int LDT = 17;
  using acc_t = doublex4;
};

__device__ __forceinline__ floatx4 mfma16(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ doublex4 mfma16(double a, double b, doublex4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Omega[i, r] and Omega[i, r + 1] for even r (one Box-Muller pair).
__device__ __forceinline__ void omega_pair(uint64_t i, uint32_t r, uint32_t tag, uint64_t seed,
                                           float& z0, float& z1) {
  const Words4 b = philox_at(i, tag, r >> 2, seed);
  const bool second = (r >> 1) & 1u;
  const uint32_t wu = second ? b.w[2] : b.w[0];
  const uint32_t wv = second ? b.w[3] : b.w[1];
  const float u = (float)((wu >> 8) + 1u) * 0x1p-24f;
  const float v = (float)(wv >> 8) * 0x1p-24f;
  const float rad = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u));
  z0 = rad * __builtin_amdgcn_cosf(v);
  z1 = rad * __builtin_amdgcn_sinf(v);
}
__device__ __forceinline__ void omega_pair(uint64_t i, uint32_t r, uint32_t tag, uint64_t seed,
                                           double& z0, double& z1) {
  double z[2];
  gauss2_f64(i, r >> 1, tag, seed, z);
  z0 = z[0];
  z1 = z[1];
}

template <typename T, int NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void gauss_sketch_kernel(
    const T* __restrict__ A, int64_t lda, const T* __restrict__ bcol, int n, int ncols,
    int64_t m, int s, int64_t kchunk, uint32_t tag, uint64_t seed, T* __restrict__ partials) {
  using Cfg = GaussCfg<T>;
  using acc_t = typename Cfg::acc_t;
  constexpr int KS = Cfg::KS;
  constexpr int LDT = Cfg::LDT;
  constexpr int NCOL = NT * 16;              // columns of the tile
  constexpr int GROUPS = NCOL * (KS / 4);    // 4-row groups per stage
  constexpr int GPT = (GROUPS + 255) / 256;  // groups per thread
  constexpr bool TWO = sizeof(T) == 4;
  __shared__ T tile[2][NCOL * LDT];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int mi = lane & 15;
  const int kk = lane >> 4;
  const int m0 = blockIdx.x * 128 + wave * 32;
  const int nbase = blockIdx.y * NCOL;
  const int sp = blockIdx.z;
  const int64_t k0 = (int64_t)sp * kchunk;
  int64_t k1 = k0 + kchunk;
  if (k1 > m) k1 = m;
  const uint32_t rpair = (uint32_t)(m0 + 2 * mi);  // even sketch row of this lane's pair
  const bool rvalid = (int)rpair < s;             // s is even or rpair + 1 == s is masked below
  const bool r1valid = (int)rpair + 1 < s;

  acc_t acc[2][NT], out[2][NT];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      acc[t][q] = acc_t{0, 0, 0, 0};
      out[t][q] = acc_t{0, 0, 0, 0};
    }

  T stage_v[GPT][4];
  auto load_stage = [&](int64_t r0) {
#pragma unroll
    for (int g = 0; g < GPT; ++g) {
      const int gi = tid + 256 * g;
      const int jc = gi / (KS / 4);
      const int rg = gi - jc * (KS / 4);
      const int64_t j = nbase + jc;
      const int64_t row = r0 + 4 * rg;
#pragma unroll
      for (int e = 0; e < 4; ++e) stage_v[g][e] = T(0);
      if (gi < GROUPS && j < ncols) {
        const T* col = j < n ? A + j * lda : bcol;
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (row + e < k1) stage_v[g][e] = col[row + e];
      }
    }
  };
  auto store_stage = [&](int b) {
#pragma unroll
    for (int g = 0; g < GPT; ++g) {
      const int gi = tid + 256 * g;
      if (gi < GROUPS) {
        const int jc = gi / (KS / 4);
        const int rg = gi - jc * (KS / 4);
#pragma unroll
        for (int e = 0; e < 4; ++e) tile[b][jc * LDT + 4 * rg + e] = stage_v[g][e];
      }
    }
  };

  const int64_t nst = (k1 - k0 + KS - 1) / KS;
  if (nst > 0) {
    load_stage(k0);
    store_stage(0);
  }
  __syncthreads();
  for (int64_t st = 0; st < nst; ++st) {
    const int b = (int)(st & 1);
    const int64_t r0 = k0 + st * KS;
    if (st + 1 < nst) load_stage(r0 + KS);
#pragma unroll 2
    for (int ks = 0; ks < KS / 4; ++ks) {
      const int64_t i = r0 + 4 * ks + kk;
      T a0 = T(0), a1 = T(0);
      if (i < k1 && rvalid) {
        omega_pair((uint64_t)i, rpair, tag, seed, a0, a1);
        if (!r1valid) a1 = T(0);
      }
      const T* tb = &tile[b][mi * LDT + 4 * ks + kk];
#pragma unroll
      for (int q = 0; q < NT; ++q) {
        const T bv = tb[q * 16 * LDT];
        acc[0][q] = mfma16(a0, bv, acc[0][q]);
        acc[1][q] = mfma16(a1, bv, acc[1][q]);
      }
    }
    if (TWO && (((st + 1) * KS) % 4096 == 0)) {
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int q = 0; q < NT; ++q) {
          out[t][q] += acc[t][q];
          acc[t][q] = acc_t{0, 0, 0, 0};
        }
    }
    if (st + 1 < nst) store_stage(b ^ 1);
    __syncthreads();
  }
  // lane holds D[row][lane & 15] of each 16x16 tile with row = 4 (lane >> 4) + v for
  // the fp32 MFMA and row = (lane >> 4) + 4 v for the fp64 MFMA
  T* dst = partials + (int64_t)sp * ncols * s;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      const acc_t tot = out[t][q] + acc[t][q];
      const int64_t j = nbase + q * 16 + mi;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = sizeof(T) == 4 ? 4 * kk + v : kk + 4 * v;
        const int r = m0 + 2 * row + t;
        if (j < ncols && r < s) dst[j * s + r] = tot[v];
      }
    }
}

template <typename T>
__global__ void splitk_reduce_kernel(const T* __restrict__ partials, int splits, int64_t plane,
                                     double scale, int s, T* __restrict__ C, int64_t ldc) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (r >= s) return;
  double acc = 0.0;
  for (int p = 0; p < splits; ++p) acc += (double)partials[p * plane + j * s + r];
  C[r + j * ldc] = (T)(acc * scale);
}

namespace {

struct GaussShape {
  int NT;
  int ntiles;
  int mtiles;
  int splits;
  int64_t kchunk;
};

template <typename T>
GaussShape gauss_shape(const rmm_ctx* h, int64_t m, int ncols, int s) {
  GaussShape g;
  g.NT = ncols > 128 ? 17 : ncols > 64 ? 8 : ncols > 16 ? 4 : 1;
  g.ntiles = (ncols + g.NT * 16 - 1) / (g.NT * 16);
  g.mtiles = (s + 127) / 128;
  const int64_t KS = GaussCfg<T>::KS;
  // enough K splits for about two workgroups per CU, at least 4096 rows each
  int64_t want = (2ll * h->cus + (int64_t)g.mtiles * g.ntiles - 1) / ((int64_t)g.mtiles * g.ntiles);
  int64_t maxsplit = (m + 4095) / 4096;
  if (want > maxsplit) want = maxsplit;
  if (want < 1) want = 1;
  int64_t kc = (m + want - 1) / want;
  kc = (kc + KS - 1) / KS * KS;
  if (kc < KS) kc = KS;
  g.kchunk = kc;
  g.splits = (int)((m + kc - 1) / kc);
  if (g.splits < 1) g.splits = 1;
  return g;
}

template <typename T, int NT>
int launch_gauss(const rmm_ctx* h, const GaussShape& g, const T* A, int64_t lda, const T* b,
                 int n, int ncols, int64_t m, int s, uint32_t tag, uint64_t seed, T* partials) {
  dim3 grid((unsigned)g.mtiles, (unsigned)g.ntiles, (unsigned)g.splits);
  hipLaunchKernelGGL((gauss_sketch_kernel<T, NT>), grid, dim3(256), 0, h->stream, A, lda, b, n,
                     ncols, m, s, g.kchunk, tag, seed, partials);
  return launch_status();
}

}  // namespace

template <typename T>
size_t gauss_sketch_workspace(const rmm_ctx* h, int64_t m, int ncols, int64_t s) {
  const GaussShape g = gauss_shape<T>(h, m, ncols, (int)s);
  Carver c(nullptr, 0);
  c.take<T>((size_t)g.splits * ncols * s);
  return c.off;
}

// Y (s x ncols) = Omega^T [A | b] * scale with Omega of stream `tag`.
template <typename T>
int gauss_project(rmm_ctx* h, int64_t m, int n, const T* A, int64_t lda, const T* b,
                  int64_t s, uint32_t tag, uint64_t seed, double scale, T* C, int64_t ldc,
                  Carver& ws) {
  const int ncols = n + (b ? 1 : 0);
  if (ncols == 0) return RMM_OK;
  if (m == 0) return launch_fill_zero<T>(C, s, ncols, ldc, h->stream);
  const GaussShape g = gauss_shape<T>(h, m, ncols, (int)s);
  T* partials = ws.take<T>((size_t)g.splits * ncols * s);
  if (!ws.fits()) return RMM_ERR_WORKSPACE_TOO_SMALL;
  int rc;
  switch (g.NT) {
    case 17: rc = launch_gauss<T, 17>(h, g, A, lda, b, n, ncols, m, (int)s, tag, seed, partials); break;
    case 8: rc = launch_gauss<T, 8>(h, g, A, lda, b, n, ncols, m, (int)s, tag, seed, partials); break;
    case 4: rc = launch_gauss<T, 4>(h, g, A, lda, b, n, ncols, m, (int)s, tag, seed, partials); break;
    default: rc = launch_gauss<T, 1>(h, g, A, lda, b, n, ncols, m, (int)s, tag, seed, partials); break;
  }
  RMM_TRY(rc);
  dim3 grid((unsigned)((s + 255) / 256), (unsigned)ncols);
  hipLaunchKernelGGL(splitk_reduce_kernel<T>, grid, dim3(256), 0, h->stream, partials, g.splits,
                     (int64_t)ncols * s, scale, (int)s, C, ldc);
  return launch_status();
}

template <typename T>
int gauss_sketch_run(rmm_ctx* h, int64_t m, int n, const T* A, int64_t lda, const T* b,
                     int64_t s, uint64_t seed, T* C, int64_t ldc, Carver& ws) {
  return gauss_project<T>(h, m, n, A, lda, b, s, TAG_GAUSS_SKETCH, seed, 1.0 / sqrt((double)s), C,
                          ldc, ws);
}

template size_t gauss_sketch_workspace<float>(const rmm_ctx*, int64_t, int, int64_t);
template size_t gauss_sketch_workspace<double>(const rmm_ctx*, int64_t, int, int64_t);
template int gauss_sketch_run<float>(rmm_ctx*, int64_t, int, const float*, int64_t, const float*,
                                     int64_t, uint64_t, float*, int64_t, Carver&);
template int gauss_sketch_run<double>(rmm_ctx*, int64_t, int, const double*, int64_t,
                                      const double*, int64_t, uint64_t, double*, int64_t, Carver&);
template int gauss_project<float>(rmm_ctx*, int64_t, int, const float*, int64_t, const float*,
                                  int64_t, uint32_t, uint64_t, double, float*, int64_t, Carver&);
template int gauss_project<double>(rmm_ctx*, int64_t, int, const double*, int64_t, const double*,
                                   int64_t, uint32_t, uint64_t, double, double*, int64_t, Carver&);

}  // namespace rmm
