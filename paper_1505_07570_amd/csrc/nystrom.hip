// Nystrom approximation of an RBF kernel matrix (Sec. 6.4, kernel of Sec. 6.1.1).
//
//   K_ij = exp(-||x_i - x_j||^2 / (2 sigma^2)),  x_i = row i of X (n x d).
//   S = c sorted indices drawn uniformly without replacement from [0, n);
//   C = K[:, S] (n x c, fp32), W = K[S, S] (c x c, fp64),
//   W = U Lam U^T, L = C U_k Lam_k^{-1/2}  so that  K ~ L L^T = C W_k^+ C^T.
//
// The kernel matrix is never formed: C is computed tile by tile from X.  The
// squared distances are formed from the differences (not from the expanded
// inner products, which cancel in fp32).  W is computed in fp64 from the same
// fp32 points, so that its eigendecomposition does not see C's rounding.
#include "common.hpp"
#include "dense.hpp"
#include "ops.hpp"
#include "rng.hpp"

namespace rmm {

constexpr int kRbfRows = 256;  // rows of C per workgroup (one per thread)
constexpr int kRbfCols = 32;   // columns of C per LDS stage
constexpr int kRbfMaxD = 64;   // point dimension held in registers

// C[i + j * ldc] = exp(-||x_i - x_{S_j}||^2 * g), g = 1 / (2 sigma^2).
// Thread = one row i.  The workgroup's 256 points sit in LDS (rows padded to
// D + 1 floats: conflict-free per-thread reads) and the workgroup walks over
// all c columns in stages of kRbfCols sampled points, stored coordinate-major
// so that one broadcast 16-byte LDS read serves four columns.  Writes are
// coalesced along i.  blockIdx.y takes columns [cpg y, cpg (y + 1)) (cpg a
// multiple of kRbfCols), so that short, wide blocks of K still give many
// workgroups.
// Column j is point idx[j] of Y, or point col_base + j when idx is null.
template <int D>
__global__ __launch_bounds__(kRbfRows) void rbf_columns_kernel(int64_t n, int d, const float* __restrict__ X,
                                                               int64_t ldx, int c, const int64_t* __restrict__ idx,
                                                               const float* __restrict__ Y, int64_t ldy,
                                                               int64_t col_base,
                                                               float g, float* __restrict__ C, int64_t ldc,
                                                               int cpg) {
  __shared__ __align__(16) float ys[D][kRbfCols];
  __shared__ float xs[kRbfRows][D + 1];
  const int64_t r0 = (int64_t)blockIdx.x * kRbfRows;
  const int64_t i = r0 + threadIdx.x;
  for (int e = threadIdx.x; e < kRbfRows * D; e += kRbfRows) {
    const int r = e / D, k = e % D;
    xs[r][k] = (r0 + r < n && k < d) ? X[(r0 + r) * ldx + k] : 0.0f;
  }
  const int jb = blockIdx.y * cpg;
  const int je = jb + cpg < c ? jb + cpg : c;
  for (int j0 = jb; j0 < je; j0 += kRbfCols) {
    __syncthreads();
    for (int e = threadIdx.x; e < kRbfCols * D; e += kRbfRows) {
      const int jj = e / D, k = e % D;
      const int j = j0 + jj;
      const int64_t pt = idx ? idx[j < je ? j : jb] : col_base + j;  // sampled or contiguous points
      ys[k][jj] = (j < je && k < d) ? Y[pt * ldy + k] : 0.0f;
    }
    __syncthreads();
    const int jn = (je - j0) < kRbfCols ? (je - j0) : kRbfCols;
    if (i >= n) continue;
    float acc[kRbfCols];
#pragma unroll
    for (int q = 0; q < kRbfCols; ++q) acc[q] = 0.0f;
#pragma unroll 2
    for (int k = 0; k < d; ++k) {
      const float xk = xs[threadIdx.x][k];
#pragma unroll
      for (int q = 0; q < kRbfCols; q += 4) {
        const float4 y = *reinterpret_cast<const float4*>(&ys[k][q]);
        float t = xk - y.x;
        acc[q] = fmaf(t, t, acc[q]);
        t = xk - y.y;
        acc[q + 1] = fmaf(t, t, acc[q + 1]);
        t = xk - y.z;
        acc[q + 2] = fmaf(t, t, acc[q + 2]);
        t = xk - y.w;
        acc[q + 3] = fmaf(t, t, acc[q + 3]);
      }
    }
#pragma unroll
    for (int q = 0; q < kRbfCols; ++q)
      if (q < jn) C[i + (int64_t)(j0 + q) * ldc] = expf(-acc[q] * g);
  }
}

// W[a + b * c] = exp(-||x_{S_a} - x_{S_b}||^2 / (2 sigma^2)) in fp64.
__global__ void rbf_gram_f64_kernel(int d, const float* __restrict__ X, int64_t ldx, int c,
                                    const int64_t* __restrict__ idx, double g, double* __restrict__ W) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (a >= c) return;
  const float* xa = X + idx[a] * ldx;
  const float* xb = X + idx[b] * ldx;
  double acc = 0.0;
  for (int k = 0; k < d; ++k) {
    const double t = (double)xa[k] - (double)xb[k];
    acc = fma(t, t, acc);
  }
  W[a + (int64_t)b * c] = exp(-acc * g);
}

// F[:, t] = V[:, t] / sqrt(lam_t) for lam_t > c * eps * lam_0, else 0 (t < k).
// F = U_k Lam_k^{-1/2} formed in FP64 and rounded once to FP32 for the
// product L = C F (C is FP32 already).
__global__ void nystrom_scale_kernel(int c, int k, const double* __restrict__ lam,
                                     const double* __restrict__ V, float* __restrict__ F) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  if (a >= c) return;
  const double cut = (double)c * 0x1p-52 * lam[0];
  const double l = lam[t];
  F[a + (int64_t)t * c] = (float)((l > cut && l > 0.0) ? V[a + (int64_t)t * c] / sqrt(l) : 0.0);
}

int launch_rbf(const rmm_ctx* h, int64_t n, int d, const float* X, int64_t ldx, int c,
               const int64_t* idx, const float* Y, int64_t ldy, int64_t col_base, double g, float* C,
               int64_t ldc) {
  if (n == 0 || c == 0) return RMM_OK;
  const unsigned blocks = (unsigned)((n + kRbfRows - 1) / kRbfRows);
  // column groups: at least 4 workgroups per CU in all
  const int stages = (c + kRbfCols - 1) / kRbfCols;
  int64_t gy = (4 * (int64_t)h->cus + blocks - 1) / blocks;
  if (gy > stages) gy = stages;
  if (gy < 1) gy = 1;
  const int cpg = (int)((stages + gy - 1) / gy) * kRbfCols;
  gy = (c + cpg - 1) / cpg;
  const dim3 grid(blocks, (unsigned)gy);
  if (d <= 32)
    hipLaunchKernelGGL(rbf_columns_kernel<32>, grid, dim3(kRbfRows), 0, h->stream, n, d, X, ldx, c, idx, Y,
                       ldy, col_base, (float)g, C, ldc, cpg);
  else
    hipLaunchKernelGGL(rbf_columns_kernel<kRbfMaxD>, grid, dim3(kRbfRows), 0, h->stream, n, d, X, ldx, c,
                       idx, Y, ldy, col_base, (float)g, C, ldc, cpg);
  return launch_status();
}

namespace {

struct NysBufs {
  double* W;
  double* V;
  float* F;
};

size_t nystrom_layout(const rmm_ctx* h, int64_t n, int c, int k, Carver& ws, NysBufs* b) {
  double* W = ws.take<double>((size_t)c * c);
  double* V = ws.take<double>((size_t)c * c);
  float* F = ws.take<float>((size_t)c * k);
  if (b) *b = NysBufs{W, V, F};
  size_t scratch = jacobi_workspace(c);
  const size_t g = gemm_workspace<float>(h, (int)n, k, c);
  if (g > scratch) scratch = g;
  return ws.off + scratch + 4 * kAlign;
}

}  // namespace

size_t nystrom_workspace(const rmm_ctx* h, int64_t n, int c, int k) {
  Carver ws(nullptr, 0);
  return nystrom_layout(h, n, c, k, ws, nullptr);
}

int nystrom_run(rmm_ctx* h, int64_t n, int d, const float* X, int64_t ldx, double sigma, int c,
                int k, uint64_t seed, int64_t* idx, float* C, int64_t ldc, float* L, int64_t ldl,
                double* evals, int32_t* status) {
  Carver ws(h->ws, h->ws_bytes);
  NysBufs b;
  const size_t need = nystrom_layout(h, n, c, k, ws, &b);
  if (need > h->ws_bytes) return RMM_ERR_WORKSPACE_TOO_SMALL;
  RMM_TRY(zero_status(h, status));
  RMM_TRY(launch_sample_indices_i64(h, (uint64_t)n, ceil_log2((uint64_t)n), c, TAG_NYSTROM_SAMPLE,
                                    seed, idx));
  const double g = 1.0 / (2.0 * sigma * sigma);
  RMM_TRY(launch_rbf(h, n, d, X, ldx, c, idx, X, ldx, 0, g, C, ldc));
  hipLaunchKernelGGL(rbf_gram_f64_kernel, dim3((unsigned)((c + 127) / 128), (unsigned)c), dim3(128), 0,
                     h->stream, d, X, ldx, c, idx, g, b.W);
  RMM_TRY(launch_status());
  RMM_TRY(jacobi_eig(h, c, b.W, c, evals, b.V, status, ws));
  hipLaunchKernelGGL(nystrom_scale_kernel, dim3((unsigned)((c + 127) / 128), (unsigned)k), dim3(128), 0,
                     h->stream, c, k, evals, b.V, b.F);
  RMM_TRY(launch_status());
  return gemm<float, float, float, float>(h, false, false, (int)n, k, c, C, ldc, b.F, c, 1.0, L, ldl,
                                            ws);
}

// ---- Gaussian-projection variant: C = K Omega, W = Omega^T C ----------------------------
//
// K (n x n) exists only as blocks of at most kKCols x kKRows entries, written
// by the RBF kernel into the workspace and multiplied into C with
// accumulation: C[rows, :] += K[rows, cols] Omega[cols, :], computed as the
// transposed product (K[cols, rows])^T Omega[cols, :] of the sketch kernel
// with a stored left operand (its 128 x 256 tiles and 32 x 32 MFMAs run
// closer to the FP32 MFMA rate than the plain GEMM on this shape; K is
// symmetric, and its block K[cols, rows] holds the same values bit for bit,
// the squared differences being symmetric).  Omega (n x c fp32, stream tag
// 7) is generated once into the workspace.
constexpr int64_t kKRows = 32768;
constexpr int64_t kKCols = 8192;

namespace {

size_t nystrom_gauss_layout(const rmm_ctx* h, int64_t n, int c, int k, Carver& ws, float** Om,
                            float** Kt, NysBufs* b) {
  const int64_t br = n < kKRows ? n : kKRows, bc = n < kKCols ? n : kKCols;
  float* o = ws.take<float>((size_t)n * c);
  float* kt = ws.take<float>((size_t)br * bc);
  double* W = ws.take<double>((size_t)c * c);
  double* V = ws.take<double>((size_t)c * c);
  float* F = ws.take<float>((size_t)c * k);
  if (Om) *Om = o;
  if (Kt) *Kt = kt;
  if (b) *b = NysBufs{W, V, F};
  size_t scratch = jacobi_workspace(c);
  scratch = scratch > gemm_workspace<float>(h, (int)n, k, c) ? scratch : gemm_workspace<float>(h, (int)n, k, c);
  const size_t g1 = gauss_sketch_workspace<float>(h, bc, (int)br, c);
  const size_t g2 = gemm_workspace<double>(h, c, c, n);
  scratch = scratch > g1 ? scratch : g1;
  scratch = scratch > g2 ? scratch : g2;
  return ws.off + scratch + 4 * kAlign;
}

}  // namespace

size_t nystrom_gauss_workspace(const rmm_ctx* h, int64_t n, int c, int k) {
  Carver ws(nullptr, 0);
  return nystrom_gauss_layout(h, n, c, k, ws, nullptr, nullptr, nullptr);
}

int nystrom_gauss_run(rmm_ctx* h, int64_t n, int d, const float* X, int64_t ldx, double sigma, int c,
                      int k, uint64_t seed, float* C, int64_t ldc, float* L, int64_t ldl, double* evals,
                      int32_t* status) {
  Carver ws(h->ws, h->ws_bytes);
  NysBufs b;
  float *Om, *Kt;
  const size_t need = nystrom_gauss_layout(h, n, c, k, ws, &Om, &Kt, &b);
  if (need > h->ws_bytes) return RMM_ERR_WORKSPACE_TOO_SMALL;
  RMM_TRY(zero_status(h, status));
  RMM_TRY(launch_gaussian<float>(h, TAG_GAUSS_NYSTROM, n, c, seed, Om, n));
  const double g = 1.0 / (2.0 * sigma * sigma);
  const int64_t br = n < kKRows ? n : kKRows, bc = n < kKCols ? n : kKCols;
  for (int64_t i0 = 0; i0 < n; i0 += br) {
    const int64_t rows = (n - i0) < br ? (n - i0) : br;
    for (int64_t l0 = 0; l0 < n; l0 += bc) {
      const int64_t cols = (n - l0) < bc ? (n - l0) : bc;
      // K[l0:l0+cols, i0:i0+rows] (cols x rows, ld cols)
      RMM_TRY(launch_rbf(h, cols, d, X + l0 * ldx, ldx, (int)rows, nullptr, X, ldx, i0, g, Kt, cols));
      // C[i0:, :] (+)= K[l0:, i0:]^T Omega[l0:l0+cols, :]
      RMM_TRY(project_tn<float>(h, cols, (int)rows, Kt, cols, Om + l0, n, c, C + i0, ldc, ws,
                                l0 == 0 ? 0.0 : 1.0));
    }
  }
  // W = Omega^T C (c x c, fp64)
  RMM_TRY((gemm<float, float, double, double>(h, true, false, c, c, n, Om, n, C, ldc, 1.0, b.W, c, ws)));
  RMM_TRY(jacobi_eig(h, c, b.W, c, evals, b.V, status, ws));
  hipLaunchKernelGGL(nystrom_scale_kernel, dim3((unsigned)((c + 127) / 128), (unsigned)k), dim3(128), 0,
                     h->stream, c, k, evals, b.V, b.F);
  RMM_TRY(launch_status());
  return gemm<float, float, float, float>(h, false, false, (int)n, k, c, C, ldc, b.F, c, 1.0, L, ldl,
                                            ws);
}

}  // namespace rmm

using namespace rmm;

namespace {

int nystrom_args(rmm_handle h, int64_t n, int64_t d, int64_t c, int64_t k, double sigma) {
  if (!h || n < 1 || d < 1 || c < 1 || c > n || k < 1 || k > c || !(sigma > 0.0) ||
      !(sigma < 1e300))
    return RMM_ERR_INVALID_ARG;
  if (d > kRbfMaxD || c > 1024 || n >= (1ll << 31)) return RMM_ERR_UNSUPPORTED;
  return RMM_OK;
}

}  // namespace

extern "C" {

int rmm_nystrom_workspace(rmm_handle h, int64_t n, int64_t d, int64_t c, int64_t k,
                          size_t* bytes) {
  RMM_TRY(nystrom_args(h, n, d, c, k, 1.0));
  if (!bytes) return RMM_ERR_INVALID_ARG;
  *bytes = nystrom_workspace(h, n, (int)c, (int)k);
  return RMM_OK;
}

int rmm_nystrom(rmm_handle h, int64_t n, int64_t d, const float* X, int64_t ldx, double sigma,
                int64_t c, int64_t k, uint64_t seed, int64_t* idx, float* C, int64_t ldc, float* L,
                int64_t ldl, double* evals, int32_t* status) {
  RMM_TRY(nystrom_args(h, n, d, c, k, sigma));
  if (!X || !idx || !C || !L || !evals || ldx < d || ldc < n || ldl < n) return RMM_ERR_INVALID_ARG;
  return nystrom_run(h, n, (int)d, X, ldx, sigma, (int)c, (int)k, seed, idx, C, ldc, L, ldl, evals,
                     status);
}

int rmm_nystrom_gaussian_workspace(rmm_handle h, int64_t n, int64_t d, int64_t c, int64_t k,
                                   size_t* bytes) {
  RMM_TRY(nystrom_args(h, n, d, c, k, 1.0));
  if (!bytes) return RMM_ERR_INVALID_ARG;
  *bytes = nystrom_gauss_workspace(h, n, (int)c, (int)k);
  return RMM_OK;
}

int rmm_nystrom_gaussian(rmm_handle h, int64_t n, int64_t d, const float* X, int64_t ldx,
                         double sigma, int64_t c, int64_t k, uint64_t seed, float* C, int64_t ldc,
                         float* L, int64_t ldl, double* evals, int32_t* status) {
  RMM_TRY(nystrom_args(h, n, d, c, k, sigma));
  if (!X || !C || !L || !evals || ldx < d || ldc < n || ldl < n) return RMM_ERR_INVALID_ARG;
  return nystrom_gauss_run(h, n, (int)d, X, ldx, sigma, (int)c, (int)k, seed, C, ldc, L, ldl, evals,
                           status);
}

}  // extern "C"
