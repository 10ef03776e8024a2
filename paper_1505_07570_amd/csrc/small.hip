// Small FP64 factorizations that run in a single workgroup: the Cholesky
// step of CholeskyQR2 with the triangular inverse, and the cyclic Jacobi
// eigensolver used for the small SVD of the projected matrix.  These sit on
// the latency path of every driver call; the matrices are at most 128 x 128
// in LDS (larger Cholesky factors are worked on in global memory).
#include "common.hpp"
#include "dense.hpp"

namespace rmm {

constexpr int kSmallThreads = 1024;
constexpr int kLdsMaxL = 128;

__device__ __forceinline__ void or_status(int32_t* status, int32_t flag) {
  if (status) atomicOr(status, flag);
}

// W: l x l column-major working array (ld = l) holding G on entry (upper
// triangle read).  Elimination of [G | I] without row scaling: step j
// subtracts W[j][i] / p_j times row j from every row i > j, where p_j is the
// j-th pivot.  Afterwards the upper triangle holds D L~^T (G = L~ D L~^T,
// L~ unit lower triangular), the strict lower triangle holds L~^{-1}, and
//   R = D^{1/2} L~^T,   R^{-1}[c][j] = L~^{-1}[j][c] / sqrt(p_j)   (c <= j).
// One barrier per step: row j is final before step j and is only read.
// The drop test of pivot j compares against orig[j * ostride] (the diagonal
// of the matrix the caller considers original), or G_jj when orig is null;
// a dropped pivot eliminates nothing and gives a zero column of R^{-1}.
__device__ void cholinv_body(int l, double* W, int ldw, double tau, const double* orig,
                             int64_t ostride, double* __restrict__ Rinv, int64_t ldr,
                             double* __restrict__ diag, int32_t* status, double* sh_orig,
                             double* sh_piv) {
  // blockDim.x == 1024, l <= 128: thread = (column c, row phase i0)
  const int tid = threadIdx.x;
  const int c = tid & 127;
  const int i0 = tid >> 7;
  if (tid < l) sh_orig[tid] = orig ? orig[tid * ostride] : W[tid + tid * ldw];
  if (c < l)
    for (int i = i0; i < l; i += 8)
      if (c < i) W[i + c * ldw] = 0.0;  // strict lower triangle: L~^{-1} below its unit diagonal
  __syncthreads();
  for (int j = 0; j < l; ++j) {
    const double p = W[j + j * ldw];
    const bool keep = p > tau * sh_orig[j] && p > 1e-300;
    if (tid == 0) {
      sh_piv[j] = keep ? p : 0.0;
      if (!keep) or_status(status, RMM_STATUS_QR_FALLBACK);
    }
    if (keep && c < l) {
      const double inv = 1.0 / p;
      const double wjc = W[j + c * ldw];
      const double lj = (c == j) ? 1.0 : wjc;  // L~^{-1}[j][c] for c <= j
      for (int i = i0; i < l; i += 8) {
        if (i <= j) continue;
        const double f = W[j + i * ldw] * inv;  // W[j][i] / p_j
        if (c >= i) W[i + c * ldw] -= f * wjc;   // Schur complement (upper)
        else if (c <= j) W[i + c * ldw] -= f * lj;
      }
    }
    __syncthreads();
  }
  if (c < l) {
    for (int j = i0; j < l; j += 8) {  // Rinv[c][j]
      const double pj = sh_piv[j];
      double v = 0.0;
      if (pj > 0.0 && c <= j) v = ((c == j) ? 1.0 : W[j + c * ldw]) / sqrt(pj);
      Rinv[c + (int64_t)j * ldr] = v;
    }
  }
  if (tid < l) diag[tid] = sqrt(sh_piv[tid]);
}

__global__ __launch_bounds__(kSmallThreads) void cholinv_lds_kernel(
    int l, const double* __restrict__ G, int64_t ldg, double tau, const double* orig,
    int64_t ostride, double* __restrict__ Rinv, int64_t ldr, double* __restrict__ diag,
    int32_t* status) {
  extern __shared__ double W[];  // l x (l + 1) (padded), then 2 l
  const int ldw = l + 1;           // odd stride: rows of W spread over the LDS banks
  double* sorig = W + (size_t)l * ldw;
  double* piv = sorig + l;
  const int c = threadIdx.x & 127;
  if (c < l)
    for (int i = threadIdx.x >> 7; i < l; i += 8) W[i + c * ldw] = G[i + (int64_t)c * ldg];
  __syncthreads();
  cholinv_body(l, W, ldw, tau, orig, ostride, Rinv, ldr, diag, status, sorig, piv);
}

__global__ void fill_block_kernel(int rows, double* __restrict__ X, int64_t ldx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < rows) X[i + (int64_t)blockIdx.y * ldx] = 0.0;
}

__global__ void copy_block_kernel(int rows, const double* __restrict__ X, int64_t ldx,
                                  double* __restrict__ Y, int64_t ldy) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < rows) Y[i + (int64_t)blockIdx.y * ldy] = X[i + (int64_t)blockIdx.y * ldx];
}

size_t cholinv_workspace(const rmm_ctx* h, int l) {
  if (l <= kLdsMaxL) return 0;
  const int l1 = (l + 1) / 2, l2 = l - l1;
  Carver c(nullptr, 0);
  c.take<double>((size_t)l1 * l2);  // R12
  c.take<double>((size_t)l2 * l2);  // S
  c.take<double>((size_t)l1 * l2);  // T2
  size_t w = gemm_workspace<double>(h, l1, l2, l1);
  const size_t w2 = gemm_workspace<double>(h, l2, l2, l1);
  const size_t w3 = gemm_workspace<double>(h, l1, l2, l2);
  const size_t w4 = cholinv_workspace(h, l1);
  const size_t w5 = cholinv_workspace(h, l2);
  w = w2 > w ? w2 : w;
  w = w3 > w ? w3 : w;
  w = w4 > w ? w4 : w;
  w = w5 > w ? w5 : w;
  return c.off + w + 4 * kAlign;
}

// Recursive 2 x 2 blocking above the LDS size:
//   G = [[G11, G12], [G12^T, G22]] = R^T R,  R = [[R11, R12], [0, R22]]
//   R11 = chol(G11), R12 = R11^{-T} G12, R22 = chol(G22 - R12^T R12)
//   R^{-1} = [[X11, -X11 R12 X22], [0, X22]],  X = R^{-1} of each block.
static int cholinv_rec(rmm_ctx* h, int l, const double* G, int64_t ldg, double tau,
                       const double* orig, int64_t ostride, double* Rinv, int64_t ldr, double* diag,
                       int32_t* status, Carver& ws) {
  if (l <= kLdsMaxL) {
    const size_t lds = ((size_t)l * (l + 1) + 2 * (size_t)l) * sizeof(double);
    RMM_HIP(hipFuncSetAttribute((const void*)cholinv_lds_kernel,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(cholinv_lds_kernel, dim3(1), dim3(kSmallThreads), lds, h->stream, l, G, ldg,
                       tau, orig, ostride, Rinv, ldr, diag, status);
    return launch_status();
  }
  const int l1 = (l + 1) / 2, l2 = l - l1;
  const size_t mark = ws.off;
  double* R12 = ws.take<double>((size_t)l1 * l2);
  double* S = ws.take<double>((size_t)l2 * l2);
  double* T2 = ws.take<double>((size_t)l1 * l2);
  if (!ws.fits()) return RMM_ERR_WORKSPACE_TOO_SMALL;
  const double* o = orig ? orig : G;
  const int64_t os = orig ? ostride : ldg + 1;
  const double* G12 = G + (int64_t)l1 * ldg;
  const double* G22 = G + l1 + (int64_t)l1 * ldg;
  double* X11 = Rinv;
  double* X12 = Rinv + (int64_t)l1 * ldr;
  double* X21 = Rinv + l1;
  double* X22 = Rinv + l1 + (int64_t)l1 * ldr;
  RMM_TRY(cholinv_rec(h, l1, G, ldg, tau, o, os, X11, ldr, diag, status, ws));
  RMM_TRY((gemm<double, double, double, double>(h, true, false, l1, l2, l1, X11, ldr, G12, ldg, 1.0,
                                                R12, l1, ws)));
  hipLaunchKernelGGL(copy_block_kernel, dim3((l2 + 255) / 256, l2), dim3(256), 0, h->stream, l2, G22,
                     ldg, S, l2);
  RMM_TRY(launch_status());
  RMM_TRY((gemm<double, double, double, double>(h, true, false, l2, l2, l1, R12, l1, R12, l1, -1.0, S,
                                                l2, ws, 1.0)));
  RMM_TRY(cholinv_rec(h, l2, S, l2, tau, o + (int64_t)l1 * os, os, X22, ldr, diag + l1, status, ws));
  RMM_TRY((gemm<double, double, double, double>(h, false, false, l1, l2, l2, R12, l1, X22, ldr, 1.0,
                                                T2, l1, ws)));
  RMM_TRY((gemm<double, double, double, double>(h, false, false, l1, l2, l1, X11, ldr, T2, l1, -1.0,
                                                X12, ldr, ws)));
  hipLaunchKernelGGL(fill_block_kernel, dim3((l2 + 255) / 256, l1), dim3(256), 0, h->stream, l2, X21,
                     ldr);
  ws.off = mark;
  return launch_status();
}

int cholinv(rmm_ctx* h, int l, const double* G, int64_t ldg, double tau, double* Rinv,
            double* diag, int32_t* status, Carver& ws) {
  if (l == 0) return RMM_OK;
  return cholinv_rec(h, l, G, ldg, tau, nullptr, 0, Rinv, l, diag, status, ws);
}

// ---- cyclic Jacobi eigensolver ------------------------------------------------------
//
// Parallel (round-robin) ordering: in each of the L-1 rounds of a sweep the
// L/2 disjoint pairs (p, q) of the circle method are rotated at once, first
// the rows (J^T G), then the columns (G J) and the eigenvector columns (V J).
// The rotation zeroing G_pq follows the classical choice
// t = sgn(theta) / (|theta| + sqrt(theta^2 + 1)), theta = (G_qq - G_pp) / (2 G_pq).
__global__ __launch_bounds__(kSmallThreads) void jacobi_kernel(int l, const double* __restrict__ G,
                                                               int64_t ldg, double* __restrict__ evals,
                                                               double* __restrict__ Vout,
                                                               double* __restrict__ Vw,
                                                               int32_t* status, int max_sweeps) {
  extern __shared__ double S[];  // l x (l + 1) (padded), then pair tables
  const int lds = l + 1;
  const int L = (l + 1) & ~1;     // even number of players
  const int npairs = L / 2;
  double* cs = S + (size_t)l * lds;     // npairs
  double* sn = cs + npairs;             // npairs
  int* pp = reinterpret_cast<int*>(sn + npairs);
  int* qq = pp + npairs;
  __shared__ double red[1];
  __shared__ int done;
  const int tid = threadIdx.x;
  // thread = (column / row index k, pair phase i0); l <= 128, 1024 threads
  const int k = tid & 127;
  const int i0 = tid >> 7;
  if (k < l)
    for (int a = i0; a < l; a += 8) {
      S[a + k * lds] = G[a + (int64_t)k * ldg];
      Vw[a + (int64_t)k * l] = (a == k) ? 1.0 : 0.0;
    }
  __syncthreads();
  // scale for the absolute part of the rotation threshold
  if (tid == 0) {
    double mx = 0.0;
    for (int i = 0; i < l; ++i) mx = fmax(mx, fabs(S[i + i * lds]));
    red[0] = mx;
  }
  __syncthreads();
  const double abs_tol = 1e-17 * red[0];
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    // a sweep that rotates nothing ends the iteration
    __syncthreads();
    if (tid == 0) done = 1;
    __syncthreads();
    for (int r = 0; r < L - 1; ++r) {
      if (tid < npairs) {
        const int i = tid;
        const int a = (i == 0) ? 0 : ((i - 1 + r) % (L - 1)) + 1;
        const int b = ((L - 2 - i + r) % (L - 1)) + 1;
        int p = a < b ? a : b, q = a < b ? b : a;
        double c = 1.0, s = 0.0;
        if (q < l) {
          const double gpq = S[p + q * lds];
          const double gpp = S[p + p * lds], gqq = S[q + q * lds];
          if (fabs(gpq) > abs_tol && fabs(gpq) > 0x1p-52 * sqrt(fabs(gpp * gqq))) {
            done = 0;
            const double theta = (gqq - gpp) / (2.0 * gpq);
            const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
          }
        }
        if (s == 0.0) p = -1;
        pp[i] = p;
        qq[i] = q;
        cs[i] = c;
        sn[i] = s;
      }
      __syncthreads();
      // rows: G <- J^T G
      if (k < l)
        for (int i = i0; i < npairs; i += 8) {
          const int p = pp[i];
          if (p < 0) continue;
          const int q = qq[i];
          const double c = cs[i], s = sn[i];
          const double gp = S[p + k * lds], gq = S[q + k * lds];
          S[p + k * lds] = c * gp - s * gq;
          S[q + k * lds] = s * gp + c * gq;
        }
      __syncthreads();
      // columns: G <- G J and V <- V J
      if (k < l)
        for (int i = i0; i < npairs; i += 8) {
          const int p = pp[i];
          if (p < 0) continue;
          const int q = qq[i];
          const double c = cs[i], s = sn[i];
          const double gp = S[k + p * lds], gq = S[k + q * lds];
          S[k + p * lds] = c * gp - s * gq;
          S[k + q * lds] = s * gp + c * gq;
          const double vp = Vw[k + (int64_t)p * l], vq = Vw[k + (int64_t)q * l];
          Vw[k + (int64_t)p * l] = c * vp - s * vq;
          Vw[k + (int64_t)q * l] = s * vp + c * vq;
        }
      __syncthreads();
    }
    if (done) break;
  }
  if (sweep == max_sweeps && tid == 0) or_status(status, RMM_STATUS_NOT_CONVERGED);
  // sort descending (ties by index) and emit
  for (int j = tid; j < l; j += blockDim.x) {
    const double v = S[j + j * lds];
    int rank = 0;
    for (int i = 0; i < l; ++i) {
      const double u = S[i + i * lds];
      rank += (u > v) || (u == v && i < j);
    }
    evals[rank] = v;
    for (int kk = 0; kk < l; ++kk) Vout[kk + (int64_t)rank * l] = Vw[kk + (int64_t)j * l];
  }
}

size_t jacobi_workspace(int l) {
  Carver c(nullptr, 0);
  c.take<double>((size_t)l * l);
  return c.off;
}

int jacobi_eig(const rmm_ctx* h, int l, const double* G, int64_t ldg, double* evals, double* V,
               int32_t* status, Carver& ws) {
  if (l == 0) return RMM_OK;
  if (l > kLdsMaxL) return RMM_ERR_UNSUPPORTED;
  const size_t mark = ws.off;
  double* Vw = ws.take<double>((size_t)l * l);
  if (!ws.fits()) return RMM_ERR_WORKSPACE_TOO_SMALL;
  const int L = (l + 1) & ~1;
  const size_t lds = (size_t)l * (l + 1) * sizeof(double) + (size_t)L * sizeof(double) + (size_t)L * sizeof(int);
  RMM_HIP(hipFuncSetAttribute((const void*)jacobi_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds));
  hipLaunchKernelGGL(jacobi_kernel, dim3(1), dim3(kSmallThreads), lds, h->stream, l, G, ldg, evals, V,
                     Vw, status, 40);
  ws.off = mark;
  return launch_status();
}

// ---- sign convention, small glue -------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void sign_fix_kernel(int64_t m, int64_t n, T* __restrict__ U,
                                                       int64_t ldu, T* __restrict__ V, int64_t ldv) {
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  const int64_t c = blockIdx.x;
  T* u = U + c * ldu;
  double best = -1.0;
  int64_t besti = 0;
  for (int64_t i = threadIdx.x; i < m; i += 256) {
    const double a = fabs((double)u[i]);
    if (a > best) { best = a; besti = i; }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = besti;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      const double o = bv[threadIdx.x + st];
      const int64_t oi = bi[threadIdx.x + st];
      if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
        bv[threadIdx.x] = o;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  const bool flip = (double)u[bi[0]] < 0.0;
  __syncthreads();
  if (!flip) return;
  for (int64_t i = threadIdx.x; i < m; i += 256) u[i] = -u[i];
  T* v = V + c * ldv;
  for (int64_t i = threadIdx.x; i < n; i += 256) v[i] = -v[i];
}

template <typename T>
int sign_fix(const rmm_ctx* h, int64_t m, int64_t n, int k, T* U, int64_t ldu, T* V, int64_t ldv) {
  if (k == 0) return RMM_OK;
  hipLaunchKernelGGL((sign_fix_kernel<T>), dim3(k), dim3(256), 0, h->stream, m, n, U, ldu, V, ldv);
  return launch_status();
}

template <typename T>
__global__ void svd_from_eig_kernel(int l, int k, const double* __restrict__ evals,
                                    const double* __restrict__ Vr, double* __restrict__ W,
                                    T* __restrict__ sigma) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= l * k) return;
  const int a = e % l, c = e / l;
  const double lam = evals[c] > 0.0 ? evals[c] : 0.0;
  const double sg = sqrt(lam);
  W[a + (int64_t)c * l] = sg > 0.0 ? Vr[a + (int64_t)c * l] / sg : 0.0;
  if (a == 0) sigma[c] = (T)sg;
}

template <typename T>
int svd_from_eig(const rmm_ctx* h, int l, int k, const double* evals, const double* Vr, double* W,
                 T* sigma) {
  if (l * k == 0) return RMM_OK;
  hipLaunchKernelGGL((svd_from_eig_kernel<T>), dim3((l * k + 255) / 256), dim3(256), 0, h->stream, l,
                     k, evals, Vr, W, sigma);
  return launch_status();
}

__global__ void rank_check_kernel(int d, const double* __restrict__ d1, const double* __restrict__ d2,
                                  double tol, int32_t* status) {
  __shared__ double mn[256], mx[256];
  double a = 1e308, b = 0.0;
  for (int j = threadIdx.x; j < d; j += 256) {
    const double v = fabs(d1[j] * (d2 ? d2[j] : 1.0));
    a = v < a ? v : a;
    b = v > b ? v : b;
  }
  mn[threadIdx.x] = a;
  mx[threadIdx.x] = b;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      mn[threadIdx.x] = fmin(mn[threadIdx.x], mn[threadIdx.x + st]);
      mx[threadIdx.x] = fmax(mx[threadIdx.x], mx[threadIdx.x + st]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && mn[0] <= tol * mx[0]) or_status(status, RMM_STATUS_RANK_DEFICIENT);
}

int rank_check(const rmm_ctx* h, int d, const double* d1, const double* d2, double tol,
               int32_t* status) {
  hipLaunchKernelGGL(rank_check_kernel, dim3(1), dim3(256), 0, h->stream, d, d1, d2, tol, status);
  return launch_status();
}

__global__ void zero_status_kernel(int32_t* status) { *status = 0; }

int zero_status(const rmm_ctx* h, int32_t* status) {
  if (!status) return RMM_OK;
  hipLaunchKernelGGL(zero_status_kernel, dim3(1), dim3(1), 0, h->stream, status);
  return launch_status();
}

__global__ void trmv_upper_kernel(int d, const double* __restrict__ R, const double* __restrict__ y,
                                  double* __restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d) return;
  double acc = 0.0;
  for (int c = i; c < d; ++c) acc += R[i + (int64_t)c * d] * y[c];
  x[i] = acc;
}

int trmv_upper(const rmm_ctx* h, int d, const double* Rinv, const double* y, double* x) {
  if (d == 0) return RMM_OK;
  hipLaunchKernelGGL(trmv_upper_kernel, dim3((d + 255) / 256), dim3(256), 0, h->stream, d, Rinv, y, x);
  return launch_status();
}

template int sign_fix<float>(const rmm_ctx*, int64_t, int64_t, int, float*, int64_t, float*, int64_t);
template int sign_fix<double>(const rmm_ctx*, int64_t, int64_t, int, double*, int64_t, double*, int64_t);
template int svd_from_eig<float>(const rmm_ctx*, int, int, const double*, const double*, double*, float*);
template int svd_from_eig<double>(const rmm_ctx*, int, int, const double*, const double*, double*, double*);

}  // namespace rmm
