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

// W: l x (l + 1) column-major working array (ld = l).  On entry the upper
// triangle holds G.  On exit: upper triangle = R, strict lower triangle =
// R^{-1} transposed, column l = diag(R^{-1}).
__device__ void cholinv_body(int l, double* W, double tau, double* __restrict__ Rinv,
                             double* __restrict__ diag, int32_t* status, double* sh_orig,
                             double* sh_piv) {
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  for (int j = tid; j < l; j += nt) sh_orig[j] = W[j + (int64_t)j * l];
  __syncthreads();
  // right-looking Cholesky on the upper triangle: G = R^T R
  for (int j = 0; j < l; ++j) {
    if (tid == 0) {
      const double p = W[j + (int64_t)j * l];
      double r = 0.0;
      if (p > tau * sh_orig[j] && p > 1e-300) r = sqrt(p);
      else or_status(status, RMM_STATUS_QR_FALLBACK);
      *sh_piv = r;
      W[j + (int64_t)j * l] = r;
    }
    __syncthreads();
    const double r = *sh_piv;
    const double inv = r > 0.0 ? 1.0 / r : 0.0;
    for (int k = j + 1 + tid; k < l; k += nt) W[j + (int64_t)k * l] *= inv;
    __syncthreads();
    const int w = l - j - 1;
    for (int e = tid; e < w * w; e += nt) {
      const int a = j + 1 + e % w, b = j + 1 + e / w;
      if (a <= b) W[a + (int64_t)b * l] -= W[j + (int64_t)a * l] * W[j + (int64_t)b * l];
    }
    __syncthreads();
  }
  // X = R^{-1} by the column-oriented back substitution of R X = I.
  // X[a][c] (a <= c) is kept at W[c + a l] for a < c and in column l for a == c.
  for (int e = tid; e < l * l; e += nt) {
    const int a = e % l, c = e / l;
    if (a < c) W[c + (int64_t)a * l] = 0.0;
  }
  for (int c = tid; c < l; c += nt) W[c + (int64_t)l * l] = 1.0;
  __syncthreads();
  for (int i = l - 1; i >= 0; --i) {
    const double r = W[i + (int64_t)i * l];
    const double inv = r > 0.0 ? 1.0 / r : 0.0;
    // row i of X is final after scaling
    for (int c = i + tid; c < l; c += nt) {
      if (c == i) W[c + (int64_t)l * l] *= inv;
      else W[c + (int64_t)i * l] *= inv;
    }
    __syncthreads();
    // X[a][c] -= R[a][i] X[i][c] for a < i <= c
    const int w = l - i;
    for (int e = tid; e < i * w; e += nt) {
      const int a = e % i, c = i + e / i;
      const double xic = (c == i) ? W[c + (int64_t)l * l] : W[c + (int64_t)i * l];
      const double rai = W[a + (int64_t)i * l];
      W[c + (int64_t)a * l] -= rai * xic;
    }
    __syncthreads();
  }
  for (int e = tid; e < l * l; e += nt) {
    const int a = e % l, c = e / l;
    double v = 0.0;
    if (a == c) v = W[c + (int64_t)l * l];
    else if (a < c) v = W[c + (int64_t)a * l];
    Rinv[a + (int64_t)c * l] = v;
  }
  for (int j = tid; j < l; j += nt) diag[j] = W[j + (int64_t)j * l];
}

__global__ __launch_bounds__(kSmallThreads) void cholinv_lds_kernel(
    int l, const double* __restrict__ G, int64_t ldg, double tau, double* __restrict__ Rinv,
    double* __restrict__ diag, int32_t* status) {
  extern __shared__ double W[];  // l * (l + 1) + l + 1
  double* orig = W + (size_t)l * (l + 1);
  double* piv = orig + l;
  for (int e = threadIdx.x; e < l * l; e += blockDim.x) {
    const int a = e % l, b = e / l;
    W[e] = G[a + (int64_t)b * ldg];
  }
  __syncthreads();
  cholinv_body(l, W, tau, Rinv, diag, status, orig, piv);
}

__global__ __launch_bounds__(kSmallThreads) void cholinv_global_kernel(
    int l, const double* __restrict__ G, int64_t ldg, double tau, double* __restrict__ Rinv,
    double* __restrict__ diag, int32_t* status, double* __restrict__ W) {
  __shared__ double piv;
  extern __shared__ double orig[];
  for (int64_t e = threadIdx.x; e < (int64_t)l * l; e += blockDim.x) {
    const int64_t a = e % l, b = e / l;
    W[e] = G[a + b * ldg];
  }
  __syncthreads();
  cholinv_body(l, W, tau, Rinv, diag, status, orig, &piv);
}

size_t cholinv_workspace(int l) {
  Carver c(nullptr, 0);
  if (l > kLdsMaxL) c.take<double>((size_t)l * (l + 1));
  return c.off;
}

int cholinv(const rmm_ctx* h, int l, const double* G, int64_t ldg, double tau, double* Rinv,
            double* diag, int32_t* status, Carver& ws) {
  if (l == 0) return RMM_OK;
  if (l <= kLdsMaxL) {
    const size_t lds = ((size_t)l * (l + 1) + l + 1) * sizeof(double);
    RMM_HIP(hipFuncSetAttribute((const void*)cholinv_lds_kernel,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(cholinv_lds_kernel, dim3(1), dim3(kSmallThreads), lds, h->stream, l, G, ldg,
                       tau, Rinv, diag, status);
    return launch_status();
  }
  const size_t mark = ws.off;
  double* W = ws.take<double>((size_t)l * (l + 1));
  if (!ws.fits()) return RMM_ERR_WORKSPACE_TOO_SMALL;
  hipLaunchKernelGGL(cholinv_global_kernel, dim3(1), dim3(kSmallThreads), (size_t)l * sizeof(double),
                     h->stream, l, G, ldg, tau, Rinv, diag, status, W);
  ws.off = mark;
  return launch_status();
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
  extern __shared__ double S[];  // l * l, then pair tables
  const int L = (l + 1) & ~1;     // even number of players
  const int npairs = L / 2;
  double* cs = S + (size_t)l * l;       // npairs
  double* sn = cs + npairs;             // npairs
  int* pp = reinterpret_cast<int*>(sn + npairs);
  int* qq = pp + npairs;
  __shared__ double red[kSmallThreads / 64];
  __shared__ int done;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < l * l; e += nt) {
    const int a = e % l, b = e / l;
    S[e] = G[a + (int64_t)b * ldg];
    Vw[e] = (a == b) ? 1.0 : 0.0;
  }
  __syncthreads();
  // scale for the absolute part of the rotation threshold
  if (tid == 0) {
    double mx = 0.0;
    for (int i = 0; i < l; ++i) mx = fmax(mx, fabs(S[i + (int64_t)i * l]));
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
      for (int i = tid; i < npairs; i += nt) {
        const int a = (i == 0) ? 0 : ((i - 1 + r) % (L - 1)) + 1;
        const int b = ((L - 2 - i + r) % (L - 1)) + 1;
        int p = a < b ? a : b, q = a < b ? b : a;
        double c = 1.0, s = 0.0;
        if (q < l) {
          const double gpq = S[p + (int64_t)q * l];
          const double gpp = S[p + (int64_t)p * l], gqq = S[q + (int64_t)q * l];
          if (fabs(gpq) > abs_tol && fabs(gpq) > 0x1p-52 * sqrt(fabs(gpp * gqq))) {
            done = 0;
            const double theta = (gqq - gpp) / (2.0 * gpq);
            const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
          }
        } else {
          p = q = -1;
        }
        pp[i] = p;
        qq[i] = q;
        cs[i] = c;
        sn[i] = s;
      }
      __syncthreads();
      // rows: G <- J^T G
      for (int e = tid; e < npairs * l; e += nt) {
        const int i = e / l, k = e % l;
        const int p = pp[i], q = qq[i];
        if (p < 0 || sn[i] == 0.0) continue;
        const double c = cs[i], s = sn[i];
        const double gp = S[p + (int64_t)k * l], gq = S[q + (int64_t)k * l];
        S[p + (int64_t)k * l] = c * gp - s * gq;
        S[q + (int64_t)k * l] = s * gp + c * gq;
      }
      __syncthreads();
      // columns: G <- G J and V <- V J
      for (int e = tid; e < npairs * l; e += nt) {
        const int i = e / l, k = e % l;
        const int p = pp[i], q = qq[i];
        if (p < 0 || sn[i] == 0.0) continue;
        const double c = cs[i], s = sn[i];
        const double gp = S[k + (int64_t)p * l], gq = S[k + (int64_t)q * l];
        S[k + (int64_t)p * l] = c * gp - s * gq;
        S[k + (int64_t)q * l] = s * gp + c * gq;
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
  for (int j = tid; j < l; j += nt) {
    const double v = S[j + (int64_t)j * l];
    int rank = 0;
    for (int i = 0; i < l; ++i) {
      const double u = S[i + (int64_t)i * l];
      rank += (u > v) || (u == v && i < j);
    }
    evals[rank] = v;
    for (int k = 0; k < l; ++k) Vout[k + (int64_t)rank * l] = Vw[k + (int64_t)j * l];
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
  const size_t lds = (size_t)l * l * sizeof(double) + (size_t)L * sizeof(double) + (size_t)L * sizeof(int);
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
