// Block cyclic Jacobi eigensolver for symmetric l x l matrices, 128 < l <= 1024
// (the c x c matrix W = K[S, S] of the Nystrom method).
//
// The index set is cut into nb blocks of 32 (padded with zero rows and
// columns, which never rotate).  A sweep pairs the blocks by the circle
// method (nb - 1 rounds of nb / 2 disjoint block pairs).  In a round, for
// every pair (I, J):
//   1. the 64 x 64 subproblem W[IJ, IJ] (IJ = I u J) is copied to LDS and
//      one cyclic Jacobi sweep of 63 rounds of 32 disjoint rotations is run
//      on it, with the rotation test and angles of the scalar solver; the
//      product of its rotations, re-orthogonalized, is the 64 x 64 Q;
//   2. W[IJ, :] <- Q^T W[IJ, :]  (all pairs at once: their rows are disjoint);
//   3. W[:, IJ] <- W[:, IJ] Q and V[:, IJ] <- V[:, IJ] Q.
// So W <- P^T W P and V <- V P with P block orthogonal, and every sweep
// visits every pair of indices.  Before each sweep a scan decides
// convergence exactly as the scalar solver does (no off-diagonal element
// passes the rotation test); after it, all later launches return at once.
// Then the eigenvalues (the diagonal, descending, ties by index) and V's
// columns are sorted out.  Compared with one launch per scalar round
// (l - 1 rounds per sweep), a sweep here is nb - 1 = 31 rounds at l = 1024.
#include <math.h>

#include "common.hpp"
#include "dense.hpp"

namespace rmm {

namespace {

constexpr int kBB = 32;          // block size
constexpr int kBS = 2 * kBB;     // subproblem size
constexpr int kBLd = kBS + 1;    // padded LDS stride
constexpr int kBMaxSweeps = 30;

struct BlkState {
  double abs_tol;
  int pending;
  int converged;
  int sweeps;
};

__device__ __forceinline__ void circle_pair(int i, int r, int n, int& p, int& q) {
  const int a = (i == 0) ? 0 : ((i - 1 + r) % (n - 1)) + 1;
  const int b = ((n - 2 - i + r) % (n - 1)) + 1;
  p = a < b ? a : b;
  q = a < b ? b : a;
}

// global index of local index a (0..63) of the pair (bi, bj)
__device__ __forceinline__ int gidx(int a, int bi, int bj) {
  return a < kBB ? bi * kBB + a : bj * kBB + (a - kBB);
}

__global__ void blk_init_kernel(int l, int L, const double* __restrict__ G, int64_t ldg,
                                double* __restrict__ W, double* __restrict__ V, BlkState* st) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < (int64_t)L * L) {
    const int a = (int)(e % L), b = (int)(e / L);
    // the upper triangle of G is read and mirrored
    const double g = (a < l && b < l) ? (a <= b ? G[a + (int64_t)b * ldg] : G[b + (int64_t)a * ldg]) : 0.0;
    W[e] = g;
    V[e] = a == b ? 1.0 : 0.0;
  }
  if (e == 0) *st = BlkState{0.0, 0, 0, 0};
}

__global__ __launch_bounds__(256) void blk_tol_kernel(int l, int L, const double* __restrict__ W,
                                                      BlkState* st) {
  __shared__ double red[256];
  double mx = 0.0;
  for (int i = threadIdx.x; i < l; i += 256) mx = fmax(mx, fabs(W[i + (int64_t)i * L]));
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) st->abs_tol = 1e-17 * red[0];
}

__device__ __forceinline__ bool rot_test(double gpq, double gpp, double gqq, double abs_tol) {
  return fabs(gpq) > abs_tol && fabs(gpq) > 1e-300 && gpq * gpq > 0x1p-104 * fabs(gpp * gqq);
}

// pending |= an off-diagonal element (a < b < l) passes the rotation test
__global__ void blk_scan_kernel(int l, int L, const double* __restrict__ W, BlkState* st) {
  if (st->converged) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)l * l) return;
  const int a = (int)(e % l), b = (int)(e / l);
  if (a >= b) return;
  if (rot_test(W[a + (int64_t)b * L], W[a + (int64_t)a * L], W[b + (int64_t)b * L], st->abs_tol))
    atomicOr(&st->pending, 1);
}

__global__ void blk_decide_kernel(BlkState* st) {
  if (st->converged) return;
  if (st->pending == 0) st->converged = 1;
  else st->sweeps += 1;
  st->pending = 0;
}

// Step 1: one Jacobi sweep on the subproblem of block pair blockIdx.x of
// round r; D = Q - I (64 x 64, column-major) to Qbuf[pair].
__global__ __launch_bounds__(256) void blk_inner_kernel(int nb, int r, int L, const double* __restrict__ W,
                                                        double* __restrict__ Qbuf, const BlkState* st) {
  if (st->converged) return;
  __shared__ double S[kBS * kBLd];
  __shared__ double Q[kBS * kBLd];
  __shared__ double cs[kBB], sn[kBB], tn[kBB];
  __shared__ int pp[kBB], qq[kBB];
  const int tid = threadIdx.x;
  int bi, bj;
  circle_pair(blockIdx.x, r, nb, bi, bj);
  for (int e = tid; e < kBS * kBS; e += 256) {
    const int a = e % kBS, b = e / kBS;
    S[a + b * kBLd] = W[gidx(a, bi, bj) + (int64_t)gidx(b, bi, bj) * L];
    Q[a + b * kBLd] = a == b ? 1.0 : 0.0;
  }
  __syncthreads();
  const double abs_tol = st->abs_tol;
  for (int rr = 0; rr < kBS - 1; ++rr) {
    if (tid < kBB) {
      int p, q;
      circle_pair(tid, rr, kBS, p, q);
      double c = 1.0, s = 0.0, t = 0.0;
      const double gpq = S[p + q * kBLd], gpp = S[p + p * kBLd], gqq = S[q + q * kBLd];
      if (rot_test(gpq, gpp, gqq, abs_tol)) {
        const double theta = (gqq - gpp) / (2.0 * gpq);
        t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        c = 1.0 / sqrt(t * t + 1.0);
        s = t * c;
      }
      pp[tid] = p;
      qq[tid] = q;
      cs[tid] = c;
      sn[tid] = s;
      tn[tid] = t;
    }
    __syncthreads();
    // S <- J^T S J, one 2 x 2 block (pair i rows, pair j columns) per item
    double v[4][4];
    int ad[4][4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int item = tid + 256 * k;  // 1024 = 32 x 32 block pairs
      const int i = item & 31, j = item >> 5;
      const int pi = pp[i], qi = qq[i], pj = pp[j], qj = qq[j];
      ad[k][0] = pi + pj * kBLd;
      ad[k][1] = pi + qj * kBLd;
      ad[k][2] = qi + pj * kBLd;
      ad[k][3] = qi + qj * kBLd;
#pragma unroll
      for (int e = 0; e < 4; ++e) v[k][e] = S[ad[k][e]];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int item = tid + 256 * k;
      const int i = item & 31, j = item >> 5;
      const double ci = cs[i], si = sn[i], cj = cs[j], sj = sn[j];
      if (i == j) {
        if (si != 0.0) {
          const double t = tn[i];
          S[ad[k][0]] = v[k][0] - t * v[k][1];
          S[ad[k][3]] = v[k][3] + t * v[k][1];
          S[ad[k][1]] = 0.0;
          S[ad[k][2]] = 0.0;
        }
        continue;
      }
      const double y00 = ci * v[k][0] - si * v[k][2], y01 = ci * v[k][1] - si * v[k][3];
      const double y10 = si * v[k][0] + ci * v[k][2], y11 = si * v[k][1] + ci * v[k][3];
      S[ad[k][0]] = cj * y00 - sj * y01;
      S[ad[k][1]] = sj * y00 + cj * y01;
      S[ad[k][2]] = cj * y10 - sj * y11;
      S[ad[k][3]] = sj * y10 + cj * y11;
    }
    // Q <- Q J: row a, pair j
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int item = tid + 256 * k;  // 2048 = 64 rows x 32 pairs
      const int a = item & 63, j = item >> 6;
      const double c = cs[j], s = sn[j];
      if (s != 0.0) {
        const int pj = pp[j], qj = qq[j];
        const double x = Q[a + pj * kBLd], y = Q[a + qj * kBLd];
        Q[a + pj * kBLd] = c * x - s * y;
        Q[a + qj * kBLd] = s * x + c * y;
      }
    }
    __syncthreads();
  }
  // Each rotation is orthogonal only to rounding, and so is Q, their product;
  // applied again and again that drift would scale the eigenvalues.  So Q is
  // re-orthogonalized, Q <- Q (I - E / 2) with E = Q^T Q - I (orthogonal to
  // second order in E), and stored as D = Q - I: the updates then add a
  // small correction D^T W or W D to W, rounding relative to its size.
  const int a = tid & 63;
  double acc[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) acc[k] = 0.0;
  for (int t = 0; t < kBS; ++t) {
    const double qa = Q[t + a * kBLd];
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = fma(qa, Q[t + ((tid >> 6) + 4 * k) * kBLd], acc[k]);
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int b = (tid >> 6) + 4 * k;
    S[a + b * kBLd] = acc[k] - (a == b ? 1.0 : 0.0);  // E, symmetric
    acc[k] = 0.0;
  }
  __syncthreads();
  for (int t = 0; t < kBS; ++t) {
    const double qa = Q[a + t * kBLd];
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = fma(qa, S[t + ((tid >> 6) + 4 * k) * kBLd], acc[k]);
  }
  double* out = Qbuf + (size_t)blockIdx.x * kBS * kBS;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int b = (tid >> 6) + 4 * k;
    out[a + b * kBS] = (Q[a + b * kBLd] - (a == b ? 1.0 : 0.0)) - 0.5 * acc[k];
  }
}

// Step 2: W[IJ, c0:c0+64] <- W[IJ, c0:c0+64] + D^T W[IJ, c0:c0+64]
// (= Q^T W[IJ, ...]) for pair blockIdx.x, column tile blockIdx.y (in place:
// the tile is read into LDS first).
__global__ __launch_bounds__(256) void blk_rows_kernel(int nb, int r, int L, double* __restrict__ W,
                                                       const double* __restrict__ Qbuf, const BlkState* st) {
  if (st->converged) return;
  __shared__ double Qs[kBS * kBLd];
  __shared__ double T[kBS * kBLd];
  const int tid = threadIdx.x;
  int bi, bj;
  circle_pair(blockIdx.x, r, nb, bi, bj);
  const double* Qg = Qbuf + (size_t)blockIdx.x * kBS * kBS;
  const int c0 = blockIdx.y * kBS;
  for (int e = tid; e < kBS * kBS; e += 256) {
    const int a = e % kBS, b = e / kBS;
    Qs[a + b * kBLd] = Qg[e];
    T[a + b * kBLd] = W[gidx(a, bi, bj) + (int64_t)(c0 + b) * L];
  }
  __syncthreads();
  // thread: output rows a = tid & 63, columns b = (tid >> 6) + 4 k
  const int a = tid & 63;
  double acc[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) acc[k] = 0.0;
  for (int t = 0; t < kBS; ++t) {
    const double qa = Qs[t + a * kBLd];  // Q^T[a][t]
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = fma(qa, T[t + ((tid >> 6) + 4 * k) * kBLd], acc[k]);
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int b = (tid >> 6) + 4 * k;
    W[gidx(a, bi, bj) + (int64_t)(c0 + b) * L] = T[a + b * kBLd] + acc[k];
  }
}

// Step 3: X[r0:r0+64, IJ] <- X[r0:r0+64, IJ] + X[r0:r0+64, IJ] D (= X Q) for
// X = W (blockIdx.z = 0) and V (1)
__global__ __launch_bounds__(256) void blk_cols_kernel(int nb, int r, int L, double* __restrict__ W,
                                                       double* __restrict__ V, const double* __restrict__ Qbuf,
                                                       const BlkState* st) {
  if (st->converged) return;
  __shared__ double Qs[kBS * kBLd];
  __shared__ double T[kBS * kBLd];
  const int tid = threadIdx.x;
  int bi, bj;
  circle_pair(blockIdx.x, r, nb, bi, bj);
  double* X = blockIdx.z == 0 ? W : V;
  const double* Qg = Qbuf + (size_t)blockIdx.x * kBS * kBS;
  const int r0 = blockIdx.y * kBS;
  for (int e = tid; e < kBS * kBS; e += 256) {
    const int a = e % kBS, b = e / kBS;
    Qs[a + b * kBLd] = Qg[e];
    T[a + b * kBLd] = X[(r0 + a) + (int64_t)gidx(b, bi, bj) * L];
  }
  __syncthreads();
  // thread: output row a = tid & 63, columns b = (tid >> 6) + 4 k
  const int a = tid & 63;
  double acc[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) acc[k] = 0.0;
  for (int t = 0; t < kBS; ++t) {
    const double xa = T[a + t * kBLd];
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = fma(xa, Qs[t + ((tid >> 6) + 4 * k) * kBLd], acc[k]);
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int b = (tid >> 6) + 4 * k;
    X[(r0 + a) + (int64_t)gidx(b, bi, bj) * L] = T[a + b * kBLd] + acc[k];
  }
}

// eigenvalues (diagonal entries of the first l indices), descending with
// ties by index; perm[rank] = the index holding that eigenvalue
__global__ void blk_rank_kernel(int l, int L, const double* __restrict__ W, double* __restrict__ evals,
                                int* __restrict__ perm, const BlkState* st, int32_t* status) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j == 0 && !st->converged && status) atomicOr(status, RMM_STATUS_NOT_CONVERGED);
  if (j >= l) return;
  const double v = W[j + (int64_t)j * L];
  int rank = 0;
  for (int i = 0; i < l; ++i) {
    const double u = W[i + (int64_t)i * L];
    rank += (u > v) || (u == v && i < j);
  }
  evals[rank] = v;
  perm[rank] = j;
}

// Vout[:, rank] = V[:l, perm[rank]] (column rank = blockIdx.y)
__global__ void blk_vectors_kernel(int l, int L, const double* __restrict__ V, const int* __restrict__ perm,
                                   double* __restrict__ Vout) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= l) return;
  const int rank = blockIdx.y;
  Vout[k + (int64_t)rank * l] = V[k + (int64_t)perm[rank] * L];
}

}  // namespace

size_t jacobi_block_workspace(int l) {
  const int nb = ((l + kBB - 1) / kBB + 1) & ~1;  // even number of blocks
  const int L = nb * kBB;
  Carver c(nullptr, 0);
  c.take<double>((size_t)L * L);                  // W
  c.take<double>((size_t)L * L);                  // V
  c.take<double>((size_t)(nb / 2) * kBS * kBS);   // Q of each pair
  c.take<BlkState>(1);
  c.take<int>((size_t)l);                         // eigenvalue order
  return c.off + 5 * kAlign;
}

int jacobi_eig_block(const rmm_ctx* h, int l, const double* G, int64_t ldg, double* evals, double* V,
                     int32_t* status, Carver& ws) {
  const int nb = ((l + kBB - 1) / kBB + 1) & ~1;
  const int L = nb * kBB;
  const int np = nb / 2;
  const size_t mark = ws.off;
  double* W = ws.take<double>((size_t)L * L);
  double* Vw = ws.take<double>((size_t)L * L);
  double* Qb = ws.take<double>((size_t)np * kBS * kBS);
  BlkState* st = ws.take<BlkState>(1);
  int* perm = ws.take<int>((size_t)l);
  if (!ws.fits()) return RMM_ERR_WORKSPACE_TOO_SMALL;
  const int64_t LL = (int64_t)L * L;
  hipLaunchKernelGGL(blk_init_kernel, dim3((unsigned)((LL + 255) / 256)), dim3(256), 0, h->stream, l, L,
                     G, ldg, W, Vw, st);
  hipLaunchKernelGGL(blk_tol_kernel, dim3(1), dim3(256), 0, h->stream, l, L, W, st);
  RMM_TRY(launch_status());
  const unsigned sgroups = (unsigned)(((int64_t)l * l + 255) / 256);
  for (int sweep = 0; sweep <= kBMaxSweeps; ++sweep) {
    hipLaunchKernelGGL(blk_scan_kernel, dim3(sgroups), dim3(256), 0, h->stream, l, L, W, st);
    hipLaunchKernelGGL(blk_decide_kernel, dim3(1), dim3(1), 0, h->stream, st);
    RMM_TRY(launch_status());
    if (sweep == kBMaxSweeps) break;  // the last scan only decides convergence
    for (int r = 0; r < nb - 1; ++r) {
      hipLaunchKernelGGL(blk_inner_kernel, dim3((unsigned)np), dim3(256), 0, h->stream, nb, r, L, W, Qb, st);
      hipLaunchKernelGGL(blk_rows_kernel, dim3((unsigned)np, (unsigned)(L / kBS)), dim3(256), 0, h->stream,
                         nb, r, L, W, Qb, st);
      hipLaunchKernelGGL(blk_cols_kernel, dim3((unsigned)np, (unsigned)(L / kBS), 2u), dim3(256), 0,
                         h->stream, nb, r, L, W, Vw, Qb, st);
    }
    RMM_TRY(launch_status());
  }
  hipLaunchKernelGGL(blk_rank_kernel, dim3((unsigned)((l + 255) / 256)), dim3(256), 0, h->stream, l, L, W,
                     evals, perm, st, status);
  hipLaunchKernelGGL(blk_vectors_kernel, dim3((unsigned)((l + 255) / 256), (unsigned)l), dim3(256), 0,
                     h->stream, l, L, Vw, perm, V);
  ws.off = mark;
  return launch_status();
}

}  // namespace rmm
