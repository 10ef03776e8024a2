// Small FP64 factorizations that run in a single workgroup: the Cholesky
// step of CholeskyQR with the triangular inverse, the cyclic Jacobi
// eigensolver (Nystrom's W) and the one-sided Jacobi SVD used for the small
// SVD of the projected matrix.  These sit on
// the latency path of every driver call; a Cholesky leaf is at most
// 128 x 128 and lives in registers (larger factors are split recursively).
#include "common.hpp"
#include "dense.hpp"

namespace rmm {

constexpr int kSmallThreads = 1024;
constexpr int kLdsMaxL = 128;

__device__ __forceinline__ void or_status(int32_t* status, int32_t flag) {
  if (status) atomicOr(status, flag);
}

// Cholesky factor and triangular inverse of an l x l SPD matrix G (l <= 128,
// upper triangle read) by elimination of [G | I] without row scaling: step j
// subtracts W[j][i] / p_j times row j from every row i > j, where p_j is the
// j-th pivot.  The working matrix W holds G's upper triangle and, below the
// diagonal, L~^{-1} (initially 0, with an implicit unit diagonal).
// Afterwards the upper triangle holds D L~^T (G = L~ D L~^T, L~ unit lower
// triangular), the strict lower triangle holds L~^{-1}, and
//   R = D^{1/2} L~^T,   R^{-1}[c][j] = L~^{-1}[j][c] / sqrt(p_j)   (c <= j).
// Entry (i, c) changes in step j < i only for c >= i (Schur complement) or
// c <= j (inverse part); there it loses f_i r_c with f_i = W[j][i] / p_j and
// r = row j of W with r_j = 1.  The multiplier f_i depends on row j alone,
// so the updates a row receives from a run of pivots can be applied
// together once those pivot rows are final.
//
// Blocked by panels of 8 rows: wave q holds rows 8q .. 8q+7 in registers,
// lane t columns t and t + 64.  Panel p is eliminated within wave p; the
// wave then publishes the 8 pivot rows and the rows scaled by 1/p_j (the
// multipliers of every later row) to LDS, and after one barrier every later
// wave subtracts the 8 rank-one terms from its rows.  Wave p + 1 does that
// before factoring its own panel, while the waves behind it are still
// updating; the LDS panel buffers alternate, so one barrier per panel
// suffices.
//
// The elimination is a chain of dependent FP64 operations, so both phases
// are arranged for instruction-level parallelism: the update of a later
// wave accumulates its 16 entries side by side, pivot by pivot, and inside a
// panel the diagonal entries of the panel rows are tracked as wave-uniform
// values with the same operations the lanes apply to them, so a pivot
// depends on the previous one through one FMA and a reciprocal while the
// row updates run beside that chain.  The reciprocal is the hardware
// estimate refined by two Newton steps.
// The drop test of pivot j compares against orig[j * ostride] (the diagonal
// of the matrix the caller considers original), or G_jj when orig is null;
// a dropped pivot eliminates nothing and gives a zero column of R^{-1}.
constexpr int kPanel = 8;

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ double recip_f64(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(fma(-x, y, 1.0), y, y);
  return fma(fma(-x, y, 1.0), y, y);
}

// Phase A of one panel (rows p0 .. p0+7, all held by this wave); HP is the
// column half that holds the panel's own columns.  Outside them every entry
// of a later row is updated (c < p0 is inverse part with c < j, c >= p0 + 8
// Schur part with c > i); inside, an entry with j < c < i is left alone and
// r_j = 1.  Rows past l have zero pivots and thresholds, so their steps
// change nothing; `live` has bit r set for rows below l.
// 1/sqrt(x), x > 0 finite: the hardware estimate refined by two Newton steps
__device__ __forceinline__ double rsqrt_f64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = y * fma(-hx * y, y, 1.5);
  return y * fma(-hx * y, y, 1.5);
}

template <int NH, int HP>
__device__ __forceinline__ void panel_factor(double (&w)[kPanel][NH], int lane, int p0, unsigned live,
                                             double thr, double (*prow)[kLdsMaxL],
                                             double (*pmul)[kLdsMaxL], double* piv,
                                             int32_t* status) {
  // W[i][i] of the panel rows, uniform
  double dg[kPanel];
#pragma unroll
  for (int r = 0; r < kPanel; ++r) dg[r] = readlane_f64(w[r][HP], (p0 + r) & 63);
#pragma unroll
  for (int r = 0; r < kPanel; ++r) {
    const int j = p0 + r;
    const double pv = dg[r];
    const bool keep = pv > readlane_f64(thr, r) && pv > 1e-300;
    const double inv = keep ? recip_f64(pv) : 0.0;
    if (lane == 0) {
      piv[j] = keep ? pv : 0.0;
      if (!keep && ((live >> r) & 1u)) or_status(status, RMM_STATUS_QR_FALLBACK);
    }
    const int c = lane + 64 * HP;
    const double rlo = c < j ? w[r][HP] : (c == j ? 1.0 : 0.0);  // r_c where c <= j
#pragma unroll
    for (int r2 = r + 1; r2 < kPanel; ++r2) {
      const int i = p0 + r2;
      const double b = readlane_f64(w[r][HP], i & 63);
      const double fi = inv * b;
      dg[r2] = fma(-fi, b, dg[r2]);  // what lane i does to W[i][i] below
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        const double rj = (h != HP || c >= i) ? w[r][h] : rlo;
        w[r2][h] = fma(-fi, rj, w[r2][h]);
      }
    }
    // row j is final: publish it and its multipliers
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      const int ch = lane + 64 * h;
      prow[r][ch] = (ch == j) ? 1.0 : w[r][h];
      pmul[r][ch] = w[r][h] * inv;
    }
  }
}

template <int NH>
__global__ __launch_bounds__(1024) void cholinv_panel_kernel(
    int l, const double* __restrict__ G, int64_t ldg, double tau, const double* orig,
    int64_t ostride, double* __restrict__ Rinv, int64_t ldr, double* __restrict__ diag,
    int32_t* status) {
  // pivot rows (r_j = 1) and multipliers [jj][i] = W[j][i] / p_j
  __shared__ __align__(16) double prow[2][kPanel][kLdsMaxL];
  __shared__ __align__(16) double pmul[2][kPanel][kLdsMaxL];
  __shared__ double piv[kLdsMaxL];
  const int lane = threadIdx.x & 63;
  const int q = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int q0 = q * kPanel;
  const int np = (l + kPanel - 1) / kPanel;  // one wave per panel
  double w[kPanel][NH];
#pragma unroll
  for (int r = 0; r < kPanel; ++r)
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      const int i = q0 + r, c = lane + 64 * h;
      w[r][h] = (i < l && c < l && i <= c) ? G[i + (int64_t)c * ldg] : 0.0;
    }
  // drop threshold of this wave's row 8q + (lane & 7)
  const int tr = q0 + (lane & (kPanel - 1));
  const double thr =
      tr < l ? tau * (orig ? orig[tr * ostride] : G[tr + (int64_t)tr * ldg]) : 0.0;
  // the wave that factors the next panel is on the critical path: it runs at
  // raised issue priority from its last update until it has published
  if (q == 0) __builtin_amdgcn_s_setprio(3);
  for (int p = 0; p < np; ++p) {
    const int buf = p & 1, p0 = p * kPanel;
    if (q == p) {
      const int nl = l - p0;
      const unsigned live = nl >= kPanel ? 0xFFu : ((1u << nl) - 1u);
      if (NH > 1 && p0 >= 64)
        panel_factor<NH, NH - 1>(w, lane, p0, live, thr, prow[buf], pmul[buf], piv, status);
      else
        panel_factor<NH, 0>(w, lane, p0, live, thr, prow[buf], pmul[buf], piv, status);
      __builtin_amdgcn_s_setprio(0);
    }
    lds_barrier();
    // later waves (always whole panels: a partial panel is the last one)
    if (q > p) {
      if (q == p + 1) __builtin_amdgcn_s_setprio(3);
      // r_c of pivot p0 + jj for this lane's columns: always for c < p0 and
      // c >= q0, for the panel's own columns when c <= p0 + jj, never for the
      // columns between the panel and this wave's rows; those inside the
      // wave's own block are masked per row below
      bool always[NH];
      unsigned pc[NH];
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        const int c = lane + 64 * h;
        always[h] = c < p0 || c >= q0;
        pc[h] = (unsigned)(c - p0);
      }
      double t[kPanel][NH];
#pragma unroll
      for (int r = 0; r < kPanel; ++r)
#pragma unroll
        for (int h = 0; h < NH; ++h) t[r][h] = 0.0;
      // pivot jj + 1's operands are read while pivot jj's are multiplied
      double f[kPanel], rv[NH];
#pragma unroll
      for (int r = 0; r < kPanel; ++r) f[r] = pmul[buf][0][q0 + r];
#pragma unroll
      for (int h = 0; h < NH; ++h) rv[h] = prow[buf][0][lane + 64 * h];
#pragma unroll
      for (int jj = 0; jj < kPanel; ++jj) {
        double fn[kPanel], rn[NH];
        if (jj + 1 < kPanel) {
#pragma unroll
          for (int r = 0; r < kPanel; ++r) fn[r] = pmul[buf][jj + 1][q0 + r];
#pragma unroll
          for (int h = 0; h < NH; ++h) rn[h] = prow[buf][jj + 1][lane + 64 * h];
        }
#pragma unroll
        for (int h = 0; h < NH; ++h) {
          const double rl = (always[h] || pc[h] <= (unsigned)jj) ? rv[h] : 0.0;
#pragma unroll
          for (int r = 0; r < kPanel; ++r) t[r][h] = fma(f[r], rl, t[r][h]);
        }
        if (jj + 1 < kPanel) {
#pragma unroll
          for (int r = 0; r < kPanel; ++r) f[r] = fn[r];
#pragma unroll
          for (int h = 0; h < NH; ++h) rv[h] = rn[h];
        }
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int r = 0; r < kPanel; ++r)
#pragma unroll
        for (int h = 0; h < NH; ++h) {
          const int c = lane + 64 * h, i = q0 + r;
          w[r][h] = (c >= i || c < q0) ? w[r][h] - t[r][h] : w[r][h];
        }
    }
  }
  __syncthreads();
  // R^{-1}[c][j] = (c == j ? 1 : W[j][c]) / sqrt(p_j) for c <= j; every value
  // is formed before the first store
#pragma unroll
  for (int r = 0; r < kPanel; ++r) {
    const int j = q0 + r;
    const double pj = j < l ? piv[j] : 0.0;
    const double rs = pj > 0.0 ? 1.0 / sqrt(pj) : 0.0;
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      const int c = lane + 64 * h;
      w[r][h] = c <= j ? ((c == j) ? 1.0 : w[r][h]) * rs : 0.0;
    }
  }
#pragma unroll
  for (int r = 0; r < kPanel; ++r)
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      const int j = q0 + r, c = lane + 64 * h;
      if (j < l && c < l) Rinv[c + (int64_t)j * ldr] = w[r][h];
    }
  if ((int)threadIdx.x < l) diag[threadIdx.x] = sqrt(piv[threadIdx.x]);
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
    const dim3 block(64 * ((l + kPanel - 1) / kPanel));
    if (l <= 64)
      hipLaunchKernelGGL((cholinv_panel_kernel<1>), dim3(1), block, 0, h->stream, l, G, ldg, tau,
                         orig, ostride, Rinv, ldr, diag, status);
    else
      hipLaunchKernelGGL((cholinv_panel_kernel<2>), dim3(1), block, 0, h->stream, l, G, ldg, tau,
                         orig, ostride, Rinv, ldr, diag, status);
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
// L/2 disjoint pairs (p, q) of the circle method are rotated at once.  The
// rotation zeroing G_pq follows the classical choice
//   t = sgn(theta) / (|theta| + sqrt(theta^2 + 1)),  theta = (G_qq - G_pp) / (2 G_pq),
//   c = 1 / sqrt(t^2 + 1),  s = t c,
// with G_pp -= t G_pq, G_qq += t G_pq, G_pq = 0 on the rotated pair.
//
// jacobi_kernel works on G only: the upper triangle sits in LDS and the
// update of one round is done per 2 x 2 block of pairs (i <= j), J_i^T G J_j,
// so every stored element is read and written once per round.  The (c, s)
// of every pair of every round are appended to a log in global memory;
// jacobi_vectors_kernel then accumulates V = J_1 J_2 ... row by row, each
// row of V being independent, with one wave per group of rows.
constexpr int kJacobiMaxSweeps = 40;
constexpr int kVecRows = 4;  // rows of V per wave

__device__ __forceinline__ void rr_pair(int i, int r, int L, int& p, int& q) {
  // circle method: player 0 fixed, players 1 .. L-1 rotate by one per round
  const int a = (i == 0) ? 0 : ((i - 1 + r) % (L - 1)) + 1;
  const int b = ((L - 2 - i + r) % (L - 1)) + 1;
  p = a < b ? a : b;
  q = a < b ? b : a;
}

// Pair order of osj_kernel.  L is a power of two and the P = L/2 lane groups
// work on L/2 disjoint pairs per round.  Level t of a sweep (t = 0, 1, ...)
// splits the columns into blocks of 2Q with Q = P >> t; the Q groups of a
// block b keep its first Q columns ("residents") and pass its last Q
// columns ("travellers") around: in round u of the level, group i = bQ + j
// pairs resident 2Qb + j with traveller 2Qb + Q + (j + u) mod Q, then hands
// its traveller to group j - 1 of the block.  Level t covers every
// resident-traveller pair of its blocks once, and the residents and the
// travellers of a block become the two blocks of level t + 1, so a sweep
// (levels Q = P, P/2, ..., 1: P + P/2 + ... + 1 = L - 1 rounds) meets
// every pair exactly once, while a group reads and writes only one column
// per round.

__host__ __device__ inline int pow2_ceil(int l) {
  int L = 2;
  while (L < l) L <<= 1;
  return L;
}

__global__ __launch_bounds__(kSmallThreads) void jacobi_kernel(int l, const double* __restrict__ G,
                                                               int64_t ldg, double* __restrict__ evals,
                                                               int* __restrict__ perm,
                                                               double2* __restrict__ rlog,
                                                               int* __restrict__ nrounds,
                                                               int32_t* status, int max_sweeps) {
  extern __shared__ double S[];  // L x (L + 1), upper triangle (a <= b at S[a + b * lds])
  const int L = (l + 1) & ~1;     // even number of players; index l is a zero dummy when l is odd
  const int lds = L + 1;
  const int npairs = L / 2;
  double* cs = S + (size_t)L * lds;  // per pair: c, s, t
  double* sn = cs + npairs;
  double* tn = sn + npairs;
  int* pp = reinterpret_cast<int*>(tn + npairs);
  int* qq = pp + npairs;
  __shared__ double red[1];
  __shared__ int done;
  const int tid = threadIdx.x;
  for (int e = tid; e < L * L; e += blockDim.x) {
    const int a = e % L, b = e / L;
    if (a <= b) S[a + b * lds] = (b < l) ? G[a + (int64_t)b * ldg] : 0.0;
  }
  __syncthreads();
  if (tid == 0) {
    double mx = 0.0;
    for (int i = 0; i < l; ++i) mx = fmax(mx, fabs(S[i + i * lds]));
    red[0] = mx;
  }
  __syncthreads();
  const double abs_tol = 1e-17 * red[0];
  // blocks (i, j), i <= j, of the pair grid: row pair (u, npairs-1-u) holds
  // npairs + 1 blocks; 32 threads share one row pair
  const int rp = tid >> 5, w = tid & 31;
  int sweep = 0, rounds = 0;
  for (; sweep < max_sweeps; ++sweep) {
    // a sweep rotates nothing exactly when no pair passes the rotation test
    // now (the matrix cannot change before the first rotation), so the sweep
    // that would only confirm convergence is replaced by this scan
    lds_barrier();
    if (tid == 0) done = 1;
    lds_barrier();
    for (int e = tid; e < l * l; e += blockDim.x) {
      const int a = e % l, b = e / l;
      if (a < b) {
        // exactly the rotation test below
        const double gpq = S[a + b * lds];
        if (fabs(gpq) > abs_tol && fabs(gpq) > 1e-300 &&
            gpq * gpq > 0x1p-104 * fabs(S[a + a * lds] * S[b + b * lds]))
          done = 0;
      }
    }
    lds_barrier();
    if (done) break;
    for (int r = 0; r < L - 1; ++r, ++rounds) {
      // the log stores are not waited for at the barriers below
      if (tid < npairs) {
        int p, q;
        rr_pair(tid, r, L, p, q);
        double c = 1.0, s = 0.0, tt = 0.0;
        if (q < l) {
          const double gpq = S[p + q * lds];
          const double gpp = S[p + p * lds], gqq = S[q + q * lds];
          // same test as |g_pq| > 2^-52 sqrt(|g_pp g_qq|), squared; the
          // rotation is built from refined hardware estimates (a short
          // dependent chain at the head of every round)
          if (fabs(gpq) > abs_tol && fabs(gpq) > 1e-300 &&
              gpq * gpq > 0x1p-104 * fabs(gpp * gqq)) {
            const double theta = (gqq - gpp) * recip_f64(2.0 * gpq);
            const double at = fabs(theta);
            const double w = at * at + 1.0;
            const double den = at > 0x1p26 ? 2.0 * at : at + w * rsqrt_f64(w);
            tt = (theta >= 0 ? 1.0 : -1.0) * recip_f64(den);
            c = rsqrt_f64(tt * tt + 1.0);
            s = tt * c;
          }
        }
        pp[tid] = p;
        qq[tid] = q;
        cs[tid] = c;
        sn[tid] = s;
        tn[tid] = tt;
        rlog[(size_t)rounds * npairs + tid] = make_double2(c, s);
      }
      lds_barrier();
      if (rp < (npairs + 1) / 2) {
        // up to 3 blocks per thread; all LDS reads of a thread's blocks are
        // issued before any arithmetic so their latencies overlap
        const int u0 = rp, u1 = npairs - 1 - rp;
        const int n0 = npairs - u0;  // blocks (u0, u0 .. npairs-1), then (u1, u1 .. npairs-1)
        const int nb = (u0 == u1) ? n0 : npairs + 1;
        int bi[3], bj[3];
        bool live[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const int b = w + 32 * k;
          live[k] = b < nb;
          bi[k] = b < n0 ? u0 : u1;
          bj[k] = b < n0 ? u0 + b : u1 + (b - n0);
          if (!live[k]) bi[k] = bj[k] = 0;
        }
        double ci[3], si[3], cj[3], sj[3], ti[3];
        int pi[3], qi[3], pj[3], qj[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          ci[k] = cs[bi[k]]; si[k] = sn[bi[k]]; ti[k] = tn[bi[k]];
          cj[k] = cs[bj[k]]; sj[k] = sn[bj[k]];
          pi[k] = pp[bi[k]]; qi[k] = qq[bi[k]]; pj[k] = pp[bj[k]]; qj[k] = qq[bj[k]];
        }
        int ad[3][4];
        double x[3][4];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          // element (a, b) of the symmetric matrix lives at (min, max)
          ad[k][0] = pi[k] < pj[k] ? pi[k] + pj[k] * lds : pj[k] + pi[k] * lds;
          ad[k][1] = pi[k] < qj[k] ? pi[k] + qj[k] * lds : qj[k] + pi[k] * lds;
          ad[k][2] = qi[k] < pj[k] ? qi[k] + pj[k] * lds : pj[k] + qi[k] * lds;
          ad[k][3] = qi[k] < qj[k] ? qi[k] + qj[k] * lds : qj[k] + qi[k] * lds;
#pragma unroll
          for (int e = 0; e < 4; ++e) x[k][e] = S[ad[k][e]];
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          if (!live[k] || (si[k] == 0.0 && sj[k] == 0.0)) continue;
          if (bi[k] == bj[k]) {
            // x = (pp, pq, qp, qq) of the rotated pair
            const double gpq = x[k][1];
            S[ad[k][0]] = x[k][0] - ti[k] * gpq;
            S[ad[k][3]] = x[k][3] + ti[k] * gpq;
            S[ad[k][1]] = 0.0;
            continue;
          }
          // rows: J_i^T X, then columns: (J_i^T X) J_j
          const double y00 = ci[k] * x[k][0] - si[k] * x[k][2];
          const double y01 = ci[k] * x[k][1] - si[k] * x[k][3];
          const double y10 = si[k] * x[k][0] + ci[k] * x[k][2];
          const double y11 = si[k] * x[k][1] + ci[k] * x[k][3];
          S[ad[k][0]] = cj[k] * y00 - sj[k] * y01;
          S[ad[k][1]] = sj[k] * y00 + cj[k] * y01;
          S[ad[k][2]] = cj[k] * y10 - sj[k] * y11;
          S[ad[k][3]] = sj[k] * y10 + cj[k] * y11;
        }
      }
      lds_barrier();
    }
  }
  if (tid == 0) {
    *nrounds = rounds;
    if (sweep == max_sweeps) or_status(status, RMM_STATUS_NOT_CONVERGED);
  }
  // sort descending (ties by index)
  for (int j = tid; j < l; j += blockDim.x) {
    const double v = S[j + j * lds];
    int rank = 0;
    for (int i = 0; i < l; ++i) {
      const double u = S[i + i * lds];
      rank += (u > v) || (u == v && i < j);
    }
    evals[rank] = v;
    perm[rank] = j;
  }
}

// V = J_1 J_2 ... J_R from the rotation log; Vout[:, rank] = V[:, perm[rank]].
// One wave owns kVecRows rows of V in LDS; lane i applies pair i of every
// round to those rows (the pairs of a round are disjoint, and one wave's LDS
// accesses are performed in program order, so no barrier is needed).
__global__ __launch_bounds__(256) void jacobi_vectors_kernel(int l, const double2* __restrict__ rlog,
                                                             const int* __restrict__ nrounds,
                                                             const int* __restrict__ perm,
                                                             double* __restrict__ Vout) {
  extern __shared__ double vs[];  // 4 waves x kVecRows x L, then the pair tables
  const int L = (l + 1) & ~1;
  const int npairs = L / 2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double* V = vs + (size_t)wave * kVecRows * L;
  unsigned char* ptab = reinterpret_cast<unsigned char*>(vs + (size_t)4 * kVecRows * L);
  unsigned char* qtab = ptab + (size_t)(L - 1) * npairs;
  for (int e = threadIdx.x; e < (L - 1) * npairs; e += blockDim.x) {
    int p, q;
    rr_pair(e % npairs, e / npairs, L, p, q);
    ptab[e] = (unsigned char)p;
    qtab[e] = (unsigned char)q;
  }
  const int row0 = (blockIdx.x * 4 + wave) * kVecRows;
  for (int e = lane; e < kVecRows * L; e += 64) {
    const int rr = e / L, c = e % L;
    V[e] = (row0 + rr == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int R = *nrounds;
  const bool active = lane < npairs;
  // the log is read kPrefetch rounds ahead: the next batch is in flight while
  // the current one is applied
  constexpr int kPrefetch = 16;
  double2 cur[kPrefetch], nxt[kPrefetch];
#pragma unroll
  for (int u = 0; u < kPrefetch; ++u)
    cur[u] = (active && u < R) ? rlog[(size_t)u * npairs + lane] : make_double2(1.0, 0.0);
  int r = 0;  // round within the sweep
  for (int t0 = 0; t0 < R; t0 += kPrefetch) {
#pragma unroll
    for (int u = 0; u < kPrefetch; ++u) {
      const int t = t0 + kPrefetch + u;
      nxt[u] = (active && t < R) ? rlog[(size_t)t * npairs + lane] : make_double2(1.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < kPrefetch; ++u) {
      if (t0 + u < R && cur[u].y != 0.0) {
        const int p = ptab[r * npairs + lane], q = qtab[r * npairs + lane];
#pragma unroll
        for (int rr = 0; rr < kVecRows; ++rr) {
          const double vp = V[rr * L + p], vq = V[rr * L + q];
          V[rr * L + p] = cur[u].x * vp - cur[u].y * vq;
          V[rr * L + q] = cur[u].y * vp + cur[u].x * vq;
        }
      }
      if (++r == L - 1) r = 0;
    }
#pragma unroll
    for (int u = 0; u < kPrefetch; ++u) cur[u] = nxt[u];
  }
  for (int rr = 0; rr < kVecRows; ++rr) {
    const int k = row0 + rr;
    if (k >= l) break;
    for (int rank = lane; rank < l; rank += 64) Vout[k + (int64_t)rank * l] = V[rr * L + perm[rank]];
  }
}

// J = J_1 J_2 ... from the log of osj_kernel; Jout[:, rank] = J[:, perm[rank]].
// Rows of J are independent and follow the column movements of the
// one-sided sweep itself: a wave holds kOsjVecRows rows, lane g the entries
// of its rows at group g's resident (x) and traveller (y) columns.  A round
// rotates (x, y) with group g's logged (cs, sn); inside a level the
// travellers pass to the next lower group of their block by a lane shuffle
// (no LDS round trip), and at a level's end the row is laid out in column
// order in the wave's LDS row buffer and read back in the next level's
// pairing.  The rounds of a sweep are therefore a chain of shuffles and
// FMAs per wave, and the rows run in parallel over the workgroups.
constexpr int kOsjVecRows = 2;

__global__ __launch_bounds__(256) void osj_vectors_kernel(int l, const double2* __restrict__ rlog,
                                                          const int* __restrict__ nrounds,
                                                          const int* __restrict__ perm,
                                                          double* __restrict__ Jout) {
  __shared__ double buf[4][kOsjVecRows][kLdsMaxL];
  const int L = pow2_ceil(l), P = L / 2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row0 = (blockIdx.x * 4 + wave) * kOsjVecRows;
  if (row0 >= l) return;  // whole waves
  const bool act = lane < P;
  const int g = act ? lane : 0;
  double x[kOsjVecRows], y[kOsjVecRows];
#pragma unroll
  for (int w = 0; w < kOsjVecRows; ++w) {
    x[w] = row0 + w == g ? 1.0 : 0.0;
    y[w] = row0 + w == P + g ? 1.0 : 0.0;
    if (act) {  // column order, for a log without rounds
      buf[wave][w][g] = x[w];
      buf[wave][w][P + g] = y[w];
    }
  }
  const int R = *nrounds;  // whole sweeps of L - 1 rounds
  int Q = P, u = 0;        // level and round within it
  constexpr int kPre = 16;  // rounds of the log in flight
  double2 cur[kPre], nxt[kPre];
#pragma unroll
  for (int k = 0; k < kPre; ++k) cur[k] = k < R ? rlog[(size_t)k * P + g] : make_double2(1.0, 0.0);
  for (int t0 = 0; t0 < R; t0 += kPre) {
#pragma unroll
    for (int k = 0; k < kPre; ++k) {
      const int t = t0 + kPre + k;
      nxt[k] = t < R ? rlog[(size_t)t * P + g] : make_double2(1.0, 0.0);
    }
#pragma unroll
    for (int k = 0; k < kPre; ++k) {
      if (t0 + k < R) {
        const double c = cur[k].x, sn = cur[k].y;
        if (sn != 0.0) {
#pragma unroll
          for (int w = 0; w < kOsjVecRows; ++w) {
            const double xv = x[w], yv = y[w];
            x[w] = c * xv - sn * yv;
            y[w] = sn * xv + c * yv;
          }
        }
        const int j = g & (Q - 1), b0 = g - j;  // block start b Q
        if (u + 1 < Q) {
          const int src = b0 + ((j + 1) & (Q - 1));
#pragma unroll
          for (int w = 0; w < kOsjVecRows; ++w) y[w] = __shfl(y[w], src);
          ++u;
        } else {
          const int pc = 2 * b0 + j, qc = 2 * b0 + Q + ((j + Q - 1) & (Q - 1));
          if (act) {
#pragma unroll
            for (int w = 0; w < kOsjVecRows; ++w) {
              buf[wave][w][pc] = x[w];
              buf[wave][w][qc] = y[w];
            }
          }
          // one wave's LDS accesses are performed in program order
          __builtin_amdgcn_wave_barrier();
          Q = Q > 1 ? Q >> 1 : P;
          u = 0;
          const int j1 = g & (Q - 1);
          const int pn = 2 * (g - j1) + j1, qn = pn + Q;
          if (act) {
#pragma unroll
            for (int w = 0; w < kOsjVecRows; ++w) {
              x[w] = buf[wave][w][pn];
              y[w] = buf[wave][w][qn];
            }
          }
          __builtin_amdgcn_wave_barrier();
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kPre; ++k) cur[k] = nxt[k];
  }
  // R is a whole number of sweeps, so the last level end left every row in
  // column order
#pragma unroll
  for (int w = 0; w < kOsjVecRows; ++w) {
    const int k = row0 + w;
    if (k >= l) break;
    for (int rank = lane; rank < l; rank += 64) Jout[k + (int64_t)rank * l] = buf[wave][w][perm[rank]];
  }
}

// ---- shared pieces of the global-memory Jacobi paths (l up to 1024) --------------------
//
// The one-sided SVD below for l > 128 runs one launch per round of the
// parallel cyclic order, logs the round's rotations, and applies a sweep's log
// to the rows of its vector matrix (row-major in the workspace) with
// big_vectors_kernel.  The symmetric eigensolver for l > 128 is the block
// Jacobi of blockjacobi.hip.
constexpr int kBigMaxL = 1024;
constexpr int kBigMaxSweeps = 30;

struct BigState {
  double abs_tol;  // 1e-17 * max |G_ii|, the absolute rotation threshold
  int pending;     // some pair of the current matrix passes the rotation test
  int converged;   // no pair passes: the next sweep would rotate nothing
  int parity;      // buffer holding the current matrix
  int sweeps;      // sweeps run
};

// Apply one sweep's logged rotations to rows of V (row-major L x L): wave =
// 2 rows, lane handles pairs lane, lane + 64, ...; the next round's
// rotations are loaded while the current round is applied.
constexpr int kBigVecRows = 2;
__global__ __launch_bounds__(256) void big_vectors_kernel(int L, const double2* __restrict__ rlog,
                                                          const uint16_t* __restrict__ ptab,
                                                          const uint16_t* __restrict__ qtab,
                                                          double* __restrict__ Vr, const BigState* st) {
  if (st->converged) return;  // the sweep's rounds did not run
  extern __shared__ double vs[];  // 4 waves x kBigVecRows x L
  const int npairs = L / 2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double* V = vs + (size_t)wave * kBigVecRows * L;
  const int row0 = (blockIdx.x * 4 + wave) * kBigVecRows;
  for (int rr = 0; rr < kBigVecRows; ++rr)
    for (int c = lane; c < L; c += 64)
      V[rr * L + c] = row0 + rr < L ? Vr[(int64_t)(row0 + rr) * L + c] : 0.0;
  constexpr int PP = kBigMaxL / 2 / 64;  // pairs per lane at most
  double2 cur[PP], nxt[PP];
#pragma unroll
  for (int k = 0; k < PP; ++k) {
    const int pr = lane + 64 * k;
    cur[k] = pr < npairs ? rlog[pr] : make_double2(1.0, 0.0);
  }
  for (int r = 0; r < L - 1; ++r) {
#pragma unroll
    for (int k = 0; k < PP; ++k) {
      const int pr = lane + 64 * k;
      nxt[k] = (pr < npairs && r + 1 < L - 1) ? rlog[(size_t)(r + 1) * npairs + pr] : make_double2(1.0, 0.0);
    }
#pragma unroll
    for (int k = 0; k < PP; ++k) {
      const int pr = lane + 64 * k;
      if (pr < npairs && cur[k].y != 0.0) {
        const int p = ptab[(size_t)r * npairs + pr], q = qtab[(size_t)r * npairs + pr];
#pragma unroll
        for (int rr = 0; rr < kBigVecRows; ++rr) {
          const double vp = V[rr * L + p], vq = V[rr * L + q];
          V[rr * L + p] = cur[k].x * vp - cur[k].y * vq;
          V[rr * L + q] = cur[k].y * vp + cur[k].x * vq;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < PP; ++k) cur[k] = nxt[k];
  }
  for (int rr = 0; rr < kBigVecRows; ++rr)
    if (row0 + rr < L)
      for (int c = lane; c < L; c += 64) Vr[(int64_t)(row0 + rr) * L + c] = V[rr * L + c];
}

size_t jacobi_workspace(int l) {
  const int L = (l + 1) & ~1;
  if (l > kLdsMaxL) return jacobi_block_workspace(l);
  Carver c(nullptr, 0);
  c.take<double2>((size_t)kJacobiMaxSweeps * (L - 1) * (L / 2));
  c.take<int>((size_t)l);
  c.take<int>(1);
  return c.off + 3 * kAlign;
}

int jacobi_eig(const rmm_ctx* h, int l, const double* G, int64_t ldg, double* evals, double* V,
               int32_t* status, Carver& ws) {
  if (l == 0) return RMM_OK;
  if (l > kBigMaxL) return RMM_ERR_UNSUPPORTED;
  if (l > kLdsMaxL) return jacobi_eig_block(h, l, G, ldg, evals, V, status, ws);
  const int L = (l + 1) & ~1;
  const int npairs = L / 2;
  const size_t mark = ws.off;
  double2* rlog = ws.take<double2>((size_t)kJacobiMaxSweeps * (L - 1) * npairs);
  int* perm = ws.take<int>((size_t)l);
  int* nr = ws.take<int>(1);
  if (!ws.fits()) return RMM_ERR_WORKSPACE_TOO_SMALL;
  const size_t lds = (size_t)L * (L + 1) * sizeof(double) + 3 * (size_t)npairs * sizeof(double) +
                     2 * (size_t)npairs * sizeof(int);
  RMM_HIP(hipFuncSetAttribute((const void*)jacobi_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds));
  // 32 threads per row pair of the pair grid: no more waves than that, since
  // every round ends in two workgroup barriers whose cost grows with the waves
  int threads = (npairs + 1) / 2 * 32;
  threads = (threads + 63) / 64 * 64;
  if (threads > kSmallThreads) threads = kSmallThreads;
  hipLaunchKernelGGL(jacobi_kernel, dim3(1), dim3(threads), lds, h->stream, l, G, ldg, evals,
                     perm, rlog, nr, status, kJacobiMaxSweeps);
  RMM_TRY(launch_status());
  const size_t vlds = (size_t)4 * kVecRows * L * sizeof(double) + 2 * (size_t)(L - 1) * npairs;
  RMM_HIP(hipFuncSetAttribute((const void*)jacobi_vectors_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)vlds));
  const int groups = (l + 4 * kVecRows - 1) / (4 * kVecRows);
  hipLaunchKernelGGL(jacobi_vectors_kernel, dim3(groups), dim3(256), vlds, h->stream, l, rlog,
                     nr, perm, V);
  ws.off = mark;
  return launch_status();
}

// ---- one-sided (Hestenes) Jacobi SVD ------------------------------------------------------
//
// The small SVD of the drivers: for an l x l FP64 matrix M, plane rotations
// J_1 J_2 ... applied to pairs of columns make the columns of M J mutually
// orthogonal; then M J = Ubar diag(sigma) with sigma_j the column norms.
// Every rotation is computed from the current columns themselves (their
// squared norms a, b and inner product c), so the singular values come out
// with an absolute error of order eps * ||M||, not eps * ||M||^2 / sigma as
// from an eigendecomposition of M^T M.  A pair is rotated when
//   c^2 > l * eps^2 * a * b,
// with the angle that makes the pair orthogonal,
//   zeta = (b - a) / (2 c),  t = sgn(zeta) / (|zeta| + sqrt(1 + zeta^2)),
//   cs = 1 / sqrt(1 + t^2),  sn = t cs,
//   col_p <- cs col_p - sn col_q,  col_q <- sn col_p + cs col_q.
// The (cs, sn) of every pair of every round go to a log from which
// osj_vectors_kernel accumulates J.  A sweep without a rotation ends the
// iteration (the columns are orthogonal to the test's precision).
//
// osj_kernel (l <= 128, one workgroup): the columns are padded with zeros to
// L = 2^ceil(log2 l) and visited in the resident/traveller order of
// hier_pair.  A group of 16 lanes holds R <= 8 rows of its resident and of
// its current traveller in registers and forms a, b, c with a butterfly
// reduction over the group.  One barrier per round (the traveller hand-over
// through LDS), three per level change.  The big path (l > 128) keeps the
// circle order of the eigensolver.
constexpr int kOsjMaxRows = 8;

// DPP lane permutations inside a row of 16 lanes
constexpr int kDppQuad1032 = 0xB1;  // quad_perm [1, 0, 3, 2]
constexpr int kDppQuad2301 = 0x4E;  // quad_perm [2, 3, 0, 1]
constexpr int kDppRowHalfMirror = 0x141;
constexpr int kDppRowMirror = 0x140;

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over aligned groups of 2^gl2 lanes; the partner of every step is an
// involution, so both lanes of a step add the same two values.
__device__ __forceinline__ double group_sum(double v, int gl2) {
  v += dpp_f64<kDppQuad1032>(v);
  v += dpp_f64<kDppQuad2301>(v);
  if (gl2 >= 3) v += dpp_f64<kDppRowHalfMirror>(v);
  if (gl2 >= 4) v += dpp_f64<kDppRowMirror>(v);
  if (gl2 >= 5) v += __shfl_xor(v, 16);
  if (gl2 >= 6) v += __shfl_xor(v, 32);
  return v;
}

// rotation of the pair with squared norms a, b and inner product c; false
// when the pair already passes the orthogonality test
__device__ __forceinline__ bool osj_rotation(double a, double b, double c, double tol2, double& cs,
                                             double& sn, double& tc) {
  cs = 1.0;
  sn = 0.0;
  tc = 0.0;
  if (!(fabs(c) > 1e-300) || !(c * c > tol2 * a * b)) return false;
  // with d = b - a, e = 2c, h = sqrt(d^2 + e^2) and g = |d| + h the tangent
  // is t = sign(d) e / g, so cs = g / sqrt(2 h g) and sn = sign(d) e / sqrt(2 h g);
  // d and e are first scaled by a power of two to keep d^2 + e^2 in range
  const int ex = __builtin_amdgcn_frexp_exp(fmax(fabs(b - a), fabs(2.0 * c)));
  const double d = __builtin_amdgcn_ldexp(b - a, -ex);
  const double e = __builtin_amdgcn_ldexp(2.0 * c, -ex);
  const double h2 = fma(d, d, e * e);
  const double h = h2 * rsqrt_f64(h2);
  const double g = fabs(d) + h;
  const double r = rsqrt_f64((h + h) * g);
  cs = g * r;
  sn = (d >= 0 ? e : -e) * r;
  // t c with t = sn / cs = sign(d) e / g = sign(d) e 2 h r^2: the rotated
  // squared norms are a - t c and b + t c
  tc = sn * (h + h) * r * c;
  return true;
}

// Sums of a, b, c over each row of 16 lanes, the three reductions in
// lockstep (DPP only; every step's partner is an involution, so both lanes
// of a step add the same two values and the row ends bitwise uniform).
__device__ __forceinline__ void row16_sum3(double& a, double& b, double& c) {
  a += dpp_f64<kDppQuad1032>(a);
  b += dpp_f64<kDppQuad1032>(b);
  c += dpp_f64<kDppQuad1032>(c);
  a += dpp_f64<kDppQuad2301>(a);
  b += dpp_f64<kDppQuad2301>(b);
  c += dpp_f64<kDppQuad2301>(c);
  a += dpp_f64<kDppRowHalfMirror>(a);
  b += dpp_f64<kDppRowHalfMirror>(b);
  c += dpp_f64<kDppRowHalfMirror>(c);
  a += dpp_f64<kDppRowMirror>(a);
  b += dpp_f64<kDppRowMirror>(b);
  c += dpp_f64<kDppRowMirror>(c);
}

__device__ __forceinline__ void row16_sum2(double& a, double& b) {
  a += dpp_f64<kDppQuad1032>(a);
  b += dpp_f64<kDppQuad1032>(b);
  a += dpp_f64<kDppQuad2301>(a);
  b += dpp_f64<kDppQuad2301>(b);
  a += dpp_f64<kDppRowHalfMirror>(a);
  b += dpp_f64<kDppRowHalfMirror>(b);
  a += dpp_f64<kDppRowMirror>(a);
  b += dpp_f64<kDppRowMirror>(b);
}

__device__ __forceinline__ double row16_sum1(double c) {
  c += dpp_f64<kDppQuad1032>(c);
  c += dpp_f64<kDppQuad2301>(c);
  c += dpp_f64<kDppRowHalfMirror>(c);
  return c + dpp_f64<kDppRowMirror>(c);
}

// One group of 16 lanes per pair; lane t holds rows t, t + 16, ...,
// t + 16 (R - 1) of its two columns.  In LDS every column has 16 R entries
// (rows past `rows` are zero and stay zero under rotations), so the round
// loop needs no bounds checks.
template <typename TI, int R>
__global__ __launch_bounds__(kSmallThreads) void osj_kernel(int rows, int l, const TI* __restrict__ M,
                                                            int64_t ldm, double* __restrict__ sigma,
                                                            int* __restrict__ perm,
                                                            double* __restrict__ Ubar,
                                                            double2* __restrict__ rlog,
                                                            int* __restrict__ nrounds,
                                                            int32_t* status, int max_sweeps) {
  // L columns of LD entries (16 R, padded by 128 bytes from R = 2 on so that
  // the columns of neighbouring groups start in opposite halves of the LDS
  // banks): the whole matrix between levels; within a level its two halves
  // are the alternating buffers through which the travellers move
  constexpr int LD = R == 1 ? 16 : 16 * R + 16;
  extern __shared__ double S[];
  __shared__ double nrm[kLdsMaxL];
  __shared__ double cn[kLdsMaxL];  // squared column norms, moved like the columns
  __shared__ int sperm[kLdsMaxL];
  __shared__ int rotated[2];
  const int L = pow2_ceil(l);
  const int P = L / 2;
  const int tid = threadIdx.x, grp = tid >> 4, t = tid & 15;
  double x[R], y[R];  // resident and traveller rows t, t + 16, ...
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int i = t + 16 * k;
    x[k] = (i < rows && grp < l) ? (double)M[i + (int64_t)grp * ldm] : 0.0;
    y[k] = (i < rows && P + grp < l) ? (double)M[i + (int64_t)(P + grp) * ldm] : 0.0;
  }
  if (tid < 2) rotated[tid] = 0;
  __syncthreads();
  const double tol2 = (double)l * 0x1p-104;
  int rounds = 0, sweep = 0;
  bool conv = false;
  // squared norms of the resident (na) and the traveller (nb) column: exact
  // at the start of every sweep, then carried through the rotations (a - t c
  // and b + t c) and summed again when one of them drops below an eighth of
  // its value before the rotation, where the difference would cancel; only
  // the inner product is summed every round
  double na = 0.0, nb = 0.0;
  for (; sweep < max_sweeps && !conv; ++sweep) {
    const int fl = sweep & 1;
    na = 0.0;
    nb = 0.0;
#pragma unroll
    for (int k = 0; k < R; ++k) {
      na = fma(x[k], x[k], na);
      nb = fma(y[k], y[k], nb);
    }
    row16_sum2(na, nb);
    for (int Q = P; Q >= 1; Q >>= 1) {
      const int b = grp / Q, j = grp & (Q - 1);
      for (int u = 0; u < Q; ++u, ++rounds) {
        double c = 0.0;
#pragma unroll
        for (int k = 0; k < R; ++k) c = fma(x[k], y[k], c);
        c = row16_sum1(c);
        double cs, sn, tc;
        const bool rot = osj_rotation(na, nb, c, tol2, cs, sn, tc);
        // a pair that does not rotate has (cs, sn) = (1, 0), whose update
        // reproduces its columns exactly; the wave skips the update only when
        // none of its pairs rotates
        if (__any(rot)) {
#pragma unroll
          for (int k = 0; k < R; ++k) {
            const double xv = x[k], yv = y[k];
            x[k] = fma(cs, xv, -sn * yv);
            y[k] = fma(sn, xv, cs * yv);
          }
          const double na1 = na - tc, nb1 = nb + tc;
          if (__any(na1 < 0.125 * na || nb1 < 0.125 * nb)) {
            na = 0.0;
            nb = 0.0;
#pragma unroll
            for (int k = 0; k < R; ++k) {
              na = fma(x[k], x[k], na);
              nb = fma(y[k], y[k], nb);
            }
            row16_sum2(na, nb);
          } else {
            na = na1;
            nb = nb1;
          }
        }
        if (rot && t == 0) rotated[fl] = 1;
        if (t == 0) rlog[(size_t)rounds * P + grp] = make_double2(cs, sn);
        if (u + 1 < Q) {
          double* buf = S + (size_t)(rounds & 1) * P * LD;
          double* nbuf = cn + (rounds & 1) * P;
          const int dst = b * Q + ((j + Q - 1) & (Q - 1));
#pragma unroll
          for (int k = 0; k < R; ++k) buf[dst * LD + t + 16 * k] = y[k];
          if (t == 0) nbuf[dst] = nb;
          lds_barrier();
#pragma unroll
          for (int k = 0; k < R; ++k) y[k] = buf[grp * LD + t + 16 * k];
          nb = nbuf[grp];
        }
      }
      // end of the level: every column to its place (after the last
      // traveller reads), then the pairs of the next level
      lds_barrier();
      const int pc = 2 * Q * b + j, qc = 2 * Q * b + Q + ((j + Q - 1) & (Q - 1));
#pragma unroll
      for (int k = 0; k < R; ++k) {
        S[pc * LD + t + 16 * k] = x[k];
        S[qc * LD + t + 16 * k] = y[k];
      }
      if (t == 0) {
        cn[pc] = na;
        cn[qc] = nb;
      }
      lds_barrier();
      if (Q == 1) conv = rotated[fl] == 0;  // every flag of the sweep is set by now
      if (conv) break;                      // S holds the final matrix
      const int Q1 = Q > 1 ? Q >> 1 : P;   // next level, or level 0 of the next sweep
      const int b1 = grp / Q1, j1 = grp & (Q1 - 1);
      const int pn = 2 * Q1 * b1 + j1, qn = pn + Q1;
#pragma unroll
      for (int k = 0; k < R; ++k) {
        x[k] = S[pn * LD + t + 16 * k];
        y[k] = S[qn * LD + t + 16 * k];
      }
      na = cn[pn];
      nb = cn[qn];
      lds_barrier();
      if (Q == 1 && tid == 0) rotated[fl] = 0;  // read by all before the barrier above
    }
  }
  if (tid == 0) {
    // the sweep that found no rotation logged identities only
    *nrounds = conv ? rounds - (L - 1) : rounds;
    if (!conv) or_status(status, RMM_STATUS_NOT_CONVERGED);
  }
  {
    // column norms of the final M J: group grp takes columns grp and P + grp
    double a = 0.0, bb = 0.0, c = 0.0;
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const double xv = S[grp * LD + t + 16 * k];
      const double yv = S[(P + grp) * LD + t + 16 * k];
      a = fma(xv, xv, a);
      bb = fma(yv, yv, bb);
    }
    row16_sum3(a, bb, c);
    if (t == 0) {
      nrm[grp] = sqrt(a);
      nrm[P + grp] = sqrt(bb);
    }
  }
  __syncthreads();
  // descending, ties by index
  if (tid < l) {
    const double v = nrm[tid];
    int rank = 0;
    for (int i = 0; i < l; ++i) {
      const double u = nrm[i];
      rank += (u > v) || (u == v && i < tid);
    }
    sigma[rank] = v;
    perm[rank] = tid;
    sperm[rank] = tid;
  }
  __syncthreads();
  for (int e = tid; e < rows * l; e += blockDim.x) {
    const int a = e % rows, rank = e / rows;
    const int j = sperm[rank];
    const double nj = nrm[j];
    Ubar[a + (int64_t)rank * rows] = nj > 0.0 ? S[j * LD + a] / nj : 0.0;
  }
}

// ---- one-sided Jacobi for 128 < l <= 1024: one launch per round ------------------------
//
// Same rotations, test, ordering and stopping rule; M (L x L, column-major)
// lives in the workspace and is rotated in place (a round's pairs are
// disjoint).  One wave per pair, lane i holding rows i, i + 64, ...; the
// sweep's log is applied to the rows of J by big_vectors_kernel.
constexpr int kOsjBigRows = kBigMaxL / 64;

__global__ void osj_big_init_kernel(int l, int L, const double* __restrict__ M, int64_t ldm,
                                    double* __restrict__ Mg, double* __restrict__ Vr,
                                    uint16_t* __restrict__ ptab, uint16_t* __restrict__ qtab,
                                    BigState* st) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int npairs = L / 2;
  if (e < (int64_t)L * L) {
    const int a = (int)(e % L), b = (int)(e / L);
    Mg[e] = (a < l && b < l) ? M[a + (int64_t)b * ldm] : 0.0;
    Vr[e] = (a == b) ? 1.0 : 0.0;  // row-major identity
  }
  if (e < (int64_t)(L - 1) * npairs) {
    int p, q;
    rr_pair((int)(e % npairs), (int)(e / npairs), L, p, q);
    ptab[e] = (uint16_t)p;
    qtab[e] = (uint16_t)q;
  }
  if (e == 0) *st = BigState{0.0, 0, 0, 0, 0};
}

__global__ __launch_bounds__(256) void osj_big_round_kernel(int l, int L, int r, double* __restrict__ Mg,
                                                            const uint16_t* __restrict__ ptab,
                                                            const uint16_t* __restrict__ qtab,
                                                            double2* __restrict__ rlog, BigState* st) {
  if (st->converged) return;
  const int npairs = L / 2;
  const int pair = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (pair >= npairs) return;
  const int p = ptab[(size_t)r * npairs + pair], q = qtab[(size_t)r * npairs + pair];
  double* cp = Mg + (int64_t)p * L;
  double* cq = Mg + (int64_t)q * L;
  double x[kOsjBigRows], y[kOsjBigRows];
  double a = 0.0, b = 0.0, c = 0.0;
#pragma unroll
  for (int k = 0; k < kOsjBigRows; ++k) {
    const int i = lane + 64 * k;
    x[k] = i < L ? cp[i] : 0.0;
    y[k] = i < L ? cq[i] : 0.0;
  }
#pragma unroll
  for (int k = 0; k < kOsjBigRows; ++k) {
    a = fma(x[k], x[k], a);
    b = fma(y[k], y[k], b);
    c = fma(x[k], y[k], c);
  }
  a = group_sum(a, 6);
  b = group_sum(b, 6);
  c = group_sum(c, 6);
  double cs, sn, tc;
  if (osj_rotation(a, b, c, (double)l * 0x1p-104, cs, sn, tc)) {
#pragma unroll
    for (int k = 0; k < kOsjBigRows; ++k) {
      const int i = lane + 64 * k;
      if (i < L) {
        cp[i] = cs * x[k] - sn * y[k];
        cq[i] = sn * x[k] + cs * y[k];
      }
    }
    if (lane == 0) atomicOr(&st->pending, 1);
  }
  if (lane == 0) rlog[(size_t)r * npairs + pair] = make_double2(cs, sn);
}

// converged when the sweep just run rotated nothing; the sweep's log (all
// identities then) is applied only otherwise
__global__ void osj_big_decide_kernel(BigState* st) {
  if (st->converged) return;
  if (st->pending == 0) st->converged = 1;
  else st->sweeps += 1;
  st->pending = 0;
}

// column norms of the rotated M, one wave per column
__global__ __launch_bounds__(256) void osj_big_norms_kernel(int L, const double* __restrict__ Mg,
                                                            double* __restrict__ nrm) {
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= L) return;
  double a = 0.0;
  for (int i = lane; i < L; i += 64) {
    const double v = Mg[i + (int64_t)j * L];
    a = fma(v, v, a);
  }
  a = group_sum(a, 6);
  if (lane == 0) nrm[j] = sqrt(a);
}

// sigma descending (ties by index), Ubar[:, rank] = M[:, j] / sigma, and
// Jout[:, rank] = J[:, j] (J row-major: J[k][j] = Vr[k * L + j])
__global__ void osj_big_finish_kernel(int l, int L, const double* __restrict__ Mg,
                                      const double* __restrict__ nrm, const double* __restrict__ Vr,
                                      double* __restrict__ sigma, double* __restrict__ Ubar,
                                      double* __restrict__ Jout, const BigState* st,
                                      int32_t* status) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j == 0 && !st->converged) or_status(status, RMM_STATUS_NOT_CONVERGED);
  if (j >= l) return;
  const double v = nrm[j];
  int rank = 0;
  for (int i = 0; i < l; ++i) {
    const double u = nrm[i];
    rank += (u > v) || (u == v && i < j);
  }
  sigma[rank] = v;
  const double inv = v > 0.0 ? 1.0 / v : 0.0;
  for (int k = 0; k < l; ++k) {
    Ubar[k + (int64_t)rank * l] = Mg[k + (int64_t)j * L] * inv;
    Jout[k + (int64_t)rank * l] = Vr[(int64_t)k * L + j];
  }
}

size_t jacobi_svd_workspace(int l) {
  const int L = l <= kLdsMaxL ? pow2_ceil(l) : (l + 1) & ~1;
  Carver c(nullptr, 0);
  if (l <= kLdsMaxL) {
    c.take<double2>((size_t)kJacobiMaxSweeps * (L - 1) * (L / 2));
    c.take<int>((size_t)l);
    c.take<int>(1);
    return c.off + 3 * kAlign;
  }
  c.take<double>((size_t)L * L);  // M
  c.take<double>((size_t)L * L);  // J
  c.take<double>((size_t)L);      // norms
  c.take<double2>((size_t)(L - 1) * (L / 2));
  c.take<uint16_t>((size_t)(L - 1) * (L / 2));
  c.take<uint16_t>((size_t)(L - 1) * (L / 2));
  c.take<BigState>(1);
  return c.off + 8 * kAlign;
}

static int jacobi_svd_big(const rmm_ctx* h, int l, const double* M, int64_t ldm, double* sigma,
                          double* Ubar, double* J, int32_t* status, Carver& ws) {
  const int L = (l + 1) & ~1;
  const int npairs = L / 2;
  const size_t mark = ws.off;
  double* Mg = ws.take<double>((size_t)L * L);
  double* Vr = ws.take<double>((size_t)L * L);
  double* nrm = ws.take<double>((size_t)L);
  double2* rlog = ws.take<double2>((size_t)(L - 1) * npairs);
  uint16_t* ptab = ws.take<uint16_t>((size_t)(L - 1) * npairs);
  uint16_t* qtab = ws.take<uint16_t>((size_t)(L - 1) * npairs);
  BigState* st = ws.take<BigState>(1);
  if (!ws.fits()) return RMM_ERR_WORKSPACE_TOO_SMALL;
  const int64_t init_n = (int64_t)L * L;
  hipLaunchKernelGGL(osj_big_init_kernel, dim3((unsigned)((init_n + 255) / 256)), dim3(256), 0,
                     h->stream, l, L, M, ldm, Mg, Vr, ptab, qtab, st);
  RMM_TRY(launch_status());
  const size_t vlds = (size_t)4 * kBigVecRows * L * sizeof(double);
  RMM_HIP(hipFuncSetAttribute((const void*)big_vectors_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)vlds));
  const unsigned vgroups = (unsigned)((L + 4 * kBigVecRows - 1) / (4 * kBigVecRows));
  const unsigned rgroups = (unsigned)((npairs + 3) / 4);
  for (int sweep = 0; sweep < kBigMaxSweeps; ++sweep) {
    for (int r = 0; r < L - 1; ++r)
      hipLaunchKernelGGL(osj_big_round_kernel, dim3(rgroups), dim3(256), 0, h->stream, l, L, r, Mg,
                         ptab, qtab, rlog, st);
    RMM_TRY(launch_status());
    hipLaunchKernelGGL(osj_big_decide_kernel, dim3(1), dim3(1), 0, h->stream, st);
    hipLaunchKernelGGL(big_vectors_kernel, dim3(vgroups), dim3(256), vlds, h->stream, L, rlog, ptab,
                       qtab, Vr, st);
    RMM_TRY(launch_status());
  }
  hipLaunchKernelGGL(osj_big_norms_kernel, dim3((unsigned)((L + 3) / 4)), dim3(256), 0, h->stream, L,
                     Mg, nrm);
  hipLaunchKernelGGL(osj_big_finish_kernel, dim3((unsigned)((l + 255) / 256)), dim3(256), 0,
                     h->stream, l, L, Mg, nrm, Vr, sigma, Ubar, J, st, status);
  ws.off = mark;
  return launch_status();
}

// Direct one-sided Jacobi on a tall X (rows <= 128, rows <= 2 L): every
// round moves half the matrix through LDS, so beyond that the QR route is
// cheaper.
bool jacobi_svd_direct_ok(int64_t rows, int l) {
  if (l > kLdsMaxL || rows < l) return false;
  return rows <= kLdsMaxL && rows <= 2 * (int64_t)pow2_ceil(l);
}

template <typename TI, int R>
static int osj_launch_r(const rmm_ctx* h, int rows, int l, const TI* M, int64_t ldm, double* sigma,
                        int* perm, double* Ubar, double2* rlog, int* nr, int32_t* status) {
  const int L = pow2_ceil(l);
  const size_t lds = (size_t)L * (R == 1 ? 16 : 16 * R + 16) * sizeof(double);
  RMM_HIP(hipFuncSetAttribute((const void*)osj_kernel<TI, R>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL((osj_kernel<TI, R>), dim3(1), dim3(L / 2 * 16), lds, h->stream, rows, l, M, ldm,
                     sigma, perm, Ubar, rlog, nr, status, kJacobiMaxSweeps);
  return launch_status();
}

template <typename TI>
static int osj_launch(const rmm_ctx* h, int rows, int l, const TI* M, int64_t ldm, double* sigma,
                      double* Ubar, double* J, int32_t* status, Carver& ws) {
  const int L = pow2_ceil(l);
  const int P = L / 2;
  const size_t mark = ws.off;
  double2* rlog = ws.take<double2>((size_t)kJacobiMaxSweeps * (L - 1) * P);
  int* perm = ws.take<int>((size_t)l);
  int* nr = ws.take<int>(1);
  if (!ws.fits()) return RMM_ERR_WORKSPACE_TOO_SMALL;
  if (rows <= 16)
    RMM_TRY((osj_launch_r<TI, 1>(h, rows, l, M, ldm, sigma, perm, Ubar, rlog, nr, status)));
  else if (rows <= 32)
    RMM_TRY((osj_launch_r<TI, 2>(h, rows, l, M, ldm, sigma, perm, Ubar, rlog, nr, status)));
  else if (rows <= 64)
    RMM_TRY((osj_launch_r<TI, 4>(h, rows, l, M, ldm, sigma, perm, Ubar, rlog, nr, status)));
  else
    RMM_TRY((osj_launch_r<TI, 8>(h, rows, l, M, ldm, sigma, perm, Ubar, rlog, nr, status)));
  const int groups = (l + 4 * kOsjVecRows - 1) / (4 * kOsjVecRows);
  hipLaunchKernelGGL(osj_vectors_kernel, dim3(groups), dim3(256), 0, h->stream, l, rlog, nr, perm, J);
  ws.off = mark;
  return launch_status();
}

int jacobi_svd(const rmm_ctx* h, int l, const double* M, int64_t ldm, double* sigma, double* Ubar,
               double* J, int32_t* status, Carver& ws) {
  if (l == 0) return RMM_OK;
  if (l > kBigMaxL) return RMM_ERR_UNSUPPORTED;
  if (l > kLdsMaxL) return jacobi_svd_big(h, l, M, ldm, sigma, Ubar, J, status, ws);
  return osj_launch<double>(h, l, l, M, ldm, sigma, Ubar, J, status, ws);
}

template <typename TI>
int jacobi_svd_direct(const rmm_ctx* h, int64_t rows, int l, const TI* X, int64_t ldx, double* sigma,
                      double* Ux, double* J, int32_t* status, Carver& ws) {
  if (l == 0) return RMM_OK;
  if (!jacobi_svd_direct_ok(rows, l)) return RMM_ERR_UNSUPPORTED;
  return osj_launch<TI>(h, (int)rows, l, X, ldx, sigma, Ux, J, status, ws);
}

template int jacobi_svd_direct<float>(const rmm_ctx*, int64_t, int, const float*, int64_t, double*,
                                      double*, double*, int32_t*, Carver&);
template int jacobi_svd_direct<double>(const rmm_ctx*, int64_t, int, const double*, int64_t, double*,
                                       double*, double*, int32_t*, Carver&);

// G_jj += c * trace(G) for the l x l matrix G (one workgroup): the shift of
// the first pass of shifted CholeskyQR
__global__ __launch_bounds__(256) void shift_diag_kernel(int l, double* __restrict__ G, int64_t ldg,
                                                         double c) {
  __shared__ double red[256];
  double s = 0.0;
  for (int j = threadIdx.x; j < l; j += 256) s += G[j + (int64_t)j * ldg];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  const double sh = c * red[0];
  for (int j = threadIdx.x; j < l; j += 256) G[j + (int64_t)j * ldg] += sh;
}

int shift_diag(const rmm_ctx* h, int l, double* G, int64_t ldg, double c) {
  if (l == 0) return RMM_OK;
  hipLaunchKernelGGL(shift_diag_kernel, dim3(1), dim3(256), 0, h->stream, l, G, ldg, c);
  return launch_status();
}

// ---- sign convention, small glue -------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(1024) void sign_fix_kernel(int64_t m, int64_t n, T* __restrict__ U,
                                                        int64_t ldu, T* __restrict__ V, int64_t ldv) {
  // argmax |u_i| with the lowest index on ties: each thread scans its rows in
  // increasing order, four independent loads per step, then a tree reduction
  __shared__ double bv[1024];
  __shared__ int64_t bi[1024];
  const int64_t c = blockIdx.x;
  T* u = U + c * ldu;
  double best = -1.0;
  int64_t besti = 0;
  for (int64_t i0 = threadIdx.x; i0 < m; i0 += 4096) {
    double a[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t i = i0 + 1024 * e;
      a[e] = i < m ? fabs((double)u[i]) : -1.0;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (a[e] > best) { best = a[e]; besti = i0 + 1024 * e; }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = besti;
  __syncthreads();
  for (int st = 512; st > 0; st >>= 1) {
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
  for (int64_t i = threadIdx.x; i < m; i += blockDim.x) u[i] = -u[i];
  T* v = V + c * ldv;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) v[i] = -v[i];
}

template <typename T>
int sign_fix(const rmm_ctx* h, int64_t m, int64_t n, int k, T* U, int64_t ldu, T* V, int64_t ldv) {
  if (k == 0) return RMM_OK;
  hipLaunchKernelGGL((sign_fix_kernel<T>), dim3(k), dim3(1024), 0, h->stream, m, n, U, ldu, V, ldv);
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

// x = R y for upper triangular R (d x d, ld d).  A workgroup owns 64 rows
// (one per lane); its 16 waves take every 16th column from the first owned
// row on, so a wave's loads of R are 512-byte column segments, and the 16
// partial sums of a row are added in wave order through LDS.
constexpr int kTrmvWaves = 16;

__global__ __launch_bounds__(64 * kTrmvWaves) void trmv_upper_kernel(
    int d, const double* __restrict__ R, const double* __restrict__ y, double* __restrict__ x) {
  __shared__ double part[kTrmvWaves][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i0 = blockIdx.x * 64;
  const int i = i0 + lane;
  const int ir = i < d ? i : d - 1;  // rows past d read a valid row and are not stored
  double acc = 0.0;
#pragma unroll 4
  for (int c = i0 + w; c < d; c += kTrmvWaves) {
    const double r = R[ir + (int64_t)c * d];
    acc = fma(c >= i ? r : 0.0, y[c], acc);
  }
  part[w][lane] = acc;
  __syncthreads();
  if (w == 0 && i < d) {
    double s = 0.0;
#pragma unroll
    for (int v = 0; v < kTrmvWaves; ++v) s += part[v][lane];
    x[i] = s;
  }
}

int trmv_upper(const rmm_ctx* h, int d, const double* Rinv, const double* y, double* x) {
  if (d == 0) return RMM_OK;
  hipLaunchKernelGGL(trmv_upper_kernel, dim3((d + 63) / 64), dim3(64 * kTrmvWaves), 0, h->stream, d,
                     Rinv, y, x);
  return launch_status();
}

template int sign_fix<float>(const rmm_ctx*, int64_t, int64_t, int, float*, int64_t, float*, int64_t);
template int sign_fix<double>(const rmm_ctx*, int64_t, int64_t, int, double*, int64_t, double*, int64_t);

}  // namespace rmm
