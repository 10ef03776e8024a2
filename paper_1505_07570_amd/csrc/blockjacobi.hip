// Block cyclic Jacobi eigensolver for symmetric l x l matrices, 128 < l <= 1024
// (the c x c matrix W = K[S, S] of the Nystrom method).
//
// The index set is cut into nb blocks of 32 (padded with zero rows and
// columns, which never rotate).  One sweep visits every pair of indices
// once, in two kinds of steps:
//   * intra step: the blocks, paired as (0, 1), (2, 3), ..., each rotate the
//     pairs inside themselves in 31 rounds of 16 disjoint rotations (a
//     hierarchical order: the two halves of 16 against each other in 16
//     rounds, then the quarters of each half in 8, and so on);
//   * nb - 1 cross steps: the blocks are paired by the circle method and each
//     pair (I, J) rotates every (i in I, j in J) in 32 rounds of 32 disjoint
//     rotations (i against j = (i + round) mod 32 of J).
// A step works on the 64 x 64 subproblem W[IJ, IJ] (IJ = I u J) in LDS:
// rotation angles and the rotation test are those of the scalar solver, and
// the product Q of the step's rotations, re-orthogonalized, is applied to
// the whole matrix afterwards by tiles, W[IJ, IJ'] <- Q^T W[IJ, IJ'] Q' and
// V[:, IJ] <- V[:, IJ] Q (all pairs of a step at once: their index sets are
// disjoint).  So W <- P^T W P and V <- V P with P block orthogonal.
// Before each sweep a scan decides convergence (no off-diagonal element
// passes the rotation test: the scalar solver's relative test, plus an
// absolute floor of 2^-52 ||W||_F, the rounding level of the block updates).  Then the
// eigenvalues (the diagonal, descending, ties by index) and V's columns are
// sorted out.
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

// abs_tol = 2^-52 ||W||_F.  The block updates apply re-orthogonalized
// products of rotations with full 64 x 64 products, so every step leaves
// rounding of order eps ||W|| in the entries it touches (the backward error
// of an orthogonal similarity); off-diagonal entries at that level carry no
// information and are not rotated.  Without this floor a cluster of
// numerically zero eigenvalues (repeated points) would be rotated forever:
// its large-angle rotations smear the rounding of the large eigenvalues back
// into it.  The relative test of the scalar solver applies on top.  Partial
// sums per column group, then one thread adds them in a fixed order (the
// threshold is reproducible).
constexpr int kTolGroups = 128;

// part[x] = sum of the squares of columns x, x + kTolGroups, ... of W
__global__ __launch_bounds__(256) void blk_fro_part_kernel(int l, int L, const double* __restrict__ W,
                                                           double* __restrict__ part) {
  __shared__ double red[256];
  double ss = 0.0;
  for (int b = blockIdx.x; b < l; b += kTolGroups)
    for (int a = threadIdx.x; a < l; a += 256) {
      const double v = W[a + (int64_t)b * L];
      ss = fma(v, v, ss);
    }
  red[threadIdx.x] = ss;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void blk_tol_kernel(const double* __restrict__ part, BlkState* st) {
  if (threadIdx.x != 0) return;
  double ss = 0.0;
  for (int x = 0; x < kTolGroups; ++x) ss += part[x];  // fixed order: reproducible
  st->abs_tol = 0x1p-52 * sqrt(ss);
}

__device__ __forceinline__ bool rot_test(double gpq, double gpp, double gqq, double abs_tol) {
  return fabs(gpq) > abs_tol && fabs(gpq) > 1e-300 && gpq * gpq > 0x1p-104 * fabs(gpp * gqq);
}

// Reciprocal and reciprocal square root from the hardware seeds refined by
// two Newton steps (a few ulps; the rotations they feed are re-orthogonalized
// as a product, so correct rounding is not needed).
__device__ __forceinline__ double rcp_nr(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  return fma(r, fma(-d, r, 1.0), r);
}

__device__ __forceinline__ double rsq_nr(double x) {
  const double h = 0.5 * x;
  double y = __builtin_amdgcn_rsq(x);
  y = fma(y, fma(-h * y, y, 0.5), y);
  return fma(y, fma(-h * y, y, 0.5), y);
}

// Rotation annihilating gpq of [[gpp, gpq], [gpq, gqq]] when it passes the
// rotation test (else c = 1, s = t = 0): theta = (gqq - gpp) / (2 gpq),
// t = sign(theta) / (|theta| + sqrt(theta^2 + 1)), c = 1 / sqrt(t^2 + 1),
// s = t c.  For |theta| > 2^500, t = 1 / (2 theta) (theta^2 would overflow;
// |theta| is capped at 2^1000 so that t stays finite and nonzero-safe).
__device__ __forceinline__ void jacobi_rotation(double gpq, double gpp, double gqq, double abs_tol, double& c,
                                                double& s, double& t) {
  const bool rot = rot_test(gpq, gpp, gqq, abs_tol);
  const double y = rot ? 2.0 * gpq : 1.0;
  const double theta = (gqq - gpp) * rcp_nr(y);
  const double at = fabs(theta);
  const bool big = at > 0x1p500;
  const double u = fma(theta, theta, 1.0);
  const double den = big ? 2.0 * fmin(at, 0x1p1000) : at + u * rsq_nr(big ? 1.0 : u);
  const double tt = copysign(rcp_nr(den), theta);
  const double cc = rsq_nr(fma(tt, tt, 1.0));
  t = rot ? tt : 0.0;
  c = rot ? cc : 1.0;
  s = rot ? tt * cc : 0.0;
}

// pending |= an off-diagonal element (a < b < l) passes the rotation test.
// One atomic per wave that finds one; workgroups starting after pending is
// set skip their reads (a stale read only costs the scan).
// Workgroup x scans columns b = x, x + G, ... (G workgroups) with the
// diagonal in LDS.
__global__ __launch_bounds__(256) void blk_scan_kernel(int l, int L, const double* __restrict__ W,
                                                       BlkState* st) {
  if (st->converged || st->pending) return;
  __shared__ double dg[1024];
  for (int i = threadIdx.x; i < l; i += 256) dg[i] = W[i + (int64_t)i * L];
  __syncthreads();
  const double tol = st->abs_tol;
  bool pass = false;
  for (int b = blockIdx.x; b < l; b += gridDim.x)
    for (int a = threadIdx.x; a < b; a += 256) pass |= rot_test(W[a + (int64_t)b * L], dg[a], dg[b], tol);
  if (__any(pass) && (threadIdx.x & 63) == 0) atomicOr(&st->pending, 1);
}

__global__ void blk_decide_kernel(BlkState* st) {
  if (st->converged) return;
  if (st->pending == 0) st->converged = 1;
  else st->sweeps += 1;
  st->pending = 0;
}

// Blocks of step pair x: cross steps pair the blocks by the circle method
// (round r), intra steps take (2x, 2x + 1).
template <int MODE>
__device__ __forceinline__ void step_blocks(int x, int r, int nb, int& bi, int& bj) {
  if (MODE == 0) {
    circle_pair(x, r, nb, bi, bj);
  } else {
    bi = 2 * x;
    bj = 2 * x + 1;
  }
}

// Rotation u (0..31) of round rr of a step on a 64-index subproblem (local
// indices 0..31 = block I, 32..63 = block J).  Cross (MODE 0, 32 rounds):
// (u, 32 + (u + rr) mod 32).  Intra (MODE 1, 31 rounds): inside each half of
// 32, at level h = 16, 8, 4, 2, 1 the groups of 2h split into two halves of
// h, index a of the first half against (a + rho) mod h of the second, rho <
// h.
constexpr int kCrossRounds = kBB;
constexpr int kIntraRounds = kBB - 1;

template <int MODE>
__device__ __forceinline__ void step_pair(int u, int rr, int& p, int& q) {
  if (MODE == 0) {
    p = u;
    q = kBB + ((u + rr) & (kBB - 1));
    return;
  }
  int lh, rho;  // log2 h, round within the level
  if (rr < 16) { lh = 4; rho = rr; }
  else if (rr < 24) { lh = 3; rho = rr - 16; }
  else if (rr < 28) { lh = 2; rho = rr - 24; }
  else if (rr < 30) { lh = 1; rho = rr - 28; }
  else { lh = 0; rho = 0; }
  const int h = 1 << lh;
  const int half = u >> 4, w = u & 15;
  const int base = half * kBB + ((w >> lh) << (lh + 1));
  const int a = w & (h - 1);
  p = base + a;
  q = base + h + ((a + rho) & (h - 1));
}

// Step kernel: the rounds of one step on the subproblem of step pair
// blockIdx.x; D = Q - I (64 x 64, column-major) to Dbuf[pair].
//
// Thread (u = tid mod 32, g = tid / 32) computes rotation u of each round
// and updates the 2 x 2 blocks (u, v) of the subproblem, v = g + kStepG m
// for m < kStepM (rows {p_u, q_u}, columns {p_v, q_v}: every element once),
// and rows u and u + 32 of Q at the column pairs v; rotation v comes from
// lane v of the same wave.  The subproblem is double-buffered in LDS (read
// one, write the other), so one barrier per round suffices.  A round is a
// short dependent chain (LDS reads, the rotation, the shuffles, the 2 x 2
// updates), so several waves per SIMD share the blocks to hide its latency.
constexpr int kStepM = 2;                    // blocks (u, v) per thread
constexpr int kStepG = kBB / kStepM;         // thread groups of 32
constexpr int kStepThreads = kBB * kStepG;
constexpr int kStepLoads = kBS * kBS / kStepThreads;
constexpr int kStepCols = kBS * kBS / (4 * kStepThreads);  // epilogue: 4 rows x kStepCols columns per thread

template <int MODE>
__global__ __launch_bounds__(kStepThreads) void blk_step_kernel(int nb, int r, int L, const double* __restrict__ W,
                                                                double* __restrict__ Dbuf, const BlkState* st) {
  if (st->converged) return;
  __shared__ double S[2][kBS * kBLd];
  __shared__ double Q[kBS * kBLd];
  const int tid = threadIdx.x;
  int bi, bj;
  step_blocks<MODE>(blockIdx.x, r, nb, bi, bj);
  {
    double v[kStepLoads];  // all loads in flight before the LDS stores
#pragma unroll
    for (int k = 0; k < kStepLoads; ++k) {
      const int e = tid + kStepThreads * k, a = e % kBS, b = e / kBS;
      v[k] = W[gidx(a, bi, bj) + (int64_t)gidx(b, bi, bj) * L];
    }
#pragma unroll
    for (int k = 0; k < kStepLoads; ++k) {
      const int e = tid + kStepThreads * k, a = e % kBS, b = e / kBS;
      S[0][a + b * kBLd] = v[k];
      Q[a + b * kBLd] = a == b ? 1.0 : 0.0;
    }
  }
  __syncthreads();
  const double abs_tol = st->abs_tol;
  const int u = tid & 31, g = tid >> 5;
  constexpr int rounds = MODE == 0 ? kCrossRounds : kIntraRounds;
  // In cross steps p_u = u and p_v = v in every round, so the block I x I
  // entries S[u][v] and the entries Q[u][v], Q[u + 32][v] of a thread never
  // change owner: they stay in registers (only S[u][u], which the rotation
  // of pair u reads, also goes to LDS each round).
  double ii[kStepM], qi[kStepM][2];
  if constexpr (MODE == 0) {
#pragma unroll
    for (int m = 0; m < kStepM; ++m) {
      const int v = g + kStepG * m;
      ii[m] = S[0][u + v * kBLd];
      qi[m][0] = u == v ? 1.0 : 0.0;
      qi[m][1] = 0.0;  // row u + 32 >= 32 > v
    }
  }
  for (int rr = 0; rr < rounds; ++rr) {
    const double* Sc = S[rr & 1];
    double* Sn = S[(rr & 1) ^ 1];
    int p, q, pv[kStepM], qv[kStepM];
    step_pair<MODE>(u, rr, p, q);
#pragma unroll
    for (int m = 0; m < kStepM; ++m) step_pair<MODE>(g + kStepG * m, rr, pv[m], qv[m]);
    // every LDS read of the round first (the compiler cannot tell the stores
    // below from these addresses)
    const double gpq = Sc[p + q * kBLd], gpp = Sc[p + p * kBLd], gqq = Sc[q + q * kBLd];
    double x[kStepM][4], y[kStepM][2][2];
#pragma unroll
    for (int m = 0; m < kStepM; ++m) {
      x[m][0] = MODE == 0 ? ii[m] : Sc[p + pv[m] * kBLd];
      x[m][1] = Sc[p + qv[m] * kBLd];
      x[m][2] = Sc[q + pv[m] * kBLd];
      x[m][3] = Sc[q + qv[m] * kBLd];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        y[m][h][0] = MODE == 0 ? qi[m][h] : Q[u + 32 * h + pv[m] * kBLd];
        y[m][h][1] = Q[u + 32 * h + qv[m] * kBLd];
      }
    }
    double c, s, t;
    jacobi_rotation(gpq, gpp, gqq, abs_tol, c, s, t);
    double cv[kStepM], sv[kStepM];
#pragma unroll
    for (int m = 0; m < kStepM; ++m) {
      cv[m] = __shfl(c, g + kStepG * m);
      sv[m] = __shfl(s, g + kStepG * m);
    }
    // blocks (u, v): R_u^T X R_v; the rotated block itself (v = u) takes the
    // scalar solver's update.  A zero rotation (c = 1, s = 0) leaves values
    // unchanged exactly, so nothing branches on it.
#pragma unroll
    for (int m = 0; m < kStepM; ++m) {
      const double y00 = c * x[m][0] - s * x[m][2], y01 = c * x[m][1] - s * x[m][3];
      const double y10 = s * x[m][0] + c * x[m][2], y11 = s * x[m][1] + c * x[m][3];
      double z00 = cv[m] * y00 - sv[m] * y01, z01 = sv[m] * y00 + cv[m] * y01;
      double z10 = cv[m] * y10 - sv[m] * y11, z11 = sv[m] * y10 + cv[m] * y11;
      if (g + kStepG * m == u) {
        const bool rot = s != 0.0;
        z00 = rot ? x[m][0] - t * x[m][1] : x[m][0];
        z11 = rot ? x[m][3] + t * x[m][1] : x[m][3];
        z01 = rot ? 0.0 : x[m][1];
        z10 = rot ? 0.0 : x[m][2];
      }
      if constexpr (MODE == 0) {
        ii[m] = z00;
        if (g + kStepG * m == u) Sn[p + pv[m] * kBLd] = z00;
      } else {
        Sn[p + pv[m] * kBLd] = z00;
      }
      Sn[p + qv[m] * kBLd] = z01;
      Sn[q + pv[m] * kBLd] = z10;
      Sn[q + qv[m] * kBLd] = z11;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const double qp = cv[m] * y[m][h][0] - sv[m] * y[m][h][1];
        if constexpr (MODE == 0) qi[m][h] = qp;
        else Q[u + 32 * h + pv[m] * kBLd] = qp;
        Q[u + 32 * h + qv[m] * kBLd] = sv[m] * y[m][h][0] + cv[m] * y[m][h][1];
      }
    }
    __syncthreads();
  }
  if constexpr (MODE == 0) {
#pragma unroll
    for (int m = 0; m < kStepM; ++m)
#pragma unroll
      for (int h = 0; h < 2; ++h) Q[u + 32 * h + (g + kStepG * m) * kBLd] = qi[m][h];
    __syncthreads();
  }
  // Each rotation is orthogonal only to rounding, and so is Q, their product;
  // applied again and again that drift would scale the eigenvalues.  So Q is
  // re-orthogonalized, Q <- Q (I - E / 2) with E = Q^T Q - I (orthogonal to
  // second order in E), and stored as D = Q - I: the updates then add a
  // small correction D^T W or W D to W, rounding relative to its size.
  double* E = S[0];
  const int a1 = tid & 15, b0 = (tid >> 4) * kStepCols;  // rows a1 + 16 i, columns b0 + j
  double acc[4][kStepCols] = {};
  for (int t = 0; t < kBS; ++t) {
    double qa[4], qb[kStepCols];
#pragma unroll
    for (int i = 0; i < 4; ++i) qa[i] = Q[t + (a1 + 16 * i) * kBLd];
#pragma unroll
    for (int j = 0; j < kStepCols; ++j) qb[j] = Q[t + (b0 + j) * kBLd];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < kStepCols; ++j) acc[i][j] = fma(qa[i], qb[j], acc[i][j]);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < kStepCols; ++j) {
      E[a1 + 16 * i + (b0 + j) * kBLd] = acc[i][j] - (a1 + 16 * i == b0 + j ? 1.0 : 0.0);
      acc[i][j] = 0.0;
    }
  __syncthreads();
  for (int t = 0; t < kBS; ++t) {
    double qa[4], eb[kStepCols];
#pragma unroll
    for (int i = 0; i < 4; ++i) qa[i] = Q[a1 + 16 * i + t * kBLd];
#pragma unroll
    for (int j = 0; j < kStepCols; ++j) eb[j] = E[t + (b0 + j) * kBLd];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < kStepCols; ++j) acc[i][j] = fma(qa[i], eb[j], acc[i][j]);
  }
  double* out = Dbuf + (size_t)blockIdx.x * kBS * kBS;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < kStepCols; ++j) {
      const int a = a1 + 16 * i, b = b0 + j;
      out[a + b * kBS] = (Q[a + b * kBLd] - (a == b ? 1.0 : 0.0)) - 0.5 * acc[i][j];
    }
}

// Update of W and V after a step: W <- P^T W P, V <- V P with P the block
// orthogonal matrix of the step's Q = I + D.  Workgroup (x, y): for y < np
// the W tile (rows IJ_y, columns IJ_x), Z = (I + D_y)^T X (I + D_x) formed
// as Y = X + D_y^T X, Z = Y + Y D_x; for y >= np the V tile (rows
// 64 (y - np) .. + 64, columns IJ_x), Z = X + X D_x.  The tiles partition W
// and V, so each is updated in place.  Thread (a1 = tid mod 16,
// b0 = 4 (tid / 16)) owns rows a1, a1 + 16, a1 + 32, a1 + 48 and columns
// b0 .. b0 + 3 of the tile; per summation index that is one read per owned
// row and two 16-byte reads of the owned columns.
constexpr int kULd = kBS + 2;  // even: 16-byte aligned rows; 2-way bank conflicts on the fills

template <int MODE>
__global__ __launch_bounds__(256) void blk_update_kernel(int nb, int r, int L, double* __restrict__ W,
                                                         double* __restrict__ V, const double* __restrict__ Dbuf,
                                                         const BlkState* st) {
  if (st->converged) return;
  __shared__ __align__(16) double B0[kBS * kULd];
  __shared__ __align__(16) double B1[kBS * kULd];
  const int np = nb / 2;
  const int tid = threadIdx.x, a1 = tid & 15, b0 = (tid >> 4) * 4;
  int xi, xj;
  step_blocks<MODE>(blockIdx.x, r, nb, xi, xj);
  const double* Dx = Dbuf + (size_t)blockIdx.x * kBS * kBS;
  double yv[4][4];
  double* X;
  int64_t row_of[4];  // global row of owned row i
  if ((int)blockIdx.y < np) {
    int yi, yj;
    step_blocks<MODE>(blockIdx.y, r, nb, yi, yj);
    const double* Dy = Dbuf + (size_t)blockIdx.y * kBS * kBS;
    X = W;
    // B0[b + t ld] = X(t, b) = W[IJ_y(t), IJ_x(b)], B1[a + t ld] = D_y(t, a)
    {
      double v[16], d[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int e = tid + 256 * k, t = e % kBS, b = e / kBS;
        v[k] = W[gidx(t, yi, yj) + (int64_t)gidx(b, xi, xj) * L];
        d[k] = Dy[e];
      }
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int e = tid + 256 * k, t = e % kBS, b = e / kBS;
        B0[b + t * kULd] = v[k];
        B1[b + t * kULd] = d[k];
      }
    }
    __syncthreads();
    double acc[4][4] = {};
    for (int t = 0; t < kBS; ++t) {
      double da[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) da[i] = B1[a1 + 16 * i + t * kULd];
      const double2 x01 = *reinterpret_cast<const double2*>(B0 + b0 + t * kULd);
      const double2 x23 = *reinterpret_cast<const double2*>(B0 + b0 + 2 + t * kULd);
      const double xb[4] = {x01.x, x01.y, x23.x, x23.y};
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(da[i], xb[j], acc[i][j]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      row_of[i] = gidx(a1 + 16 * i, yi, yj);
#pragma unroll
      for (int j = 0; j < 4; ++j) yv[i][j] = B0[b0 + j + (a1 + 16 * i) * kULd] + acc[i][j];
    }
    __syncthreads();
    // B0[a + t ld] = Y(a, t), B1[b + t ld] = D_x(t, b)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) B0[a1 + 16 * i + (b0 + j) * kULd] = yv[i][j];
    {
      double d[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) d[k] = Dx[tid + 256 * k];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int e = tid + 256 * k, t = e % kBS, b = e / kBS;
        B1[b + t * kULd] = d[k];
      }
    }
    __syncthreads();
  } else {
    const int r0 = ((int)blockIdx.y - np) * kBS;
    X = V;
    // B0[a + t ld] = V[r0 + a, IJ_x(t)], B1[b + t ld] = D_x(t, b)
    {
      double v[16], d[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int e = tid + 256 * k, a = e % kBS, t = e / kBS;
        v[k] = V[(r0 + a) + (int64_t)gidx(t, xi, xj) * L];
        d[k] = Dx[e];
      }
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int e = tid + 256 * k, a = e % kBS, t = e / kBS;
        B0[a + t * kULd] = v[k];
        B1[t + a * kULd] = d[k];
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      row_of[i] = r0 + a1 + 16 * i;
#pragma unroll
      for (int j = 0; j < 4; ++j) yv[i][j] = B0[a1 + 16 * i + (b0 + j) * kULd];
    }
  }
  double acc[4][4] = {};
  for (int t = 0; t < kBS; ++t) {
    double ya[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) ya[i] = B0[a1 + 16 * i + t * kULd];
    const double2 d01 = *reinterpret_cast<const double2*>(B1 + b0 + t * kULd);
    const double2 d23 = *reinterpret_cast<const double2*>(B1 + b0 + 2 + t * kULd);
    const double db[4] = {d01.x, d01.y, d23.x, d23.y};
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = fma(ya[i], db[j], acc[i][j]);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) X[row_of[i] + (int64_t)gidx(b0 + j, xi, xj) * L] = yv[i][j] + acc[i][j];
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
  c.take<double>((size_t)kTolGroups);             // partial sums of ||W||_F^2
  return c.off + 6 * kAlign;
}

namespace {

// Enqueue one step (rotations, then the update of W and V) of all pairs.
template <int MODE>
int enqueue_step(const rmm_ctx* h, int nb, int r, int L, double* W, double* Vw, double* Db, BlkState* st) {
  const unsigned np = (unsigned)(nb / 2);
  hipLaunchKernelGGL(blk_step_kernel<MODE>, dim3(np), dim3(kStepThreads), 0, h->stream, nb, r, L, W, Db, st);
  hipLaunchKernelGGL(blk_update_kernel<MODE>, dim3(np, 2 * np), dim3(256), 0, h->stream, nb, r, L, W, Vw, Db,
                     st);
  return launch_status();
}

struct EventPair {
  hipEvent_t e[2] = {nullptr, nullptr};
  ~EventPair() {
    for (hipEvent_t x : e)
      if (x) (void)hipEventDestroy(x);
  }
};

}  // namespace

int jacobi_eig_block(const rmm_ctx* h, int l, const double* G, int64_t ldg, double* evals, double* V,
                     int32_t* status, Carver& ws) {
  if (l > 1024) return RMM_ERR_UNSUPPORTED;  // the scan's LDS copy of the diagonal
  const int nb = ((l + kBB - 1) / kBB + 1) & ~1;
  const int L = nb * kBB;
  const int np = nb / 2;
  const size_t mark = ws.off;
  double* W = ws.take<double>((size_t)L * L);
  double* Vw = ws.take<double>((size_t)L * L);
  double* Db = ws.take<double>((size_t)np * kBS * kBS);
  BlkState* st = ws.take<BlkState>(1);
  int* perm = ws.take<int>((size_t)l);
  double* part = ws.take<double>((size_t)kTolGroups);
  if (!ws.fits()) return RMM_ERR_WORKSPACE_TOO_SMALL;
  const int64_t LL = (int64_t)L * L;
  hipLaunchKernelGGL(blk_init_kernel, dim3((unsigned)((LL + 255) / 256)), dim3(256), 0, h->stream, l, L,
                     G, ldg, W, Vw, st);
  hipLaunchKernelGGL(blk_fro_part_kernel, dim3(kTolGroups), dim3(256), 0, h->stream, l, L, W, part);
  hipLaunchKernelGGL(blk_tol_kernel, dim3(1), dim3(64), 0, h->stream, part, st);
  RMM_TRY(launch_status());
  // Sweeps stop on the device once converged (later launches return at
  // once).  Outside stream capture the host also stops enqueueing them: each
  // sweep's decision is copied to pinned host memory and read one sweep
  // later, so the device always has a sweep queued meanwhile.
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  RMM_HIP(hipStreamIsCapturing(h->stream, &cap));
  EventPair ev;
  const bool early = h->hflag && cap == hipStreamCaptureStatusNone &&
                     hipEventCreateWithFlags(&ev.e[0], hipEventDisableTiming) == hipSuccess &&
                     hipEventCreateWithFlags(&ev.e[1], hipEventDisableTiming) == hipSuccess;
  const dim3 sgrid((unsigned)(l < 256 ? l : 256));
  for (int sweep = 0; sweep <= kBMaxSweeps; ++sweep) {
    hipLaunchKernelGGL(blk_scan_kernel, sgrid, dim3(256), 0, h->stream, l, L, W, st);
    hipLaunchKernelGGL(blk_decide_kernel, dim3(1), dim3(1), 0, h->stream, st);
    RMM_TRY(launch_status());
    if (sweep == kBMaxSweeps) break;  // the last scan only decides convergence
    if (early) {
      RMM_HIP(hipMemcpyAsync(h->hflag + (sweep & 1), &st->converged, sizeof(int), hipMemcpyDeviceToHost,
                             h->stream));
      RMM_HIP(hipEventRecord(ev.e[sweep & 1], h->stream));
      if (sweep > 0) {
        RMM_HIP(hipEventSynchronize(ev.e[(sweep - 1) & 1]));
        if (h->hflag[(sweep - 1) & 1]) break;
      }
    }
    RMM_TRY(enqueue_step<1>(h, nb, 0, L, W, Vw, Db, st));
    for (int r = 0; r < nb - 1; ++r) RMM_TRY(enqueue_step<0>(h, nb, r, L, W, Vw, Db, st));
  }
  hipLaunchKernelGGL(blk_rank_kernel, dim3((unsigned)((l + 255) / 256)), dim3(256), 0, h->stream, l, L, W,
                     evals, perm, st, status);
  hipLaunchKernelGGL(blk_vectors_kernel, dim3((unsigned)((l + 255) / 256), (unsigned)l), dim3(256), 0,
                     h->stream, l, L, Vw, perm, V);
  ws.off = mark;
  return launch_status();
}

}  // namespace rmm
