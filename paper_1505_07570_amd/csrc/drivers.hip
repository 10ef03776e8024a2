// Drivers: randomized k-SVD (Alg. 5.2 with the subspace iteration of
// Alg. 5.1), sketch-and-solve least squares (eq. 4.2) and the exact
// least-squares comparator (Sec. 4.1).
//
// Everything is enqueued on the handle's stream; no host synchronization.
// Orthonormalization is shifted CholeskyQR in fp64: one pass on the Gram
// matrix shifted by c tr(G) I, which cannot break down for any numerically
// full-rank input, then plain CholeskyQR passes (two of them where the basis
// is an output, one inside the subspace iteration where only its span is
// used).  The small SVD of B = Q^T A is taken from Z = A^T Q = B^T without
// squaring its condition: Z = Q_z M_z with Q_z from shifted CholeskyQR and
// M_z = Q_z^T Z (l x l), then one-sided Jacobi on M_z, M_z J = Ubar Sigma, so
// that B = J Sigma (Q_z Ubar)^T: U = Q J, V = Q_z Ubar.
#include <math.h>

#include "common.hpp"
#include "dense.hpp"
#include "mixed.hpp"
#include "ops.hpp"
#include "rng.hpp"

namespace rmm {

template <typename T>
int launch_gaussian(const rmm_ctx* h, uint32_t tag, int64_t rows, int64_t cols, uint64_t seed,
                    T* out, int64_t ld);

namespace {

constexpr double kEps = 2.220446049250313e-16;

size_t smax(size_t a, size_t b) { return a > b ? a : b; }

// ---- shifted CholeskyQR ---------------------------------------------------------
//
// Shift of the first pass: c tr(G) with c = 11 (rows l + l (l + 1)) u,
// u = 2^-53 (Fukaya, Kannan, Nakatsukasa, Yamamoto, Yanagisawa, "Shifted
// Cholesky QR for computing the QR factorization of ill-conditioned
// matrices", SIAM J. Sci. Comput. 2020, with ||X||_F^2 for ||X||_2^2).
// Its Cholesky factor R1 exists whenever the condition number of X is below
// about u^-1, and X R1^{-1} has a condition number of order u^{-1/2}, which
// plain CholeskyQR then orthonormalizes.

struct OrthBufs {
  double* G;
  double* Rinv;
  double* diag;
  double* Xd;   // rows x l fp64
  double* Xd2;  // rows x l fp64 (second intermediate of three passes)
};

OrthBufs take_orth(Carver& ws, int64_t rows, int l) {
  OrthBufs b;
  b.G = ws.take<double>((size_t)l * l);
  b.Rinv = ws.take<double>((size_t)l * l);
  b.diag = ws.take<double>((size_t)l);
  b.Xd = ws.take<double>((size_t)rows * l);
  b.Xd2 = ws.take<double>((size_t)rows * l);
  return b;
}

double chol_shift(int64_t rows, int l) {
  return 11.0 * ((double)rows * l + (double)l * (l + 1)) * 0x1p-53;
}

template <typename T>
size_t orth_scratch(const rmm_ctx* h, int64_t rows, int l) {
  size_t w = gemm_workspace<double>(h, l, l, rows);
  w = smax(w, gemm_workspace<double>(h, (int)rows, l, l));
  w = smax(w, cholinv_workspace(h, l));
  return w;
}

// Q (rows x l, type TQ) = orthonormal basis of range(X): the shifted pass,
// then passes - 1 (>= 1) CholeskyQR passes.  Directions whose pivot falls
// below tau G_jj in a pass are dropped (zero columns of Q) and
// RMM_STATUS_QR_FALLBACK is raised.
template <typename T, typename TQ>
int orth(rmm_ctx* h, int64_t rows, int l, const T* X, int64_t ldx, TQ* Q, int64_t ldq,
         const OrthBufs& b, double tau, int32_t* status, Carver& ws, int passes) {
  const int r = (int)rows;
  RMM_TRY((gemm<T, T, double, double>(h, true, false, l, l, rows, X, ldx, X, ldx, 1.0, b.G, l, ws)));
  RMM_TRY(shift_diag(h, l, b.G, l, chol_shift(rows, l)));
  RMM_TRY(cholinv(h, l, b.G, l, tau, b.Rinv, b.diag, status, ws));
  RMM_TRY((gemm<T, double, double, double>(h, false, false, r, l, l, X, ldx, b.Rinv, l, 1.0, b.Xd,
                                           rows, ws)));
  double* cur = b.Xd;
  double* nxt = b.Xd2;
  for (int pass = 1;; ++pass) {
    RMM_TRY((gemm<double, double, double, double>(h, true, false, l, l, rows, cur, rows, cur, rows,
                                                  1.0, b.G, l, ws)));
    RMM_TRY(cholinv(h, l, b.G, l, tau, b.Rinv, b.diag, status, ws));
    if (pass + 1 >= passes)
      return gemm<double, double, double, TQ>(h, false, false, r, l, l, cur, rows, b.Rinv, l, 1.0, Q,
                                              ldq, ws);
    RMM_TRY((gemm<double, double, double, double>(h, false, false, r, l, l, cur, rows, b.Rinv, l, 1.0,
                                                  nxt, rows, ws)));
    double* t = cur;
    cur = nxt;
    nxt = t;
  }
}

// ---- small SVD of a tall matrix ----------------------------------------------------
//
// X (rows x l) = Ux diag(sigma) J^T with sigma descending, J (l x l)
// orthogonal and Ux (rows x kk) the first kk left singular vectors, all fp64:
// * when X fits in one workgroup's LDS, one-sided Jacobi on X itself
//   (X J = Ux diag(sigma));
// * otherwise X = Qx Mx with Qx from shifted CholeskyQR with three passes and
//   Mx = Qx^T X (l x l), one-sided Jacobi on Mx (Mx J = Ubar diag(sigma)) and
//   Ux = Qx Ubar[:, :kk].
struct SvdBufs {
  OrthBufs ob;
  double* Qx;     // rows x l
  double* Mx;     // l x l
  double* sigma;  // l
  double* Ubar;   // l x l
  double* J;      // l x l
  double* Ux;     // rows x l
};

SvdBufs take_svd(Carver& ws, int64_t rows, int l) {
  SvdBufs b;
  b.ob = take_orth(ws, rows, l);
  b.Qx = ws.take<double>((size_t)rows * l);
  b.Mx = ws.take<double>((size_t)l * l);
  b.sigma = ws.take<double>((size_t)l);
  b.Ubar = ws.take<double>((size_t)l * l);
  b.J = ws.take<double>((size_t)l * l);
  b.Ux = ws.take<double>((size_t)rows * l);
  return b;
}

template <typename T>
size_t svd_scratch(const rmm_ctx* h, int64_t rows, int l) {
  size_t w = orth_scratch<T>(h, rows, l);
  w = smax(w, gemm_workspace<double>(h, l, l, rows));
  w = smax(w, gemm_workspace<double>(h, (int)rows, l, l));
  w = smax(w, jacobi_svd_workspace(l));
  return w;
}

template <typename T>
int tall_svd(rmm_ctx* h, int64_t rows, int l, int kk, const T* X, int64_t ldx, const SvdBufs& b,
             int32_t* status, Carver& ws) {
  if (jacobi_svd_direct_ok(rows, l))
    return jacobi_svd_direct<T>(h, rows, l, X, ldx, b.sigma, b.Ux, b.J, status, ws);
  const double tau = 64.0 * kEps * (double)(rows > l ? rows : l);
  RMM_TRY((orth<T, double>(h, rows, l, X, ldx, b.Qx, rows, b.ob, tau, status, ws, 3)));
  RMM_TRY((gemm<double, T, double, double>(h, true, false, l, l, rows, b.Qx, rows, X, ldx, 1.0, b.Mx,
                                           l, ws)));
  RMM_TRY(jacobi_svd(h, l, b.Mx, l, b.sigma, b.Ubar, b.J, status, ws));
  return gemm<double, double, double, double>(h, false, false, (int)rows, kk, l, b.Qx, rows, b.Ubar, l,
                                              1.0, b.Ux, rows, ws);
}

// ---- randomized SVD --------------------------------------------------------------

// U = Q J[:, :k], V = Ux[:, :k], sigma = sigma[:k] from the small SVD of
// Z = A^T Q = Ux diag(sigma) J^T; then the sign convention.
template <typename T>
int finish_rsvd(rmm_ctx* h, int64_t m, int64_t n, int l, int k, const T* Q, const SvdBufs& sb,
                T* U, int64_t ldu, T* sigma, T* V, int64_t ldv, Carver& ws) {
  RMM_TRY((gemm<T, double, double, T>(h, false, false, (int)m, k, l, Q, m, sb.J, l, 1.0, U, ldu, ws)));
  RMM_TRY((copy_cast<double, T>(h, n, k, sb.Ux, n, V, ldv)));
  RMM_TRY((copy_cast<double, T>(h, k, 1, sb.sigma, k, sigma, k)));
  return sign_fix<T>(h, m, n, k, U, ldu, V, ldv);
}

template <typename T>
int rsvd_impl(rmm_ctx* h, bool run, int64_t m, int64_t n, const T* A, int64_t lda, int k, int p,
              int q, uint64_t seed, T* U, int64_t ldu, T* sigma, T* V, int64_t ldv, int32_t* status,
              size_t* bytes) {
  const int l = k + p;
  Carver ws(run ? h->ws : nullptr, run ? h->ws_bytes : 0);
  T* Om = ws.take<T>((size_t)n * l);
  T* Y = ws.take<T>((size_t)m * l);
  T* Q = ws.take<T>((size_t)m * l);
  T* Z = ws.take<T>((size_t)n * l);
  T* Qz = ws.take<T>((size_t)n * l);
  OrthBufs ob = take_orth(ws, m > n ? m : n, l);
  SvdBufs sb = take_svd(ws, n, l);
  // scratch shared by the steps below (released after each)
  size_t scratch = orth_scratch<T>(h, m, l);
  scratch = smax(scratch, orth_scratch<T>(h, n, l));
  scratch = smax(scratch, gemm_workspace<T>(h, (int)m, l, n));
  scratch = smax(scratch, gauss_sketch_workspace<T>(h, m, (int)n, l));
  scratch = smax(scratch, svd_scratch<T>(h, n, l));
  scratch = smax(scratch, gemm_workspace<double>(h, (int)m, k, l));
  scratch = smax(scratch, gemm_workspace<double>(h, (int)n, k, l));
  if (!run) {
    *bytes = ws.off + scratch + 8 * kAlign;
    return RMM_OK;
  }
  if (ws.off + scratch + 8 * kAlign > ws.cap) return RMM_ERR_WORKSPACE_TOO_SMALL;
  const double tau_m = 64.0 * kEps * (double)(m > l ? m : l);
  const double tau_n = 64.0 * kEps * (double)(n > l ? n : l);
  RMM_TRY(zero_status(h, status));
  RMM_TRY(launch_gaussian<T>(h, TAG_GAUSS_RSVD, n, l, seed, Om, n));
  // range finder: Y = A Omega; q times (Q = qr(Y), Z = A^T Q, Qz = qr(Z),
  // Y = A Qz); Q = qr(Y)
  RMM_TRY((gemm<T, T, T, T>(h, false, false, (int)m, l, n, A, lda, Om, n, 1.0, Y, m, ws)));
  for (int t = 0; t < q; ++t) {
    RMM_TRY((orth<T, T>(h, m, l, Y, m, Q, m, ob, tau_m, status, ws, 2)));
    RMM_TRY(project_tn<T>(h, m, (int)n, A, lda, Q, m, l, Z, n, ws));
    RMM_TRY((orth<T, T>(h, n, l, Z, n, Qz, n, ob, tau_n, status, ws, 2)));
    RMM_TRY((gemm<T, T, T, T>(h, false, false, (int)m, l, n, A, lda, Qz, n, 1.0, Y, m, ws)));
  }
  RMM_TRY((orth<T, T>(h, m, l, Y, m, Q, m, ob, tau_m, status, ws, 3)));
  // projection: Z = A^T Q = B^T, and the small SVD of B from that of Z
  RMM_TRY(project_tn<T>(h, m, (int)n, A, lda, Q, m, l, Z, n, ws));
  RMM_TRY(tall_svd<T>(h, n, l, k, Z, n, sb, status, ws));
  return finish_rsvd<T>(h, m, n, l, k, Q, sb, U, ldu, sigma, V, ldv, ws);
}

// ---- k-SVD by block Lanczos (Sec. 5.1, Alg. 5.1) ----------------------------------
//
// q Krylov blocks of width s: Q_0 = qr(A Omega); block i + 1 = A (A^T Q_i),
// orthogonalized against every earlier block by two passes of block
// Gram-Schmidt, then orthonormalized (the blocks span range(K) of Alg. 5.1).
// Then Z = A^T Q_C (n x sq) and the small SVD of B = Z^T, as in the prototype.
template <typename T>
int lanczos_impl(rmm_ctx* h, bool run, int64_t m, int64_t n, const T* A, int64_t lda, int k, int s,
                 int q, uint64_t seed, T* U, int64_t ldu, T* sigma, T* V, int64_t ldv,
                 int32_t* status, size_t* bytes) {
  const int L = s * q;
  Carver ws(run ? h->ws : nullptr, run ? h->ws_bytes : 0);
  T* Om = ws.take<T>((size_t)n * s);
  T* Qc = ws.take<T>((size_t)m * L);
  T* Y = ws.take<T>((size_t)m * s);
  T* Z = ws.take<T>((size_t)n * L);
  OrthBufs ob = take_orth(ws, m, s);
  double* Wb = ws.take<double>((size_t)s * s);
  SvdBufs sb = take_svd(ws, n, L);
  size_t scratch = orth_scratch<T>(h, m, s);
  scratch = smax(scratch, gemm_workspace<T>(h, (int)m, s, n));
  scratch = smax(scratch, gauss_sketch_workspace<T>(h, m, (int)n, s));
  scratch = smax(scratch, gauss_sketch_workspace<T>(h, m, (int)n, L));
  scratch = smax(scratch, gemm_workspace<double>(h, s, s, m));
  scratch = smax(scratch, gemm_workspace<double>(h, (int)m, s, s));
  scratch = smax(scratch, svd_scratch<T>(h, n, L));
  scratch = smax(scratch, gemm_workspace<double>(h, (int)m, k, L));
  scratch = smax(scratch, gemm_workspace<double>(h, (int)n, k, L));
  if (!run) {
    *bytes = ws.off + scratch + 8 * kAlign;
    return RMM_OK;
  }
  if (ws.off + scratch + 8 * kAlign > ws.cap) return RMM_ERR_WORKSPACE_TOO_SMALL;
  const double tau_m = 64.0 * kEps * (double)(m > s ? m : s);
  RMM_TRY(zero_status(h, status));
  RMM_TRY(launch_gaussian<T>(h, TAG_GAUSS_RSVD, n, s, seed, Om, n));
  RMM_TRY((gemm<T, T, T, T>(h, false, false, (int)m, s, n, A, lda, Om, n, 1.0, Y, m, ws)));
  RMM_TRY((orth<T, T>(h, m, s, Y, m, Qc, m, ob, tau_m, status, ws, 3)));
  for (int i = 1; i < q; ++i) {
    const T* Qp = Qc + (int64_t)(i - 1) * s * m;
    RMM_TRY(project_tn<T>(h, m, (int)n, A, lda, Qp, m, s, Z, n, ws));  // Z = A^T Q_{i-1}
    RMM_TRY((gemm<T, T, T, T>(h, false, false, (int)m, s, n, A, lda, Z, n, 1.0, Y, m, ws)));
    for (int pass = 0; pass < 2; ++pass)
      for (int b = 0; b < i; ++b) {
        const T* Qb = Qc + (int64_t)b * s * m;
        RMM_TRY((gemm<T, T, double, double>(h, true, false, s, s, m, Qb, m, Y, m, 1.0, Wb, s, ws)));
        RMM_TRY((gemm<T, double, double, T>(h, false, false, (int)m, s, s, Qb, m, Wb, s, -1.0, Y, m,
                                            ws, 1.0)));
      }
    RMM_TRY((orth<T, T>(h, m, s, Y, m, Qc + (int64_t)i * s * m, m, ob, tau_m, status, ws, 3)));
  }
  // Z = A^T Q_C = B^T and the small SVD of B from that of Z
  RMM_TRY(project_tn<T>(h, m, (int)n, A, lda, Qc, m, L, Z, n, ws));
  RMM_TRY(tall_svd<T>(h, n, L, k, Z, n, sb, status, ws));
  return finish_rsvd<T>(h, m, n, L, k, Qc, sb, U, ldu, sigma, V, ldv, ws);
}

// ---- randomized SVD with BF16 / FP8 passes over A ----------------------------------------
//
// Same steps as rsvd_impl; every product with A runs on a one-time quantized
// copy of A (mixed.hip), the small operands are quantized per column before
// each pass, and the results come back in fp32 for the fp64 orthonormalization
// and small SVD.
int rsvd_mixed(rmm_ctx* h, bool run, rmm_precision prec, int64_t m, int64_t n, const float* A,
               int64_t lda, int k, int p, int q, uint64_t seed, float* U, int64_t ldu, float* sigma,
               float* V, int64_t ldv, int32_t* status, size_t* bytes) {
  const int l = k + p;
  const size_t eb = mp_elem_bytes(prec);
  const int64_t pm = mp_pad(m), pn = mp_pad(n);
  Carver ws(run ? h->ws : nullptr, run ? h->ws_bytes : 0);
  float* sc = ws.take<float>((size_t)n);
  unsigned char* Aq = ws.take<unsigned char>((size_t)pm * n * eb);
  unsigned char* Aqt = ws.take<unsigned char>((size_t)pn * m * eb);
  unsigned char* Qq = ws.take<unsigned char>((size_t)pm * l * eb);
  unsigned char* Xq = ws.take<unsigned char>((size_t)pn * l * eb);
  float* uq = ws.take<float>((size_t)l);
  float* ux = ws.take<float>((size_t)l);
  unsigned* umax = ws.take<unsigned>((size_t)l);
  float* Om = ws.take<float>((size_t)n * l);
  float* Y = ws.take<float>((size_t)m * l);
  float* Q = ws.take<float>((size_t)m * l);
  float* Z = ws.take<float>((size_t)n * l);
  float* Qz = ws.take<float>((size_t)n * l);
  OrthBufs ob = take_orth(ws, m > n ? m : n, l);
  SvdBufs sb = take_svd(ws, n, l);
  size_t scratch = orth_scratch<float>(h, m, l);
  scratch = smax(scratch, orth_scratch<float>(h, n, l));
  scratch = smax(scratch, qgemm_workspace(h, (int)m, l, pn));
  scratch = smax(scratch, qgemm_workspace(h, (int)n, l, pm));
  scratch = smax(scratch, svd_scratch<float>(h, n, l));
  scratch = smax(scratch, gemm_workspace<double>(h, (int)m, k, l));
  scratch = smax(scratch, gemm_workspace<double>(h, (int)n, k, l));
  if (!run) {
    *bytes = ws.off + scratch + 8 * kAlign;
    return RMM_OK;
  }
  if (ws.off + scratch + 8 * kAlign > ws.cap) return RMM_ERR_WORKSPACE_TOO_SMALL;
  const double tau_m = 64.0 * kEps * (double)(m > l ? m : l);
  const double tau_n = 64.0 * kEps * (double)(n > l ? n : l);
  RMM_TRY(zero_status(h, status));
  RMM_TRY(mp_quantize_matrix(h, prec, m, n, A, lda, sc, Aq, Aqt));
  RMM_TRY(launch_gaussian<float>(h, TAG_GAUSS_RSVD, n, l, seed, Om, n));
  // Y = A Omega = Aq_t^T q(diag(sc) Omega)
  RMM_TRY(mp_quantize_cols(h, prec, n, l, Om, n, sc, Xq, ux, umax));
  RMM_TRY(mp_gemm_tn(h, prec, (int)m, l, pn, Aqt, Xq, nullptr, ux, Y, m, ws));
  for (int t = 0; t < q; ++t) {
    RMM_TRY((orth<float, float>(h, m, l, Y, m, Q, m, ob, tau_m, status, ws, 2)));
    RMM_TRY(mp_quantize_cols(h, prec, m, l, Q, m, nullptr, Qq, uq, umax));
    RMM_TRY(mp_gemm_tn(h, prec, (int)n, l, pm, Aq, Qq, sc, uq, Z, n, ws));
    RMM_TRY((orth<float, float>(h, n, l, Z, n, Qz, n, ob, tau_n, status, ws, 2)));
    RMM_TRY(mp_quantize_cols(h, prec, n, l, Qz, n, sc, Xq, ux, umax));
    RMM_TRY(mp_gemm_tn(h, prec, (int)m, l, pn, Aqt, Xq, nullptr, ux, Y, m, ws));
  }
  RMM_TRY((orth<float, float>(h, m, l, Y, m, Q, m, ob, tau_m, status, ws, 3)));
  RMM_TRY(mp_quantize_cols(h, prec, m, l, Q, m, nullptr, Qq, uq, umax));
  RMM_TRY(mp_gemm_tn(h, prec, (int)n, l, pm, Aq, Qq, sc, uq, Z, n, ws));
  RMM_TRY(tall_svd<float>(h, n, l, k, Z, n, sb, status, ws));
  return finish_rsvd<float>(h, m, n, l, k, Q, sb, U, ldu, sigma, V, ldv, ws);
}

// ---- sketch-and-solve least squares ---------------------------------------------------

template <typename T>
size_t sketch_scratch(const rmm_ctx* h, rmm_sketch_kind kind, int64_t m, int ncols, int64_t s) {
  switch (kind) {
    case RMM_COUNTSKETCH: return countsketch_workspace<T>(h, m, ncols, s);
    case RMM_SRHT: return srht_workspace<T>(h, m, ncols, s);
    default: return gauss_sketch_workspace<T>(h, m, ncols, s);
  }
}

template <typename T>
int run_sketch(rmm_ctx* h, rmm_sketch_kind kind, int64_t m, int n, const T* A, int64_t lda,
               const T* b, int64_t s, uint64_t seed, T* C, int64_t ldc, Carver& ws) {
  switch (kind) {
    case RMM_COUNTSKETCH: return countsketch_run<T>(h, m, n, A, lda, b, s, seed, C, ldc, ws);
    case RMM_SRHT: return srht_run<T>(h, m, n, A, lda, b, s, seed, C, ldc, ws);
    default: return gauss_sketch_run<T>(h, m, n, A, lda, b, s, seed, C, ldc, ws);
  }
}

// x = argmin ||Cs[:, :d] x - Cs[:, d]|| for the s x (d+1) fp64 system by
// CholeskyQR2: Q R = Cs[:, :d], x = R^{-1} Q^T b~.
struct LsBufs {
  double *G, *R1, *R2, *d1, *d2, *Q1, *Q, *y, *t;
};

size_t ls_scratch(const rmm_ctx* h, int64_t s, int d) {
  size_t w = gemm_workspace<double>(h, d, d, s);
  w = smax(w, gemm_workspace<double>(h, (int)s, d, d));
  w = smax(w, gemm_workspace<double>(h, d, 1, s));
  w = smax(w, cholinv_workspace(h, d));
  return w;
}

LsBufs take_ls(Carver& ws, int64_t s, int d) {
  LsBufs b;
  b.G = ws.take<double>((size_t)d * d);
  b.R1 = ws.take<double>((size_t)d * d);
  b.R2 = ws.take<double>((size_t)d * d);
  b.d1 = ws.take<double>((size_t)d);
  b.d2 = ws.take<double>((size_t)d);
  b.Q1 = ws.take<double>((size_t)s * d);
  b.Q = ws.take<double>((size_t)s * d);
  b.y = ws.take<double>((size_t)d);
  b.t = ws.take<double>((size_t)d);
  return b;
}

// CholeskyQR2 of the s x d FP64 matrix Cs (ld s): b.Q = Cs R1 R2 with the
// two inverse factors kept in b.R1, b.R2 (their diagonals in b.d1, b.d2)
int cholqr2(rmm_ctx* h, int64_t s, int d, const double* Cs, const LsBufs& b, Carver& ws) {
  const double tau = 64.0 * kEps * (double)s;
  RMM_TRY((gemm<double, double, double, double>(h, true, false, d, d, s, Cs, s, Cs, s, 1.0, b.G, d, ws)));
  RMM_TRY(cholinv(h, d, b.G, d, tau, b.R1, b.d1, nullptr, ws));
  RMM_TRY((gemm<double, double, double, double>(h, false, false, (int)s, d, d, Cs, s, b.R1, d, 1.0,
                                                b.Q1, s, ws)));
  RMM_TRY((gemm<double, double, double, double>(h, true, false, d, d, s, b.Q1, s, b.Q1, s, 1.0, b.G,
                                                d, ws)));
  RMM_TRY(cholinv(h, d, b.G, d, tau, b.R2, b.d2, nullptr, ws));
  return gemm<double, double, double, double>(h, false, false, (int)s, d, d, b.Q1, s, b.R2, d, 1.0,
                                              b.Q, s, ws);
}

int ls_solve(rmm_ctx* h, int64_t s, int d, const double* Cs, const LsBufs& b, double* x,
             int32_t* status, Carver& ws) {
  const double tau = 64.0 * kEps * (double)s;
  const double* bt = Cs + (int64_t)d * s;
  RMM_TRY((gemm<double, double, double, double>(h, true, false, d, d, s, Cs, s, Cs, s, 1.0, b.G, d, ws)));
  RMM_TRY(cholinv(h, d, b.G, d, tau, b.R1, b.d1, nullptr, ws));
  RMM_TRY((gemm<double, double, double, double>(h, false, false, (int)s, d, d, Cs, s, b.R1, d, 1.0,
                                                b.Q1, s, ws)));
  RMM_TRY((gemm<double, double, double, double>(h, true, false, d, d, s, b.Q1, s, b.Q1, s, 1.0, b.G,
                                                d, ws)));
  RMM_TRY(cholinv(h, d, b.G, d, tau, b.R2, b.d2, nullptr, ws));
  RMM_TRY((gemm<double, double, double, double>(h, false, false, (int)s, d, d, b.Q1, s, b.R2, d, 1.0,
                                                b.Q, s, ws)));
  RMM_TRY((gemm<double, double, double, double>(h, true, false, d, 1, s, b.Q, s, bt, s, 1.0, b.y, d, ws)));
  RMM_TRY(trmv_upper(h, d, b.R2, b.y, b.t));
  RMM_TRY(trmv_upper(h, d, b.R1, b.t, x));
  // R = R2 R1 has diagonal d2 * d1 (a dropped pivot shows up as a zero)
  return rank_check(h, d, b.d1, b.d2, 10.0 * (double)s * kEps, status);
}

template <typename T>
int lsr_impl(rmm_ctx* h, bool run, rmm_sketch_kind kind, int64_t m, int d, const T* A, int64_t lda,
             const T* b, int64_t s, uint64_t seed, double* x, double* resid, int32_t* status,
             size_t* bytes) {
  Carver ws(run ? h->ws : nullptr, run ? h->ws_bytes : 0);
  T* Cs = ws.take<T>((size_t)s * (d + 1));
  double* Csd = ws.take<double>((size_t)s * (d + 1));
  LsBufs lb = take_ls(ws, s, d);
  size_t scratch = sketch_scratch<T>(h, kind, m, d + 1, s);
  scratch = smax(scratch, ls_scratch(h, s, d));
  scratch = smax(scratch, residual_workspace(m));
  if (!run) {
    *bytes = ws.off + scratch + 8 * kAlign;
    return RMM_OK;
  }
  if (ws.off + scratch + 8 * kAlign > ws.cap) return RMM_ERR_WORKSPACE_TOO_SMALL;
  RMM_TRY(zero_status(h, status));
  {
    const size_t mark = ws.off;
    RMM_TRY(run_sketch<T>(h, kind, m, d, A, lda, b, s, seed, Cs, s, ws));
    ws.off = mark;
  }
  RMM_TRY((copy_cast<T, double>(h, s, d + 1, Cs, s, Csd, s)));
  RMM_TRY(ls_solve(h, s, d, Csd, lb, x, status, ws));
  if (resid) RMM_TRY(residual_norm<T>(h, m, d, A, lda, b, x, resid, ws));
  return RMM_OK;
}

// Alg. 4.1: the sketch-and-solve start x0 = T Q_Y^T (S^T b) and T = R_Y^{-1}
// (T = R1 R2, the two inverse factors of CholeskyQR2), then `iters` steps of
// preconditioned CG on A^T A x = A^T b with M = T T^T (refine.hip), each one
// fused pass over A.  resid = ||A x - b|| from one more pass.
template <typename T>
int lsr_precise_impl(rmm_ctx* h, bool run, rmm_sketch_kind kind, int64_t m, int d, const T* A,
                     int64_t lda, const T* b, int64_t s, uint64_t seed, int64_t iters, double* x,
                     double* resid, int32_t* status, size_t* bytes) {
  Carver ws(run ? h->ws : nullptr, run ? h->ws_bytes : 0);
  T* Cs = ws.take<T>((size_t)s * (d + 1));
  double* Csd = ws.take<double>((size_t)s * (d + 1));
  LsBufs lb = take_ls(ws, s, d);
  double* Tm = ws.take<double>((size_t)d * d);
  double* M = ws.take<double>((size_t)d * d);
  double* g = ws.take<double>((size_t)d);
  double* y = ws.take<double>((size_t)d);
  double* p = ws.take<double>((size_t)d);
  double* sc = ws.take<double>(4);
  double* part = ws.take<double>(refine_part_elems(h, d));
  size_t scratch = sketch_scratch<T>(h, kind, m, d + 1, s);
  scratch = smax(scratch, ls_scratch(h, s, d));
  scratch = smax(scratch, gemm_workspace<double>(h, d, d, d));
  if (!run) {
    *bytes = ws.off + scratch + 8 * kAlign;
    return RMM_OK;
  }
  if (ws.off + scratch + 8 * kAlign > ws.cap) return RMM_ERR_WORKSPACE_TOO_SMALL;
  RMM_TRY(zero_status(h, status));
  {
    const size_t mark = ws.off;
    RMM_TRY(run_sketch<T>(h, kind, m, d, A, lda, b, s, seed, Cs, s, ws));
    ws.off = mark;
  }
  RMM_TRY((copy_cast<T, double>(h, s, d + 1, Cs, s, Csd, s)));
  RMM_TRY(ls_solve(h, s, d, Csd, lb, x, status, ws));
  RMM_TRY((gemm<double, double, double, double>(h, false, false, d, d, d, lb.R1, d, lb.R2, d, 1.0,
                                                Tm, d, ws)));
  RMM_TRY((gemm<double, double, double, double>(h, false, true, d, d, d, Tm, d, Tm, d, 1.0, M, d,
                                                ws)));
  RMM_TRY(normal_pass<T>(h, m, d, A, lda, b, x, part));
  RMM_TRY(pcg_init(h, d, part, M, g, y, p, sc));
  for (int64_t t = 0; t < iters; ++t) {
    RMM_TRY(normal_pass<T>(h, m, d, A, lda, nullptr, p, part));
    RMM_TRY(pcg_step(h, d, part, M, x, g, y, p, sc));
  }
  if (resid) {
    RMM_TRY(normal_pass<T>(h, m, d, A, lda, b, x, part));
    RMM_TRY(pass_resid(h, d, part, resid));
  }
  return RMM_OK;
}

// exact solution by the normal equations in fp64: (A^T A) x = A^T b
template <typename T>
int plain_impl(rmm_ctx* h, bool run, int64_t m, int d, const T* A, int64_t lda, const T* b,
               double* x, double* resid, int32_t* status, size_t* bytes) {
  Carver ws(run ? h->ws : nullptr, run ? h->ws_bytes : 0);
  double* G = ws.take<double>((size_t)d * d);
  double* c = ws.take<double>((size_t)d);
  double* Rinv = ws.take<double>((size_t)d * d);
  double* dg = ws.take<double>((size_t)d);
  double* t = ws.take<double>((size_t)d);
  size_t scratch = gemm_workspace<double>(h, d, d, m);
  scratch = smax(scratch, gemm_workspace<double>(h, d, 1, m));
  scratch = smax(scratch, gemm_workspace<double>(h, d, 1, d));
  scratch = smax(scratch, cholinv_workspace(h, d));
  scratch = smax(scratch, residual_workspace(m));
  if (!run) {
    *bytes = ws.off + scratch + 8 * kAlign;
    return RMM_OK;
  }
  if (ws.off + scratch + 8 * kAlign > ws.cap) return RMM_ERR_WORKSPACE_TOO_SMALL;
  RMM_TRY(zero_status(h, status));
  RMM_TRY((gemm<T, T, double, double>(h, true, false, d, d, m, A, lda, A, lda, 1.0, G, d, ws)));
  RMM_TRY((gemm<T, T, double, double>(h, true, false, d, 1, m, A, lda, b, m, 1.0, c, d, ws)));
  RMM_TRY(cholinv(h, d, G, d, 64.0 * kEps * (double)m, Rinv, dg, nullptr, ws));
  RMM_TRY((gemm<double, double, double, double>(h, true, false, d, 1, d, Rinv, d, c, d, 1.0, t, d, ws)));
  RMM_TRY(trmv_upper(h, d, Rinv, t, x));
  RMM_TRY(rank_check(h, d, dg, nullptr, 10.0 * (double)m * kEps, status));
  if (resid) RMM_TRY(residual_norm<T>(h, m, d, A, lda, b, x, resid, ws));
  return RMM_OK;
}

bool ld_bad(int64_t ld, int64_t rows) { return ld < (rows > 1 ? rows : 1); }

bool kind_ok(rmm_sketch_kind k) { return k == RMM_GAUSSIAN || k == RMM_SRHT || k == RMM_COUNTSKETCH; }

// ---- faster randomized k-SVD (Sec. 5.3, Alg. 5.3) ----------------------------

__global__ void scale_cols_kernel(int rows, int k, const double* __restrict__ X, int64_t ldx,
                                  const double* __restrict__ sc, double* __restrict__ Y) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * k) return;
  const int a = e % rows, c = e / rows;
  Y[a + (int64_t)c * rows] = X[a + (int64_t)c * ldx] * sc[c];
}

// Steps of Alg. 5.3: C = A S (column count sketch, stream seed + 1);
// L = P^T A, D = P^T C with P = P_cs P_2 (composite, stream seed); Q_D R_D =
// D by CholeskyQR2 (R_D^{-1} = R1 R2); Ubar Sigmabar Vbar^T = rank-k SVD of
// Z = Q_D^T L, taken from the small SVD of the tall Z^T = L^T Q_D; M = C
// R_D^{-1} Ubar Sigmabar and its SVD U Sigma Vhat^T by the same route; V =
// Vbar Vhat.  C, L, D in the input type, the small algebra in FP64.
template <typename T>
int rsvd_faster_impl(rmm_ctx* h, bool run, rmm_sketch_kind kind2, int64_t m, int64_t n, const T* A,
                     int64_t lda, int k, int s, int64_t pcs, int p, uint64_t seed, T* U, int64_t ldu,
                     T* sigma, T* V, int64_t ldv, int32_t* status, size_t* bytes) {
  Carver ws(run ? h->ws : nullptr, run ? h->ws_bytes : 0);
  const int64_t wide = n > s ? n : s;
  T* C = ws.take<T>((size_t)m * s);
  T* Y = ws.take<T>((size_t)pcs * wide);
  T* L = ws.take<T>((size_t)p * n);
  T* D = ws.take<T>((size_t)p * s);
  double* Dd = ws.take<double>((size_t)p * s);
  LsBufs lb = take_ls(ws, p, s);
  double* Ri = ws.take<double>((size_t)s * s);
  double* Zt = ws.take<double>((size_t)n * s);
  SvdBufs sz = take_svd(ws, n, s);
  double* T1 = ws.take<double>((size_t)s * k);
  double* T2 = ws.take<double>((size_t)s * k);
  double* M = ws.take<double>((size_t)m * k);
  SvdBufs sm = take_svd(ws, m, k);
  size_t scratch = countsketch_cols_workspace(n);
  scratch = smax(scratch, countsketch_workspace<T>(h, m, (int)n, pcs));
  scratch = smax(scratch, countsketch_workspace<T>(h, m, s, pcs));
  scratch = smax(scratch, sketch_scratch<T>(h, kind2, pcs, (int)n, p));
  scratch = smax(scratch, sketch_scratch<T>(h, kind2, pcs, s, p));
  scratch = smax(scratch, ls_scratch(h, p, s));
  scratch = smax(scratch, gemm_workspace<double>(h, (int)n, s, p));
  scratch = smax(scratch, svd_scratch<double>(h, n, s));
  scratch = smax(scratch, gemm_workspace<double>(h, (int)n, k, s));
  scratch = smax(scratch, gemm_workspace<double>(h, s, k, s));
  scratch = smax(scratch, gemm_workspace<double>(h, (int)m, k, s));
  scratch = smax(scratch, svd_scratch<double>(h, m, k));
  scratch = smax(scratch, gemm_workspace<double>(h, (int)m, k, k));
  scratch = smax(scratch, gemm_workspace<double>(h, (int)n, k, k));
  if (!run) {
    *bytes = ws.off + scratch + 8 * kAlign;
    return RMM_OK;
  }
  if (ws.off + scratch + 8 * kAlign > ws.cap) return RMM_ERR_WORKSPACE_TOO_SMALL;
  RMM_TRY(zero_status(h, status));
  const size_t mark = ws.off;
  // step 1 and the two composite sketches of step 2
  RMM_TRY(countsketch_cols_run<T>(h, m, n, A, lda, s, seed + 1, C, m, ws));
  ws.off = mark;
  RMM_TRY(countsketch_run<T>(h, m, (int)n, A, lda, nullptr, pcs, seed, Y, pcs, ws));
  ws.off = mark;
  RMM_TRY(run_sketch<T>(h, kind2, pcs, (int)n, Y, pcs, nullptr, p, seed, L, p, ws));
  ws.off = mark;
  RMM_TRY(countsketch_run<T>(h, m, s, C, m, nullptr, pcs, seed, Y, pcs, ws));
  ws.off = mark;
  RMM_TRY(run_sketch<T>(h, kind2, pcs, s, Y, pcs, nullptr, p, seed, D, p, ws));
  ws.off = mark;
  // step 3: CholeskyQR2 of D, R_D^{-1} = R1 R2
  RMM_TRY((copy_cast<T, double>(h, p, s, D, p, Dd, p)));
  RMM_TRY(cholqr2(h, p, s, Dd, lb, ws));
  RMM_TRY(rank_check(h, s, lb.d1, lb.d2, 10.0 * (double)p * kEps, status));
  RMM_TRY((gemm<double, double, double, double>(h, false, false, s, s, s, lb.R1, s, lb.R2, s, 1.0, Ri,
                                                s, ws)));
  // step 4: Z^T = L^T Q_D = Ux_z Sigma_z J_z^T, so that Z = J_z Sigma_z Ux_z^T:
  // Ubar = J_z[:, :k], Sigmabar = Sigma_z[:k], Vbar = Ux_z[:, :k]
  RMM_TRY((gemm<T, double, double, double>(h, true, false, (int)n, s, p, L, p, lb.Q, p, 1.0, Zt, n,
                                           ws)));
  RMM_TRY(tall_svd<double>(h, n, s, k, Zt, n, sz, status, ws));
  // step 5: M = C R_D^{-1} Ubar Sigmabar = Ux_m Sigma J_m^T
  hipLaunchKernelGGL(scale_cols_kernel, dim3((s * k + 255) / 256), dim3(256), 0, h->stream, s, k, sz.J,
                     (int64_t)s, sz.sigma, T1);
  RMM_TRY(launch_status());
  RMM_TRY((gemm<double, double, double, double>(h, false, false, s, k, s, Ri, s, T1, s, 1.0, T2, s, ws)));
  RMM_TRY((gemm<T, double, double, double>(h, false, false, (int)m, k, s, C, m, T2, s, 1.0, M, m, ws)));
  RMM_TRY(tall_svd<double>(h, m, k, k, M, m, sm, status, ws));
  RMM_TRY((copy_cast<double, T>(h, m, k, sm.Ux, m, U, ldu)));
  RMM_TRY((copy_cast<double, T>(h, k, 1, sm.sigma, k, sigma, k)));
  // step 6: V = Vbar Vhat, Vhat = J_m
  RMM_TRY((gemm<double, double, double, T>(h, false, false, (int)n, k, k, sz.Ux, n, sm.J, k, 1.0, V,
                                           ldv, ws)));
  return sign_fix<T>(h, m, n, k, U, ldu, V, ldv);
}

int rsvd_faster_args(rmm_handle h, rmm_dtype dt, rmm_sketch_kind kind2, int64_t m, int64_t n,
                     int64_t k, int64_t s, int64_t pcs, int64_t p) {
  if (!h || !dt_ok(dt) || m < 1 || n < 1 || k < 1 || s < k || p < s || pcs < p)
    return RMM_ERR_INVALID_ARG;
  if (kind2 != RMM_GAUSSIAN && kind2 != RMM_SRHT) return RMM_ERR_UNSUPPORTED;
  if (kind2 == RMM_SRHT && p > (1ll << ceil_log2((uint64_t)pcs))) return RMM_ERR_INVALID_ARG;
  if (s > 1024 || p > (1 << 20) || pcs >= (1ll << 30) || m >= (1ll << 31) || n >= (1ll << 30))
    return RMM_ERR_UNSUPPORTED;
  return RMM_OK;
}

int rsvd_args(rmm_handle h, rmm_dtype dt, rmm_precision prec, int64_t m, int64_t n, int64_t k,
              int64_t p) {
  if (!h || !dt_ok(dt) || m < 1 || n < 1 || k < 1 || p < 0) return RMM_ERR_INVALID_ARG;
  if (k + p > (m < n ? m : n)) return RMM_ERR_INVALID_ARG;
  if (k + p > 1024) return RMM_ERR_UNSUPPORTED;
  if (m >= (1ll << 31) || n >= (1ll << 31)) return RMM_ERR_UNSUPPORTED;
  if (prec != RMM_PREC_NATIVE && prec != RMM_PREC_BF16 && prec != RMM_PREC_FP8)
    return RMM_ERR_INVALID_ARG;
  if (prec != RMM_PREC_NATIVE && dt != RMM_F32) return RMM_ERR_UNSUPPORTED;
  return RMM_OK;
}

// ---- faster SPSD sketching (Sec. 6.3, Alg. 6.1) on the RBF kernel -----------------------
//
// S: s sorted uniform indices (stream TAG_SPSD_SAMPLE); C = K[:, S] in the
// points' type; Q_C (n x s, FP64) by shifted CholeskyQR with three passes;
// q = squared row norms of Q_C; p draws with replacement with probability
// ~ q (TAG_LEVERAGE); P = unique([draws; S]) (length np <= p + s, stored
// padded to pm = p + s); G = Q_C[P, :] (zero rows past np), K[P, P] in FP64
// (zero past np); G = Q_G R_G by CholeskyQR2, G^+ = R_G^{-1} Q_G^T; Z~ =
// G^+ K[P, P] G^+T = R_G^{-1} (Q_G^T K[P, P] Q_G) R_G^{-T}.
template <typename T>
int rbf_cols_any(rmm_ctx* h, int64_t n, int d, const T* X, int64_t ldx, int c, const int64_t* idx,
                 const T* Y, int64_t ldy, double g, T* C, int64_t ldc) {
  if constexpr (sizeof(T) == 4)
    return launch_rbf(h, n, d, X, ldx, c, idx, Y, ldy, 0, g, C, ldc);
  else
    return rbf_cols_f64(h, n, d, X, ldx, c, idx, Y, ldy, g, C, ldc);
}

template <typename T>
int spsd_impl(rmm_ctx* h, bool run, int64_t n, int d, const T* X, int64_t ldx, double sigma, int s,
              int64_t p, uint64_t seed, int64_t* S, int64_t* P, int64_t* np, double* Qc, int64_t ldq,
              double* Z, int32_t* status, size_t* bytes) {
  const int64_t pm = p + s;
  Carver ws(run ? h->ws : nullptr, run ? h->ws_bytes : 0);
  T* C = ws.take<T>((size_t)n * s);
  OrthBufs ob = take_orth(ws, n, s);
  double* q = ws.take<double>((size_t)n);
  uint64_t* cdf = ws.take<uint64_t>((size_t)n);
  int64_t* draws = ws.take<int64_t>((size_t)(p > 0 ? p : 1));
  double* G = ws.take<double>((size_t)pm * s);
  double* Kp = ws.take<double>((size_t)pm * pm);
  LsBufs lb = take_ls(ws, pm, s);
  double* Ri = ws.take<double>((size_t)s * s);
  double* T1 = ws.take<double>((size_t)pm * s);
  double* T2 = ws.take<double>((size_t)s * s);
  double* T3 = ws.take<double>((size_t)s * s);
  size_t scratch = orth_scratch<T>(h, n, s);
  scratch = smax(scratch, ls_scratch(h, pm, s));
  scratch = smax(scratch, gemm_workspace<double>(h, s, s, s));
  scratch = smax(scratch, gemm_workspace<double>(h, (int)pm, s, pm));
  scratch = smax(scratch, gemm_workspace<double>(h, s, s, pm));
  if (!run) {
    *bytes = ws.off + scratch + 8 * kAlign;
    return RMM_OK;
  }
  if (ws.off + scratch + 8 * kAlign > ws.cap) return RMM_ERR_WORKSPACE_TOO_SMALL;
  const double g = 1.0 / (2.0 * sigma * sigma);
  RMM_TRY(zero_status(h, status));
  RMM_TRY(launch_sample_indices_i64(h, (uint64_t)n, ceil_log2((uint64_t)n), s, TAG_SPSD_SAMPLE, seed, S));
  RMM_TRY(rbf_cols_any<T>(h, n, d, X, ldx, s, S, X, ldx, g, C, n));
  RMM_TRY((orth<T, double>(h, n, s, C, n, Qc, ldq, ob, 64.0 * kEps * (double)(n > s ? n : s), status,
                           ws, 3)));
  RMM_TRY(leverage_scores(h, n, s, Qc, ldq, q));
  RMM_TRY(weighted_sample(h, n, q, p, TAG_LEVERAGE, seed, cdf, draws));
  RMM_TRY(union_sorted(h, n, draws, p, S, s, pm, P, np));
  RMM_TRY(gather_rows<double>(h, pm, s, P, np, Qc, ldq, G));
  RMM_TRY(rbf_block_f64<T>(h, d, X, ldx, P, np, pm, X, ldx, P, np, pm, g, Kp));
  RMM_TRY(cholqr2(h, pm, s, G, lb, ws));
  RMM_TRY(rank_check(h, s, lb.d1, lb.d2, 10.0 * (double)pm * kEps, status));
  RMM_TRY((gemm<double, double, double, double>(h, false, false, s, s, s, lb.R1, s, lb.R2, s, 1.0, Ri,
                                                s, ws)));
  RMM_TRY((gemm<double, double, double, double>(h, false, false, (int)pm, s, pm, Kp, pm, lb.Q, pm, 1.0,
                                                T1, pm, ws)));
  RMM_TRY((gemm<double, double, double, double>(h, true, false, s, s, pm, lb.Q, pm, T1, pm, 1.0, T2, s,
                                                ws)));
  RMM_TRY((gemm<double, double, double, double>(h, false, false, s, s, s, Ri, s, T2, s, 1.0, T3, s, ws)));
  return gemm<double, double, double, double>(h, false, true, s, s, s, T3, s, Ri, s, 1.0, Z, s, ws);
}

// ---- faster CUR (Sec. 6.6.3) of the RBF kernel A = K(Xtest, Xtrain) ---------------------
//
// SC: c of the n training points, SR: r of the m test points (sorted
// uniform, TAG_CUR_COLS / TAG_CUR_ROWS); C = A[:, SC] (m x c), R^T =
// A[SR, :]^T (n x r), both in the points' type; P_C (p_c of m, TAG_CUR_PC)
// and P_R (p_r of n, TAG_CUR_PR) uniform without replacement (the
// listing) or by the leverage scores of C and R^T with replacement (the
// remark), joined with SR and SC; U = (C[P_C, :])^+ A[P_C, P_R]
// (R[:, P_R])^+ with both pseudo-inverses from CholeskyQR2 of the gathered
// tall blocks: (C[P_C, :])^+ = R_a^{-1} Q_a^T and (R[:, P_R])^+ =
// ((R^T)[P_R, :])^{+T} = Q_b R_b^{-T}.
template <typename T>
int cur_impl(rmm_ctx* h, bool run, int64_t m, int64_t n, int d, const T* Xte, int64_t ldte,
             const T* Xtr, int64_t ldtr, double sigma, int c, int r, int64_t pc, int64_t pr, int mode,
             uint64_t seed, int64_t* SC, int64_t* SR, int64_t* PC, int64_t* PR, int64_t* lens, T* C,
             int64_t ldc, double* U, int64_t ldu, T* Rt, int64_t ldrt, int32_t* status, size_t* bytes) {
  const int64_t pcm = pc + r, prm = pr + c;
  const int64_t big = m * c > n * r ? m * c : n * r;
  Carver ws(run ? h->ws : nullptr, run ? h->ws_bytes : 0);
  int64_t* dC = ws.take<int64_t>((size_t)(pc > 0 ? pc : 1));
  int64_t* dR = ws.take<int64_t>((size_t)(pr > 0 ? pr : 1));
  double* Gc = ws.take<double>((size_t)pcm * c);
  double* Gr = ws.take<double>((size_t)prm * r);
  double* Ab = ws.take<double>((size_t)pcm * prm);
  LsBufs la = take_ls(ws, pcm, c);
  LsBufs lr = take_ls(ws, prm, r);
  double* Ria = ws.take<double>((size_t)c * c);
  double* Rib = ws.take<double>((size_t)r * r);
  double* T1 = ws.take<double>((size_t)pcm * r);
  double* T2 = ws.take<double>((size_t)c * r);
  double* T3 = ws.take<double>((size_t)c * r);
  double *Qb = nullptr, *q = nullptr;
  uint64_t* cdf = nullptr;
  OrthBufs ob{};
  const int kmax = c > r ? c : r;
  if (mode == 1) {
    Qb = ws.take<double>((size_t)big);
    q = ws.take<double>((size_t)(m > n ? m : n));
    cdf = ws.take<uint64_t>((size_t)(m > n ? m : n));
    ob.G = ws.take<double>((size_t)kmax * kmax);
    ob.Rinv = ws.take<double>((size_t)kmax * kmax);
    ob.diag = ws.take<double>((size_t)kmax);
    ob.Xd = ws.take<double>((size_t)big);
    ob.Xd2 = ws.take<double>((size_t)big);
  }
  size_t scratch = ls_scratch(h, pcm, c);
  scratch = smax(scratch, ls_scratch(h, prm, r));
  scratch = smax(scratch, gemm_workspace<double>(h, c, c, c));
  scratch = smax(scratch, gemm_workspace<double>(h, r, r, r));
  scratch = smax(scratch, gemm_workspace<double>(h, (int)pcm, r, prm));
  scratch = smax(scratch, gemm_workspace<double>(h, c, r, pcm));
  scratch = smax(scratch, gemm_workspace<double>(h, c, r, c));
  scratch = smax(scratch, gemm_workspace<double>(h, c, r, r));
  if (mode == 1) {
    scratch = smax(scratch, orth_scratch<T>(h, m, c));
    scratch = smax(scratch, orth_scratch<T>(h, n, r));
  }
  if (!run) {
    *bytes = ws.off + scratch + 8 * kAlign;
    return RMM_OK;
  }
  if (ws.off + scratch + 8 * kAlign > ws.cap) return RMM_ERR_WORKSPACE_TOO_SMALL;
  const double g = 1.0 / (2.0 * sigma * sigma);
  RMM_TRY(zero_status(h, status));
  RMM_TRY(launch_sample_indices_i64(h, (uint64_t)n, ceil_log2((uint64_t)n), c, TAG_CUR_COLS, seed, SC));
  RMM_TRY(launch_sample_indices_i64(h, (uint64_t)m, ceil_log2((uint64_t)m), r, TAG_CUR_ROWS, seed, SR));
  RMM_TRY(rbf_cols_any<T>(h, m, d, Xte, ldte, c, SC, Xtr, ldtr, g, C, ldc));
  RMM_TRY(rbf_cols_any<T>(h, n, d, Xtr, ldtr, r, SR, Xte, ldte, g, Rt, ldrt));
  if (mode == 0) {
    RMM_TRY(launch_sample_indices_i64(h, (uint64_t)m, ceil_log2((uint64_t)m), pc, TAG_CUR_PC, seed, dC));
    RMM_TRY(launch_sample_indices_i64(h, (uint64_t)n, ceil_log2((uint64_t)n), pr, TAG_CUR_PR, seed, dR));
  } else {
    RMM_TRY((orth<T, double>(h, m, c, C, ldc, Qb, m, ob, 64.0 * kEps * (double)(m > c ? m : c), status,
                             ws, 3)));
    RMM_TRY(leverage_scores(h, m, c, Qb, m, q));
    RMM_TRY(weighted_sample(h, m, q, pc, TAG_CUR_PC, seed, cdf, dC));
    RMM_TRY((orth<T, double>(h, n, r, Rt, ldrt, Qb, n, ob, 64.0 * kEps * (double)(n > r ? n : r),
                             status, ws, 3)));
    RMM_TRY(leverage_scores(h, n, r, Qb, n, q));
    RMM_TRY(weighted_sample(h, n, q, pr, TAG_CUR_PR, seed, cdf, dR));
  }
  RMM_TRY(union_sorted(h, m, dC, pc, SR, r, pcm, PC, lens));
  RMM_TRY(union_sorted(h, n, dR, pr, SC, c, prm, PR, lens + 1));
  RMM_TRY(gather_rows<T>(h, pcm, c, PC, lens, C, ldc, Gc));
  RMM_TRY(gather_rows<T>(h, prm, r, PR, lens + 1, Rt, ldrt, Gr));
  RMM_TRY(rbf_block_f64<T>(h, d, Xte, ldte, PC, lens, pcm, Xtr, ldtr, PR, lens + 1, prm, g, Ab));
  RMM_TRY(cholqr2(h, pcm, c, Gc, la, ws));
  RMM_TRY(rank_check(h, c, la.d1, la.d2, 10.0 * (double)pcm * kEps, status));
  RMM_TRY(cholqr2(h, prm, r, Gr, lr, ws));
  RMM_TRY(rank_check(h, r, lr.d1, lr.d2, 10.0 * (double)prm * kEps, status));
  RMM_TRY((gemm<double, double, double, double>(h, false, false, c, c, c, la.R1, c, la.R2, c, 1.0, Ria,
                                                c, ws)));
  RMM_TRY((gemm<double, double, double, double>(h, false, false, r, r, r, lr.R1, r, lr.R2, r, 1.0, Rib,
                                                r, ws)));
  // U = R_a^{-1} Q_a^T A[P_C, P_R] Q_b R_b^{-T}
  RMM_TRY((gemm<double, double, double, double>(h, false, false, (int)pcm, r, prm, Ab, pcm, lr.Q, prm,
                                                1.0, T1, pcm, ws)));
  RMM_TRY((gemm<double, double, double, double>(h, true, false, c, r, pcm, la.Q, pcm, T1, pcm, 1.0, T2,
                                                c, ws)));
  RMM_TRY((gemm<double, double, double, double>(h, false, false, c, r, c, Ria, c, T2, c, 1.0, T3, c,
                                                ws)));
  return gemm<double, double, double, double>(h, false, true, c, r, r, T3, c, Rib, r, 1.0, U, ldu, ws);
}

int spsd_args(rmm_handle h, rmm_dtype dt, int64_t n, int64_t d, double sigma, int64_t s, int64_t p) {
  if (!h || !dt_ok(dt) || n < 1 || d < 1 || s < 1 || s > n || p < 0 || !(sigma > 0.0) ||
      !(sigma < 1e300))
    return RMM_ERR_INVALID_ARG;
  if (n > kUnionMaxDomain || s > 4096 || p > (1 << 20) || d > 64) return RMM_ERR_UNSUPPORTED;
  return RMM_OK;
}

int cur_args(rmm_handle h, rmm_dtype dt, int64_t m, int64_t n, int64_t d, double sigma, int64_t c,
             int64_t r, int64_t pc, int64_t pr, int mode) {
  if (!h || !dt_ok(dt) || m < 1 || n < 1 || d < 1 || c < 1 || r < 1 || c > n || r > m || pc < 0 ||
      pr < 0 || !(sigma > 0.0) || !(sigma < 1e300) || (mode != 0 && mode != 1))
    return RMM_ERR_INVALID_ARG;
  if (mode == 0 && (pc > m || pr > n)) return RMM_ERR_INVALID_ARG;  // without replacement
  if (m > kUnionMaxDomain || n > kUnionMaxDomain || c > 4096 || r > 4096 || pc > (1 << 20) ||
      pr > (1 << 20) || d > 64)
    return RMM_ERR_UNSUPPORTED;
  return RMM_OK;
}

int lsr_args(rmm_handle h, rmm_dtype dt, int64_t m, int64_t d, int64_t s) {
  if (!h || !dt_ok(dt) || m < 1 || d < 1 || s < d || d > m) return RMM_ERR_INVALID_ARG;
  if (d > 4096 || s >= (1ll << 30) || m >= (1ll << 31)) return RMM_ERR_UNSUPPORTED;
  return RMM_OK;
}

}  // namespace

}  // namespace rmm

using namespace rmm;

extern "C" {

int rmm_rsvd_workspace(rmm_handle h, rmm_dtype dt, rmm_precision prec, int64_t m, int64_t n,
                       int64_t k, int64_t p, size_t* bytes) {
  RMM_TRY(rsvd_args(h, dt, prec, m, n, k, p));
  if (!bytes) return RMM_ERR_INVALID_ARG;
  if (prec != RMM_PREC_NATIVE)
    return rsvd_mixed(h, false, prec, m, n, nullptr, m, (int)k, (int)p, 0, 0, nullptr, m, nullptr,
                      nullptr, n, nullptr, bytes);
  if (dt == RMM_F32)
    return rsvd_impl<float>(h, false, m, n, nullptr, m, (int)k, (int)p, 0, 0, nullptr, m, nullptr,
                            nullptr, n, nullptr, bytes);
  return rsvd_impl<double>(h, false, m, n, nullptr, m, (int)k, (int)p, 0, 0, nullptr, m, nullptr,
                           nullptr, n, nullptr, bytes);
}

int rmm_rsvd(rmm_handle h, rmm_dtype dt, rmm_precision prec, int64_t m, int64_t n, const void* A,
             int64_t lda, int64_t k, int64_t p, int64_t q, uint64_t seed, void* U, int64_t ldu,
             void* sigma, void* V, int64_t ldv, int32_t* status) {
  RMM_TRY(rsvd_args(h, dt, prec, m, n, k, p));
  if (!A || !U || !sigma || !V || q < 0 || ld_bad(lda, m) || ld_bad(ldu, m) || ld_bad(ldv, n))
    return RMM_ERR_INVALID_ARG;
  if (prec != RMM_PREC_NATIVE)
    return rsvd_mixed(h, true, prec, m, n, (const float*)A, lda, (int)k, (int)p, (int)q, seed,
                      (float*)U, ldu, (float*)sigma, (float*)V, ldv, status, nullptr);
  if (dt == RMM_F32)
    return rsvd_impl<float>(h, true, m, n, (const float*)A, lda, (int)k, (int)p, (int)q, seed,
                            (float*)U, ldu, (float*)sigma, (float*)V, ldv, status, nullptr);
  return rsvd_impl<double>(h, true, m, n, (const double*)A, lda, (int)k, (int)p, (int)q, seed,
                           (double*)U, ldu, (double*)sigma, (double*)V, ldv, status, nullptr);
}

int rmm_rsvd_faster_workspace(rmm_handle h, rmm_dtype dt, rmm_sketch_kind kind2, int64_t m,
                              int64_t n, int64_t k, int64_t s, int64_t pcs, int64_t p,
                              size_t* bytes) {
  RMM_TRY(rsvd_faster_args(h, dt, kind2, m, n, k, s, pcs, p));
  if (!bytes) return RMM_ERR_INVALID_ARG;
  if (dt == RMM_F32)
    return rsvd_faster_impl<float>(h, false, kind2, m, n, nullptr, m, (int)k, (int)s, pcs, (int)p, 0,
                                   nullptr, m, nullptr, nullptr, n, nullptr, bytes);
  return rsvd_faster_impl<double>(h, false, kind2, m, n, nullptr, m, (int)k, (int)s, pcs, (int)p, 0,
                                  nullptr, m, nullptr, nullptr, n, nullptr, bytes);
}

int rmm_rsvd_faster(rmm_handle h, rmm_dtype dt, rmm_sketch_kind kind2, int64_t m, int64_t n,
                    const void* A, int64_t lda, int64_t k, int64_t s, int64_t pcs, int64_t p,
                    uint64_t seed, void* U, int64_t ldu, void* sigma, void* V, int64_t ldv,
                    int32_t* status) {
  RMM_TRY(rsvd_faster_args(h, dt, kind2, m, n, k, s, pcs, p));
  if (!A || !U || !sigma || !V || ld_bad(lda, m) || ld_bad(ldu, m) || ld_bad(ldv, n))
    return RMM_ERR_INVALID_ARG;
  if (dt == RMM_F32)
    return rsvd_faster_impl<float>(h, true, kind2, m, n, (const float*)A, lda, (int)k, (int)s, pcs,
                                   (int)p, seed, (float*)U, ldu, (float*)sigma, (float*)V, ldv, status,
                                   nullptr);
  return rsvd_faster_impl<double>(h, true, kind2, m, n, (const double*)A, lda, (int)k, (int)s, pcs,
                                  (int)p, seed, (double*)U, ldu, (double*)sigma, (double*)V, ldv,
                                  status, nullptr);
}

int rmm_rsvd_lanczos_workspace(rmm_handle h, rmm_dtype dt, int64_t m, int64_t n, int64_t k,
                               int64_t s, int64_t q, size_t* bytes) {
  if (!h || !dt_ok(dt) || k < 1 || s < 1 || q < 1 || k > s * q || s * q > m || s * q > n || !bytes)
    return RMM_ERR_INVALID_ARG;
  if (s * q > 1024 || m >= (1ll << 31) || n >= (1ll << 30)) return RMM_ERR_UNSUPPORTED;
  if (dt == RMM_F32)
    return lanczos_impl<float>(h, false, m, n, nullptr, m, (int)k, (int)s, (int)q, 0, nullptr, m,
                               nullptr, nullptr, n, nullptr, bytes);
  return lanczos_impl<double>(h, false, m, n, nullptr, m, (int)k, (int)s, (int)q, 0, nullptr, m,
                              nullptr, nullptr, n, nullptr, bytes);
}

int rmm_rsvd_lanczos(rmm_handle h, rmm_dtype dt, int64_t m, int64_t n, const void* A, int64_t lda,
                     int64_t k, int64_t s, int64_t q, uint64_t seed, void* U, int64_t ldu,
                     void* sigma, void* V, int64_t ldv, int32_t* status) {
  if (!h || !dt_ok(dt) || k < 1 || s < 1 || q < 1 || k > s * q || s * q > m || s * q > n)
    return RMM_ERR_INVALID_ARG;
  if (s * q > 1024 || m >= (1ll << 31) || n >= (1ll << 30)) return RMM_ERR_UNSUPPORTED;
  if (!A || !U || !sigma || !V || ld_bad(lda, m) || ld_bad(ldu, m) || ld_bad(ldv, n))
    return RMM_ERR_INVALID_ARG;
  if (dt == RMM_F32)
    return lanczos_impl<float>(h, true, m, n, (const float*)A, lda, (int)k, (int)s, (int)q, seed,
                               (float*)U, ldu, (float*)sigma, (float*)V, ldv, status, nullptr);
  return lanczos_impl<double>(h, true, m, n, (const double*)A, lda, (int)k, (int)s, (int)q, seed,
                              (double*)U, ldu, (double*)sigma, (double*)V, ldv, status, nullptr);
}

int rmm_lsr_workspace(rmm_handle h, rmm_dtype dt, rmm_sketch_kind kind, int64_t m, int64_t d,
                      int64_t s, size_t* bytes) {
  RMM_TRY(lsr_args(h, dt, m, d, s));
  if (!bytes || !kind_ok(kind)) return RMM_ERR_INVALID_ARG;
  if (dt == RMM_F32)
    return lsr_impl<float>(h, false, kind, m, (int)d, nullptr, m, nullptr, s, 0, nullptr, nullptr,
                           nullptr, bytes);
  return lsr_impl<double>(h, false, kind, m, (int)d, nullptr, m, nullptr, s, 0, nullptr, nullptr,
                          nullptr, bytes);
}

int rmm_sketched_lsr(rmm_handle h, rmm_dtype dt, rmm_sketch_kind kind, int64_t m, int64_t d,
                     const void* A, int64_t lda, const void* b, int64_t s, uint64_t seed, double* x,
                     double* resid, int32_t* status) {
  RMM_TRY(lsr_args(h, dt, m, d, s));
  if (!kind_ok(kind) || !A || !b || !x || ld_bad(lda, m)) return RMM_ERR_INVALID_ARG;
  if (kind == RMM_SRHT) {
    const int k = ceil_log2((uint64_t)m);
    if (s > (1ll << k)) return RMM_ERR_INVALID_ARG;
  }
  if (dt == RMM_F32)
    return lsr_impl<float>(h, true, kind, m, (int)d, (const float*)A, lda, (const float*)b, s, seed,
                           x, resid, status, nullptr);
  return lsr_impl<double>(h, true, kind, m, (int)d, (const double*)A, lda, (const double*)b, s, seed,
                          x, resid, status, nullptr);
}

int rmm_precise_lsr_workspace(rmm_handle h, rmm_dtype dt, rmm_sketch_kind kind, int64_t m,
                              int64_t d, int64_t s, size_t* bytes) {
  if (!bytes || !kind_ok(kind)) return RMM_ERR_INVALID_ARG;
  RMM_TRY(lsr_args(h, dt, m, d, s));
  if (d > 1024) return RMM_ERR_UNSUPPORTED;
  if (dt == RMM_F32)
    return lsr_precise_impl<float>(h, false, kind, m, (int)d, nullptr, m, nullptr, s, 0, 0,
                                   nullptr, nullptr, nullptr, bytes);
  return lsr_precise_impl<double>(h, false, kind, m, (int)d, nullptr, m, nullptr, s, 0, 0,
                                  nullptr, nullptr, nullptr, bytes);
}

int rmm_precise_lsr(rmm_handle h, rmm_dtype dt, rmm_sketch_kind kind, int64_t m, int64_t d,
                    const void* A, int64_t lda, const void* b, int64_t s, uint64_t seed,
                    int64_t iters, double* x, double* resid, int32_t* status) {
  RMM_TRY(lsr_args(h, dt, m, d, s));
  if (!kind_ok(kind) || !A || !b || !x || ld_bad(lda, m) || iters < 0) return RMM_ERR_INVALID_ARG;
  if (kind == RMM_SRHT) {
    const int k = ceil_log2((uint64_t)m);
    if (s > (1ll << k)) return RMM_ERR_INVALID_ARG;
  }
  if (d > 1024) return RMM_ERR_UNSUPPORTED;
  if (dt == RMM_F32)
    return lsr_precise_impl<float>(h, true, kind, m, (int)d, (const float*)A, lda,
                                   (const float*)b, s, seed, iters, x, resid, status, nullptr);
  return lsr_precise_impl<double>(h, true, kind, m, (int)d, (const double*)A, lda,
                                  (const double*)b, s, seed, iters, x, resid, status, nullptr);
}

int rmm_lsr_solve_workspace(rmm_handle h, int64_t s, int64_t d, size_t* bytes) {
  if (!h || !bytes || d < 1 || s < d || d > 4096 || s >= (1ll << 30)) return RMM_ERR_INVALID_ARG;
  Carver ws(nullptr, 0);
  ws.take<double>((size_t)s * (d + 1));
  take_ls(ws, s, d);
  *bytes = ws.off + ls_scratch(h, s, d) + 8 * kAlign;
  return RMM_OK;
}

int rmm_lsr_solve(rmm_handle h, rmm_dtype dt, int64_t s, int64_t d, const void* Cs, int64_t ldc,
                  double* x, int32_t* status) {
  if (!h || !dt_ok(dt) || !Cs || !x || d < 1 || s < d || ld_bad(ldc, s)) return RMM_ERR_INVALID_ARG;
  if (d > 4096 || s >= (1ll << 30)) return RMM_ERR_UNSUPPORTED;
  Carver ws(h->ws, h->ws_bytes);
  double* Csd = ws.take<double>((size_t)s * (d + 1));
  LsBufs lb = take_ls(ws, s, d);
  if (ws.off + ls_scratch(h, s, d) + 8 * kAlign > ws.cap) return RMM_ERR_WORKSPACE_TOO_SMALL;
  RMM_TRY(zero_status(h, status));
  if (dt == RMM_F32) RMM_TRY((copy_cast<float, double>(h, s, d + 1, (const float*)Cs, ldc, Csd, s)));
  else RMM_TRY((copy_cast<double, double>(h, s, d + 1, (const double*)Cs, ldc, Csd, s)));
  return ls_solve(h, s, (int)d, Csd, lb, x, status, ws);
}

int rmm_residual_workspace(rmm_handle h, int64_t m, size_t* bytes) {
  if (!h || !bytes || m < 0) return RMM_ERR_INVALID_ARG;
  *bytes = residual_workspace(m) + kAlign;
  return RMM_OK;
}

int rmm_residual(rmm_handle h, rmm_dtype dt, int64_t m, int64_t d, const void* A, int64_t lda,
                 const void* b, const double* x, double* resid) {
  if (!h || !dt_ok(dt) || m < 0 || d < 1 || !b || !x || !resid || (m > 0 && !A) || ld_bad(lda, m))
    return RMM_ERR_INVALID_ARG;
  if (d > (1 << 30) || m >= (1ll << 40)) return RMM_ERR_UNSUPPORTED;
  Carver ws(h->ws, h->ws_bytes);
  if (dt == RMM_F32)
    return residual_norm<float>(h, m, (int)d, (const float*)A, lda, (const float*)b, x, resid, ws);
  return residual_norm<double>(h, m, (int)d, (const double*)A, lda, (const double*)b, x, resid, ws);
}

int rmm_plain_lsr_workspace(rmm_handle h, rmm_dtype dt, int64_t m, int64_t d, size_t* bytes) {
  RMM_TRY(lsr_args(h, dt, m, d, d));
  if (!bytes) return RMM_ERR_INVALID_ARG;
  if (dt == RMM_F32)
    return plain_impl<float>(h, false, m, (int)d, nullptr, m, nullptr, nullptr, nullptr, nullptr, bytes);
  return plain_impl<double>(h, false, m, (int)d, nullptr, m, nullptr, nullptr, nullptr, nullptr, bytes);
}

int rmm_plain_lsr(rmm_handle h, rmm_dtype dt, int64_t m, int64_t d, const void* A, int64_t lda,
                  const void* b, double* x, double* resid, int32_t* status) {
  RMM_TRY(lsr_args(h, dt, m, d, d));
  if (!A || !b || !x || ld_bad(lda, m)) return RMM_ERR_INVALID_ARG;
  if (dt == RMM_F32)
    return plain_impl<float>(h, true, m, (int)d, (const float*)A, lda, (const float*)b, x, resid,
                             status, nullptr);
  return plain_impl<double>(h, true, m, (int)d, (const double*)A, lda, (const double*)b, x, resid,
                            status, nullptr);
}

}  // extern "C"

extern "C" {

int rmm_spsd_faster_workspace(rmm_handle h, rmm_dtype dt, int64_t n, int64_t d, int64_t s,
                              int64_t p, size_t* bytes) {
  RMM_TRY(spsd_args(h, dt, n, d, 1.0, s, p));
  if (!bytes) return RMM_ERR_INVALID_ARG;
  if (dt == RMM_F32)
    return spsd_impl<float>(h, false, n, (int)d, nullptr, d, 1.0, (int)s, p, 0, nullptr, nullptr,
                            nullptr, nullptr, n, nullptr, nullptr, bytes);
  return spsd_impl<double>(h, false, n, (int)d, nullptr, d, 1.0, (int)s, p, 0, nullptr, nullptr,
                           nullptr, nullptr, n, nullptr, nullptr, bytes);
}

int rmm_spsd_faster(rmm_handle h, rmm_dtype dt, int64_t n, int64_t d, const void* X, int64_t ldx,
                    double sigma, int64_t s, int64_t p, uint64_t seed, int64_t* S, int64_t* P,
                    int64_t* np, double* Qc, int64_t ldq, double* Z, int32_t* status) {
  RMM_TRY(spsd_args(h, dt, n, d, sigma, s, p));
  if (!X || !S || !P || !np || !Qc || !Z || ldx < d || ldq < n) return RMM_ERR_INVALID_ARG;
  if (dt == RMM_F32)
    return spsd_impl<float>(h, true, n, (int)d, (const float*)X, ldx, sigma, (int)s, p, seed, S, P, np,
                            Qc, ldq, Z, status, nullptr);
  return spsd_impl<double>(h, true, n, (int)d, (const double*)X, ldx, sigma, (int)s, p, seed, S, P, np,
                           Qc, ldq, Z, status, nullptr);
}

int rmm_cur_faster_workspace(rmm_handle h, rmm_dtype dt, int64_t m, int64_t n, int64_t d, int64_t c,
                             int64_t r, int64_t pc, int64_t pr, int mode, size_t* bytes) {
  RMM_TRY(cur_args(h, dt, m, n, d, 1.0, c, r, pc, pr, mode));
  if (!bytes) return RMM_ERR_INVALID_ARG;
  if (dt == RMM_F32)
    return cur_impl<float>(h, false, m, n, (int)d, nullptr, d, nullptr, d, 1.0, (int)c, (int)r, pc, pr,
                           mode, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, m, nullptr,
                           c, nullptr, n, nullptr, bytes);
  return cur_impl<double>(h, false, m, n, (int)d, nullptr, d, nullptr, d, 1.0, (int)c, (int)r, pc, pr,
                          mode, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, m, nullptr, c,
                          nullptr, n, nullptr, bytes);
}

int rmm_cur_faster(rmm_handle h, rmm_dtype dt, int64_t m, int64_t n, int64_t d, const void* Xtest,
                   int64_t ldte, const void* Xtrain, int64_t ldtr, double sigma, int64_t c,
                   int64_t r, int64_t pc, int64_t pr, int mode, uint64_t seed, int64_t* SC,
                   int64_t* SR, int64_t* PC, int64_t* PR, int64_t* lens, void* C, int64_t ldc,
                   double* U, int64_t ldu, void* Rt, int64_t ldrt, int32_t* status) {
  RMM_TRY(cur_args(h, dt, m, n, d, sigma, c, r, pc, pr, mode));
  if (!Xtest || !Xtrain || !SC || !SR || !PC || !PR || !lens || !C || !U || !Rt || ldte < d ||
      ldtr < d || ldc < m || ldu < c || ldrt < n)
    return RMM_ERR_INVALID_ARG;
  if (dt == RMM_F32)
    return cur_impl<float>(h, true, m, n, (int)d, (const float*)Xtest, ldte, (const float*)Xtrain, ldtr,
                           sigma, (int)c, (int)r, pc, pr, mode, seed, SC, SR, PC, PR, lens, (float*)C,
                           ldc, U, ldu, (float*)Rt, ldrt, status, nullptr);
  return cur_impl<double>(h, true, m, n, (int)d, (const double*)Xtest, ldte, (const double*)Xtrain,
                          ldtr, sigma, (int)c, (int)r, pc, pr, mode, seed, SC, SR, PC, PR, lens,
                          (double*)C, ldc, U, ldu, (double*)Rt, ldrt, status, nullptr);
}

int rmm_leverage_sample_workspace(rmm_handle h, int64_t n, size_t* bytes) {
  if (!h || !bytes || n < 1) return RMM_ERR_INVALID_ARG;
  Carver c(nullptr, 0);
  c.take<uint64_t>((size_t)n);
  *bytes = c.off + kAlign;
  return RMM_OK;
}

int rmm_leverage_sample(rmm_handle h, int64_t n, const double* q, int64_t p, int32_t tag,
                        uint64_t seed, int64_t* out) {
  if (!h || !q || !out || n < 1 || p < 0 || tag < 0) return RMM_ERR_INVALID_ARG;
  Carver ws(h->ws, h->ws_bytes);
  uint64_t* cdf = ws.take<uint64_t>((size_t)n);
  if (!ws.fits()) return RMM_ERR_WORKSPACE_TOO_SMALL;
  return weighted_sample(h, n, q, p, (uint32_t)tag, seed, cdf, out);
}

}  // extern "C"
