// Dense building blocks used by the drivers (see dense.hip, small.hip).
#pragma once

#include "common.hpp"

namespace rmm {

// C (M x N, ldc) = alpha * op(A) * op(B); op(A) is M x K, op(B) is K x N.
// TC is the MFMA compute type; partial sums need gemm_workspace<TC> bytes.
// With beta != 0 the result is alpha * op(A) op(B) + beta * C.
template <typename TAI, typename TBI, typename TC, typename TO>
int gemm(rmm_ctx* h, bool ta, bool tb, int M, int N, int64_t K, const TAI* A, int64_t lda,
         const TBI* B, int64_t ldb, double alpha, TO* C, int64_t ldc, Carver& ws,
         double beta = 0.0);
template <typename TC>
size_t gemm_workspace(const rmm_ctx* h, int M, int N, int64_t K);

template <typename TI, typename TO>
int copy_cast(const rmm_ctx* h, int64_t rows, int64_t cols, const TI* X, int64_t ldx, TO* Y,
              int64_t ldy);

// out = ||A x - b||_2 (fp64); workspace residual_workspace(m)
template <typename T>
int residual_norm(const rmm_ctx* h, int64_t m, int d, const T* A, int64_t lda, const T* b,
                  const double* x, double* out, Carver& ws);
size_t residual_workspace(int64_t m);

// G (l x l, fp64, symmetric positive semidefinite) = R^T R with R upper
// triangular; writes Rinv = R^{-1} (l x l, ld l, upper) and diag(R).
// Directions whose pivot falls below tau * G_jj are dropped (zero row and
// column in Rinv, zero diagonal) and RMM_STATUS_QR_FALLBACK is raised.
// Above 128 the factorization recurses on 2 x 2 blocks (needs
// cholinv_workspace(h, l) bytes).
int cholinv(rmm_ctx* h, int l, const double* G, int64_t ldg, double tau, double* Rinv,
            double* diag, int32_t* status, Carver& ws);
size_t cholinv_workspace(const rmm_ctx* h, int l);

// Symmetric eigendecomposition by cyclic Jacobi: evals descending, V (l x l,
// ld l) orthonormal eigenvectors.  l <= 1024.
int jacobi_eig(const rmm_ctx* h, int l, const double* G, int64_t ldg, double* evals, double* V,
               int32_t* status, Carver& ws);
size_t jacobi_workspace(int l);
// Block Jacobi used by jacobi_eig for 128 < l <= 1024 (blockjacobi.hip).
int jacobi_eig_block(const rmm_ctx* h, int l, const double* G, int64_t ldg, double* evals, double* V,
                     int32_t* status, Carver& ws);
size_t jacobi_block_workspace(int l);

// SVD of an l x l FP64 matrix by one-sided Jacobi: M J = Ubar diag(sigma)
// with sigma (l, descending, ties by index) the column norms of M J, Ubar
// (l x l, ld l) their normalized columns (zero for sigma = 0) and J (l x l,
// ld l) the accumulated rotations.  l <= 1024.  RMM_STATUS_NOT_CONVERGED is
// raised when the sweep limit is reached.
int jacobi_svd(const rmm_ctx* h, int l, const double* M, int64_t ldm, double* sigma, double* Ubar,
               double* J, int32_t* status, Carver& ws);
size_t jacobi_svd_workspace(int l);
// The same one-sided Jacobi applied directly to the columns of a tall X
// (rows x l, rows >= l, input type TI): X J = Ux diag(sigma) with Ux (rows x
// l, ld rows) the normalized columns; possible when jacobi_svd_direct_ok
// (X fits in one workgroup's LDS, l <= 128).  Workspace jacobi_svd_workspace(l).
bool jacobi_svd_direct_ok(int64_t rows, int l);
template <typename TI>
int jacobi_svd_direct(const rmm_ctx* h, int64_t rows, int l, const TI* X, int64_t ldx, double* sigma,
                      double* Ux, double* J, int32_t* status, Carver& ws);

// G_jj += c * trace(G) (l x l, fp64): the shift of shifted CholeskyQR.
int shift_diag(const rmm_ctx* h, int l, double* G, int64_t ldg, double c);

// Flip (u_i, v_i) so that the largest-magnitude entry of u_i is positive.
template <typename T>
int sign_fix(const rmm_ctx* h, int64_t m, int64_t n, int k, T* U, int64_t ldu, T* V, int64_t ldv);

// status |= RANK_DEFICIENT if min|d1 d2| <= tol * max|d1 d2|
int rank_check(const rmm_ctx* h, int d, const double* d1, const double* d2, double tol,
               int32_t* status);

int zero_status(const rmm_ctx* h, int32_t* status);

// x = Rinv * y for upper-triangular Rinv (d x d) and vector y (both fp64)
int trmv_upper(const rmm_ctx* h, int d, const double* Rinv, const double* y, double* x);

}  // namespace rmm
