// Mixed-precision (BF16 / FP8 e4m3) passes over A for the randomized SVD.
#pragma once

#include "common.hpp"

namespace rmm {

// Round n up to the K granularity of the quantized GEMM (16 elements).
inline int64_t mp_pad(int64_t n) { return (n + 15) / 16 * 16; }
size_t mp_elem_bytes(rmm_precision p);

// sc = per-column scales of A (m x n); Aq: ldq = mp_pad(m) x n column-major,
// Aqt: ldqt = mp_pad(n) x m column-major (A^T), zero padded.
int mp_quantize_matrix(const rmm_ctx* h, rmm_precision p, int64_t m, int64_t n, const float* A,
                       int64_t lda, float* sc, void* Aq, void* Aqt);
// Xq (ld = mp_pad(rows)) = q(rs .* X[:, c] / u_c) per column, zero padded;
// umax: cols words of scratch for the column maxima.
int mp_quantize_cols(const rmm_ctx* h, rmm_precision p, int64_t rows, int64_t cols, const float* X,
                     int64_t ldx, const float* rs, void* Xq, float* u, unsigned* umax);
// C (M x N) = diag(rs) * X^T Y * diag(cs) with X (Kpad x M) and Y (Kpad x N),
// ld = Kpad (a multiple of 16); rs may be null.
int mp_gemm_tn(rmm_ctx* h, rmm_precision p, int M, int N, int64_t Kpad, const void* X, const void* Y,
               const float* rs, const float* cs, float* C, int64_t ldc, Carver& ws);
size_t qgemm_workspace(const rmm_ctx* h, int M, int N, int64_t K);

}  // namespace rmm
