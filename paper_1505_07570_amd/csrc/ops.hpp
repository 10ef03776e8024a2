// Internal entry points of the kernels, called by the C ABI layer.
#pragma once

#include "common.hpp"

namespace rmm {

// C (m x s) = A S for an n x s count sketch S of the columns of A (stream of seed)
size_t countsketch_cols_workspace(int64_t n);
template <typename T>
int countsketch_cols_run(rmm_ctx* h, int64_t m, int64_t n, const T* A, int64_t lda, int64_t s,
                         uint64_t seed, T* C, int64_t ldc, Carver& ws);

template <typename T>
size_t countsketch_workspace(const rmm_ctx* h, int64_t m, int ncols, int64_t s);
template <typename T>
int countsketch_run(rmm_ctx* h, int64_t m, int n, const T* A, int64_t lda, const T* b,
                    int64_t s, uint64_t seed, T* C, int64_t ldc, Carver& ws);

template <typename T>
size_t srht_workspace(const rmm_ctx* h, int64_t m, int ncols, int64_t s);
template <typename T>
int srht_run(rmm_ctx* h, int64_t m, int n, const T* A, int64_t lda, const T* b, int64_t s,
             uint64_t seed, T* C, int64_t ldc, Carver& ws);

template <typename T>
size_t gauss_sketch_workspace(const rmm_ctx* h, int64_t m, int ncols, int64_t s);
template <typename T>
int gauss_sketch_run(rmm_ctx* h, int64_t m, int n, const T* A, int64_t lda, const T* b,
                     int64_t s, uint64_t seed, T* C, int64_t ldc, Carver& ws);

// Batch of CountSketch problems (see rmm_sketch_batch): grouped launches when
// every problem takes the scheduled path (s <= 16384), results bitwise equal
// to the solo calls.
template <typename T>
bool countsketch_batch_grouped(int count, const rmm_sketch_desc* d);
template <typename T>
size_t countsketch_batch_workspace(const rmm_ctx* h, int count, const rmm_sketch_desc* d);
template <typename T>
int countsketch_batch_run(rmm_ctx* h, int count, const rmm_sketch_desc* d, Carver& ws);

// C = scale * Omega^T [A | b] with Omega of stream `tag` (the Gaussian-sketch
// kernel with another stream and scale); workspace gauss_sketch_workspace.
template <typename T>
int gauss_project(rmm_ctx* h, int64_t m, int n, const T* A, int64_t lda, const T* b,
                  int64_t s, uint32_t tag, uint64_t seed, double scale, T* C, int64_t ldc,
                  Carver& ws);
// Z (ncols x s, ld ldz) = A^T Qm + beta Z (A m x ncols, Qm m x s): the same
// kernel with a stored left operand; workspace gauss_sketch_workspace<T>(h, m,
// ncols, s).
template <typename T>
int project_tn(rmm_ctx* h, int64_t m, int ncols, const T* A, int64_t lda, const T* Qm, int64_t ldq,
               int64_t s, T* Z, int64_t ldz, Carver& ws, double beta = 0.0);

// Machine-precision LSR iterations (refine.hip): one fused pass over A giving
// per-workgroup partials of A^T r and ||r||^2 for r = [b] - A p (G = refine_groups
// partial rows of d + 1 doubles), and the one-workgroup CG steps.
int refine_groups(const rmm_ctx* h);
size_t refine_part_elems(const rmm_ctx* h, int d);  // doubles of the `part` buffer
template <typename T>
int normal_pass(const rmm_ctx* h, int64_t m, int d, const T* A, int64_t lda, const T* b,
                const double* p, double* part);
int pcg_init(const rmm_ctx* h, int d, const double* part, const double* M, double* g, double* y,
             double* p, double* sc);
int pcg_step(const rmm_ctx* h, int d, const double* part, const double* M, double* x, double* g,
             double* y, double* p, double* sc);
int pass_resid(const rmm_ctx* h, int d, const double* part, double* out);

// Leverage-score sampling and the index/gather kernels of the faster SPSD
// sketching and CUR (spsd.hip).
constexpr int64_t kUnionMaxDomain = 1 << 20;  // domain of union_sorted (LDS bitmap)
int leverage_scores(const rmm_ctx* h, int64_t n, int k, const double* Q, int64_t ldq, double* q);
// p draws with replacement, probability ~ q_i (cdf: n uint64 of workspace)
int weighted_sample(const rmm_ctx* h, int64_t n, const double* q, int64_t p, uint32_t tag,
                    uint64_t seed, uint64_t* cdf, int64_t* out);
// out[0:cap] = sorted unique(a u b) padded with -1, *len = its length
int union_sorted(const rmm_ctx* h, int64_t n, const int64_t* a, int64_t na, const int64_t* b,
                 int64_t nb, int64_t cap, int64_t* out, int64_t* len);
template <typename T>
int gather_rows(const rmm_ctx* h, int64_t pm, int k, const int64_t* P, const int64_t* np, const T* X,
                int64_t ldx, double* G);
template <typename T>
int rbf_block_f64(const rmm_ctx* h, int d, const T* X, int64_t ldx, const int64_t* A,
                  const int64_t* na, int64_t ma, const T* Y, int64_t ldy, const int64_t* B,
                  const int64_t* nb, int64_t mb, double g, double* K);
int rbf_cols_f64(const rmm_ctx* h, int64_t n, int d, const double* X, int64_t ldx, int c,
                 const int64_t* idx, const double* Y, int64_t ldy, double g, double* C, int64_t ldc);
// RBF columns in FP32 (nystrom.hip): C[:, j] = K(X rows, point idx[j] of Y)
int launch_rbf(const rmm_ctx* h, int64_t n, int d, const float* X, int64_t ldx, int c,
               const int64_t* idx, const float* Y, int64_t ldy, int64_t col_base, double g, float* C,
               int64_t ldc);

// Device address of the static scratch array of rmm_sketched_lsr_noalloc on
// `device` (looked up once per device; null when the lookup failed).
void* noalloc_scratch(int device);

int launch_sample_indices_u32(const rmm_ctx* h, uint64_t domain, int k, int64_t s,
                              uint32_t tag, uint64_t seed, uint32_t* out);
int launch_sample_indices_i64(const rmm_ctx* h, uint64_t domain, int k, int64_t s,
                              uint32_t tag, uint64_t seed, int64_t* out);
int launch_cs_hashes(const rmm_ctx* h, int64_t m, int64_t s, uint64_t seed, int32_t* out);
int launch_signs(const rmm_ctx* h, int kind, int64_t m, uint64_t seed, int8_t* out);
template <typename T>
int launch_gaussian(const rmm_ctx* h, uint32_t tag, int64_t rows, int64_t cols, uint64_t seed,
                    T* out, int64_t ld);

}  // namespace rmm
