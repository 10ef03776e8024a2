/*
 * rmm.h -- C ABI of the MI355X (gfx950) randomized sketching library.
 *
 * Operations follow the problem statements of S. Wang, "A Practical Guide to
 * Randomized Matrix Computations with MATLAB Implementations"
 * (arXiv:1505.07570):
 *   - sketching C = S^T A                     (Ch. 3, Sec. 3.2; row form of eq. 4.2)
 *   - randomized k-SVD with subspace iteration (Alg. 5.2, power step of Alg. 5.1)
 *   - sketch-and-solve least squares          (eq. 4.2, Sec. 4.2)
 *   - exact least squares x* = A^+ b           (Sec. 4.1), the "plain" comparator
 *   - Nystrom approximation of an RBF kernel   (Sec. 6.4, kernel of Sec. 6.1.1)
 *
 * Conventions shared by every call
 * --------------------------------
 *  Layout     Matrices are column-major (BLAS convention): element (i, j) of
 *             an r x c matrix X with leading dimension ldx >= max(1, r) is
 *             X[i + j * ldx].
 *  Memory     Every pointer argument named A, b, C, U, V, sigma, x, resid,
 *             status, out is DEVICE memory owned by the caller.  The library
 *             never allocates or frees device memory inside a call: scratch
 *             space is the caller-owned workspace registered with
 *             rmm_set_workspace, sized with the matching *_workspace query.
 *  Streams    All work is enqueued on the stream set by rmm_set_stream
 *             (default: the null stream) and is asynchronous with respect to
 *             the host; no call synchronizes the device.
 *  Errors     Every call returns RMM_OK (0) or a negative rmm_status.
 *             Argument errors are detected on the host before anything is
 *             enqueued.  Numerical conditions found on the device (rank
 *             deficiency, breakdown of the Gram-based orthonormalization,
 *             Jacobi sweeps exhausted) are OR-ed into the int32 status word
 *             passed by the caller (RMM_STATUS_* flags), which is set to 0
 *             at the start of the call.
 *  Randomness Every random quantity is a pure function of (seed, stream tag,
 *             index) through Philox4x32-10 (Salmon et al., SC'11); results
 *             are bitwise reproducible run to run for the same arguments.
 *  Threads    A handle holds a stream, a workspace and cached device
 *             properties; use one handle per host thread.
 */
#ifndef RMM_H
#define RMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rmm_ctx* rmm_handle;

typedef enum { RMM_F32 = 0, RMM_F64 = 1 } rmm_dtype;

/* Sketch families of Sec. 3.2. */
typedef enum {
  RMM_GAUSSIAN = 0,    /* S = G / sqrt(s), G i.i.d. N(0,1)            (Sec. 3.2.1) */
  RMM_SRHT = 1,        /* S = s^{-1/2} D H_N P, zero padding to N = 2^ceil(log2 m)
                          (Sec. 3.2.2)                                             */
  RMM_COUNTSKETCH = 2  /* one +-1 per row of S, uniform bucket       (Sec. 3.2.3, Alg. 3.1) */
} rmm_sketch_kind;

/* Operand precision of the pass-over-A GEMMs of rmm_rsvd. */
typedef enum { RMM_PREC_NATIVE = 0, RMM_PREC_BF16 = 1, RMM_PREC_FP8 = 2 } rmm_precision;

typedef enum {
  RMM_OK = 0,
  RMM_ERR_INVALID_ARG = -1,        /* null pointer, bad size or leading dimension */
  RMM_ERR_WORKSPACE_TOO_SMALL = -2,
  RMM_ERR_HIP = -3,                /* a HIP runtime call failed */
  RMM_ERR_UNSUPPORTED = -4,        /* valid but unsupported combination */
  RMM_ERR_SCRATCH_LIMIT = -5       /* rmm_sketched_lsr_noalloc: the problem needs more
                                      than RMM_NOALLOC_SCRATCH_BYTES of scratch */
} rmm_status;

/* device-side status flags */
#define RMM_STATUS_RANK_DEFICIENT 1  /* sketched LSR: min|R_jj| <= 10 s eps max|R_jj| */
#define RMM_STATUS_QR_FALLBACK 2     /* a CholeskyQR pass met a numerically singular
                                        Gram matrix and dropped directions */
#define RMM_STATUS_NOT_CONVERGED 4   /* Jacobi sweep limit reached */

/* ---- handle ------------------------------------------------------------ */

/* Creates a handle bound to HIP device `device`.  Allocates host memory only. */
int rmm_create(rmm_handle* h, int device);
int rmm_destroy(rmm_handle h);
/* Autotuning of the dense products inside the drivers (rsvd, the LSR solves,
 * Nystrom): with autotune on, the first product of each new shape (types,
 * transposes, M, N, K) runs every candidate launch plan (column tile,
 * workgroups per CU of the K split, 128 x 128 fast path or not) twice on the
 * caller's operands, timed on the handle's stream, and the fastest is kept in
 * the handle for that shape; later calls use it whether or not autotune is
 * on.  Tuning synchronizes the stream: off by default, not during graph
 * capture.  The plans can be saved to and loaded from a text file (one
 * "key<TAB>plan" line per shape); rmm_create loads the file named by the
 * environment variable RMM_TUNE_CACHE when it is set.  A tuned plan changes
 * only the order of the FP64/FP32 partial sums, within the stated
 * tolerances; the same handle state gives bitwise-identical results.
 * count: the number of shapes with a kept plan. */
int rmm_set_autotune(rmm_handle h, int on);
int rmm_autotune_count(rmm_handle h, int64_t* count);
int rmm_autotune_save(rmm_handle h, const char* path);
int rmm_autotune_load(rmm_handle h, const char* path);
/* Kernel timing: with it on, the handle records a HIP event on its stream
 * right before and right after the main kernel of each sketch (the
 * CountSketch scatter-add, the SRHT transform and sample, the Gaussian
 * product; not the index, schedule or reduction kernels around them),
 * whether it runs for rmm_sketch or inside a driver; the grouped CountSketch
 * launch of rmm_sketch_batch is not timed.  rmm_kernel_time waits for the later event and
 * returns the milliseconds between the two of the last such kernel; it
 * returns RMM_ERR_INVALID_ARG when timing is off or no kernel has been
 * timed since it was turned on.  Off by default (the events serialize
 * nothing, but are not meant for graph capture). */
int rmm_set_kernel_timing(rmm_handle h, int on);
int rmm_kernel_time(rmm_handle h, float* ms);
/* Measurement hook (no section of the paper): reads `bytes` of device memory
 * at x once with 16-byte nontemporal loads, the access pattern of the
 * library's HBM-bound passes without their arithmetic, and writes 4096 floats (one
 * partial sum per workgroup) to the device buffer sink.  Its rate is the
 * practical HBM read ceiling that the bench reports beside the rated peak.
 * Requires bytes >= 16, bytes and x multiples of 16.  Asynchronous on the
 * handle's stream. */
int rmm_stream_read(rmm_handle h, const void* x, int64_t bytes, float* sink);

/* Sets the hipStream_t (passed as void*) on which later calls enqueue work. */
int rmm_set_stream(rmm_handle h, void* hip_stream);
/* Registers caller-owned device scratch memory (256-byte aligned). */
int rmm_set_workspace(rmm_handle h, void* dptr, size_t bytes);
/* Human-readable name of an rmm_status code. */
const char* rmm_strerror(int code);
/* Number of compute units of the handle's device. */
int rmm_device_cus(rmm_handle h, int* cus);

/* ---- sketching (Ch. 3) ----------------------------------------------------
 * C = S^T [A | b]: A is m x n (lda >= m), b an optional extra column of
 * length m (NULL for none).  C is s x n' with n' = n + (b != NULL), ldc >= s.
 * The extra column is sketched with the same S (the joint sketch of [A, b]
 * used by InexactLSR, Sec. 4.2.1).  S is m x s:
 *   GAUSSIAN     S[i, r] = Omega[i, r] / sqrt(s), Omega from stream tag 4
 *   SRHT         S[i, r] = d_i H[i, idx_r] / sqrt(s); H Sylvester-ordered
 *                (H[i, r] = (-1)^popcount(i & r)); idx = sorted sample of s
 *                distinct rows of [0, N); requires s <= N (else
 *                RMM_ERR_INVALID_ARG), s <= 8192 (each workgroup keeps one
 *                accumulator per sampled row in registers; larger s is
 *                RMM_ERR_UNSUPPORTED) and N <= 2^30
 *   COUNTSKETCH  S[i, h_i] = g_i, zero elsewhere; no scaling
 * m = 0 yields C = 0.  Requires n >= 0, s >= 1. */
int rmm_sketch_workspace(rmm_handle h, rmm_dtype dt, rmm_sketch_kind kind,
                         int64_t m, int64_t n_total, int64_t s, size_t* bytes);
int rmm_sketch(rmm_handle h, rmm_dtype dt, rmm_sketch_kind kind, int64_t m,
               int64_t n, const void* A, int64_t lda, const void* b, int64_t s,
               uint64_t seed, void* C, int64_t ldc);

/* Composite sketch (Sec. 3.2.4): C = S^T [A | b] with S = S_cs S_2, an
 * m x s1 COUNTSKETCH followed by an s1 x s sketch of kind `kind2` (GAUSSIAN,
 * the section's GaussianProjection+CountSketch, or SRHT, the combination
 * the paper suggests with the faster k-SVD of Sec. 5.3).  Both factors are
 * the rmm_sketch operators above, drawn from the same seed (their streams
 * differ by tag): the call equals rmm_sketch(COUNTSKETCH, s1) into an
 * s1 x n' buffer followed by rmm_sketch(kind2, s) of that buffer.  The
 * intermediate lives in the workspace.  C is s x n', ldc >= s.  Requires
 * s1 >= 1, s >= 1 and, for SRHT, s <= N = 2^ceil(log2 s1); kind2 =
 * COUNTSKETCH is RMM_ERR_UNSUPPORTED. */
int rmm_sketch_composite_workspace(rmm_handle h, rmm_dtype dt, rmm_sketch_kind kind2,
                                   int64_t m, int64_t n_total, int64_t s1, int64_t s,
                                   size_t* bytes);
int rmm_sketch_composite(rmm_handle h, rmm_dtype dt, rmm_sketch_kind kind2, int64_t m,
                         int64_t n, const void* A, int64_t lda, const void* b, int64_t s1,
                         int64_t s, uint64_t seed, void* C, int64_t ldc);

/* ---- batches of sketches (grouped execution) ----------------------------------
 * One call sketches `count` independent problems of different shapes, each
 * as in rmm_sketch (C_i = S_i^T [A_i | b_i] with its own s_i and seed_i; A_i
 * m_i x n_i column-major, b_i optional).  descs is a HOST array of `count`
 * descriptors; the pointers in it are device pointers.  For COUNTSKETCH with
 * every s_i <= 16384 the batch runs as one grouped launch per stage over a
 * descriptor table uploaded to the workspace (hipMemcpyAsync on the handle's
 * stream); otherwise the problems run one after another.  Either way each
 * C_i is bitwise identical to rmm_sketch on problem i alone.  Workspace from
 * rmm_sketch_batch_workspace with the same descriptors. */
typedef struct {
  int64_t m, n;      /* A is m x n */
  const void* A;
  int64_t lda;
  const void* b;     /* optional extra column (NULL: none) */
  int64_t s;
  uint64_t seed;
  void* C;           /* s x (n + (b != NULL)), ldc >= s */
  int64_t ldc;
} rmm_sketch_desc;
int rmm_sketch_batch_workspace(rmm_handle h, rmm_dtype dt, rmm_sketch_kind kind,
                               int64_t count, const rmm_sketch_desc* descs,
                               size_t* bytes);
int rmm_sketch_batch(rmm_handle h, rmm_dtype dt, rmm_sketch_kind kind, int64_t count,
                     const rmm_sketch_desc* descs);

/* ---- admission for serving (host only; no device calls) ---------------------
 * A first-come-first-served queue of requests, each holding `bytes` of
 * device memory while it runs, under a total budget.  rmm_sched_admit moves
 * queued requests to running, in arrival order, while they fit next to the
 * running ones, and stops at the first that does not (no starvation);
 * rmm_sched_complete releases a running request.  A request larger than the
 * budget is rejected by rmm_sched_submit (RMM_ERR_INVALID_ARG), as is a
 * duplicate id.  Not thread safe: one scheduler per serving thread. */
typedef struct rmm_sched* rmm_sched_t;
int rmm_sched_create(size_t budget_bytes, rmm_sched_t* out);
int rmm_sched_destroy(rmm_sched_t s);
int rmm_sched_submit(rmm_sched_t s, int64_t id, size_t bytes);
int rmm_sched_admit(rmm_sched_t s, int64_t max_ids, int64_t* ids, int64_t* n);
int rmm_sched_complete(rmm_sched_t s, int64_t id);
int rmm_sched_stats(rmm_sched_t s, size_t* in_use, int64_t* queued, int64_t* running);

/* ---- randomized k-SVD (Alg. 5.2 with the subspace iteration of Alg. 5.1) --
 * A (m x n) ~ U diag(sigma) V^T with U m x k (ldu >= m), sigma k entries,
 * V n x k (ldv >= n), all in dtype dt.  l = k + p <= min(m, n); q >= 0 is the
 * number of A A^T applications, the basis being re-orthonormalized after
 * every product.  Singular values are descending; each u_i has its
 * largest-magnitude entry positive.  prec selects the operand precision of
 * the passes over A (RMM_PREC_NATIVE: dt itself; BF16/FP8 need dt = RMM_F32
 * and accumulate in FP32); orthonormalization and the small SVD are FP64.
 * Orthonormalization is shifted CholeskyQR (a shifted first pass, then one
 * more pass inside the subspace iteration and two for the final basis); the
 * small SVD of B = Q^T A is taken from Z = A^T Q = B^T: Z = Q_z M_z (shifted
 * CholeskyQR, M_z = Q_z^T Z), then one-sided Jacobi on the l x l M_z, so
 * sigma carries an absolute error of order eps * sigma_1 (the condition
 * number is not squared).  l <= 1024.
 * status: device int32, see RMM_STATUS_*. */
int rmm_rsvd_workspace(rmm_handle h, rmm_dtype dt, rmm_precision prec,
                       int64_t m, int64_t n, int64_t k, int64_t p, size_t* bytes);
int rmm_rsvd(rmm_handle h, rmm_dtype dt, rmm_precision prec, int64_t m,
             int64_t n, const void* A, int64_t lda, int64_t k, int64_t p,
             int64_t q, uint64_t seed, void* U, int64_t ldu, void* sigma,
             void* V, int64_t ldv, int32_t* status);

/* Faster randomized k-SVD (Sec. 5.3, Alg. 5.3): two passes over A.
 *   C = A S            S an n x s count sketch of the columns (stream seed + 1)
 *   L = P^T A, D = P^T C   P = P_cs P_2 (rmm_sketch_composite with p_cs and p,
 *                      stream seed; kind2 = SRHT as in the algorithm, or
 *                      GAUSSIAN as in its listing)
 *   Q_D R_D = D        CholeskyQR2 in FP64
 *   Ubar Sigmabar Vbar^T = rank-k SVD of Q_D^T L (s x n), FP64
 *   U Sigma Vhat^T = SVD of C R_D^{-1} Ubar Sigmabar (m x k), FP64;  V = Vbar Vhat
 * (both SVDs as the small SVD of rmm_rsvd: shifted CholeskyQR of the tall
 * factor, then one-sided Jacobi)
 * A is m x n (lda >= m); U m x k (ldu >= m), sigma k (descending), V n x k
 * (ldv >= n), in the input type, signs as rmm_rsvd.  Requires 1 <= k <= s <=
 * p <= p_cs, s <= 1024, p <= N = 2^ceil(log2 p_cs) for SRHT.  status as
 * rmm_rsvd (RANK_DEFICIENT when D is numerically rank deficient). */
/* k-SVD by the block Lanczos method (Sec. 5.1, Alg. 5.1): q Krylov blocks
 * K = [C, (A A^T) C, ..., (A A^T)^{q-1} C], C = A Omega (Omega n x s, the
 * stream of rmm_rsvd); each block after the first is (A A^T) of the previous
 * orthonormal block, orthogonalized against all earlier ones (two passes of
 * block Gram-Schmidt) and orthonormalized (shifted CholeskyQR, three
 * passes), so Q_C (m x sq) spans range(K).
 * Then B = Q_C^T A, its top-k SVD, U = Q_C Ubar; outputs, signs and status
 * as rmm_rsvd.  Requires 1 <= k <= s q <= min(m, n), s q <= 1024. */
int rmm_rsvd_lanczos_workspace(rmm_handle h, rmm_dtype dt, int64_t m, int64_t n, int64_t k,
                               int64_t s, int64_t q, size_t* bytes);
int rmm_rsvd_lanczos(rmm_handle h, rmm_dtype dt, int64_t m, int64_t n, const void* A,
                     int64_t lda, int64_t k, int64_t s, int64_t q, uint64_t seed, void* U,
                     int64_t ldu, void* sigma, void* V, int64_t ldv, int32_t* status);

int rmm_rsvd_faster_workspace(rmm_handle h, rmm_dtype dt, rmm_sketch_kind kind2, int64_t m,
                              int64_t n, int64_t k, int64_t s, int64_t p_cs, int64_t p,
                              size_t* bytes);
int rmm_rsvd_faster(rmm_handle h, rmm_dtype dt, rmm_sketch_kind kind2, int64_t m, int64_t n,
                    const void* A, int64_t lda, int64_t k, int64_t s, int64_t p_cs, int64_t p,
                    uint64_t seed, void* U, int64_t ldu, void* sigma, void* V, int64_t ldv,
                    int32_t* status);

/* ---- least squares (Ch. 4) --------------------------------------------------
 * Sketch-and-solve (eq. 4.2): x~ = argmin ||S^T (A x - b)||_2 with one S of
 * the given kind applied to [A | b] (A m x d, lda >= m; b length m; d <= s).
 * The s x (d+1) sketch is promoted to FP64 and solved by CholeskyQR2;
 * x (d doubles) and, if resid != NULL, resid = ||A x~ - b||_2 (one double)
 * are written in FP64.  status: RMM_STATUS_RANK_DEFICIENT when the sketched
 * system is numerically rank deficient. */
int rmm_lsr_workspace(rmm_handle h, rmm_dtype dt, rmm_sketch_kind kind,
                      int64_t m, int64_t d, int64_t s, size_t* bytes);
int rmm_sketched_lsr(rmm_handle h, rmm_dtype dt, rmm_sketch_kind kind,
                     int64_t m, int64_t d, const void* A, int64_t lda,
                     const void* b, int64_t s, uint64_t seed, double* x,
                     double* resid, int32_t* status);
/* rmm_sketched_lsr without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and results as
 * rmm_sketched_lsr (bitwise); the scratch comes from a static device array of
 * RMM_NOALLOC_SCRATCH_BYTES (128 MiB) per device, set up by rmm_create and
 * held until the process ends.  The handle's registered workspace is neither
 * used nor changed.  Nothing is allocated: no hipMalloc, hipFree or
 * allocating library call.  Returns RMM_ERR_SCRATCH_LIMIT when
 * rmm_lsr_workspace reports more than RMM_NOALLOC_SCRATCH_BYTES (e.g. the
 * Gaussian sketch of a 2^20 x 257 FP32 [A | b] to s = 4096, whose split-K
 * partials alone take 270 MB; CountSketch and SRHT of that problem fit) and
 * RMM_ERR_HIP when the array's address could not be looked up.  Every call
 * on one device shares that device's array: calls that overlap on one device
 * (two streams, two host threads) race and give wrong results. */
#define RMM_NOALLOC_SCRATCH_BYTES (128u << 20)
int rmm_sketched_lsr_noalloc(rmm_handle h, rmm_dtype dt, rmm_sketch_kind kind, int64_t m,
                             int64_t d, const void* A, int64_t lda, const void* b, int64_t s,
                             uint64_t seed, double* x, double* resid, int32_t* status);
/* Machine-precision least squares (Alg. 4.1, Sec. 4.3): the sketch of [A | b]
 * gives the preconditioner T = R^{-1} (R from the FP64 CholeskyQR2 of S^T A)
 * and the start x0 (the sketch-and-solve solution of rmm_sketched_lsr); then
 * `iters` conjugate-gradient steps on the normal equations of A T (the
 * reading of the printed gradient step, whose step size the paper leaves
 * open), each one pass over A in FP64 arithmetic.  With s a small multiple
 * of d, A T is well conditioned and each step gains a constant factor, so a
 * few tens of steps reach x* = A^+ b to machine precision.  Arguments as for
 * rmm_sketched_lsr plus iters >= 0 (0 returns x0); d <= 1024
 * (RMM_ERR_UNSUPPORTED above).  x and resid = ||A x - b||_2 (if non-NULL)
 * are FP64 device buffers. */
int rmm_precise_lsr_workspace(rmm_handle h, rmm_dtype dt, rmm_sketch_kind kind,
                              int64_t m, int64_t d, int64_t s, size_t* bytes);
int rmm_precise_lsr(rmm_handle h, rmm_dtype dt, rmm_sketch_kind kind, int64_t m,
                    int64_t d, const void* A, int64_t lda, const void* b, int64_t s,
                    uint64_t seed, int64_t iters, double* x, double* resid,
                    int32_t* status);
/* The two halves of rmm_sketched_lsr, for callers that sketch once and
 * solve separately.  rmm_lsr_solve: x = argmin ||Cs[:, :d] x - Cs[:, d]||_2
 * for an s x (d+1) sketched system Cs (ldc >= s, dtype dt, device), solved
 * in FP64 by CholeskyQR2 (eq. 4.2; the backslash of InexactLSR, Sec. 4.2.1);
 * status as for rmm_sketched_lsr.  rmm_residual: resid = ||A x - b||_2 in
 * FP64 (one pass over A; x is d doubles on the device). */
int rmm_lsr_solve_workspace(rmm_handle h, int64_t s, int64_t d, size_t* bytes);
int rmm_lsr_solve(rmm_handle h, rmm_dtype dt, int64_t s, int64_t d, const void* Cs,
                  int64_t ldc, double* x, int32_t* status);
int rmm_residual_workspace(rmm_handle h, int64_t m, size_t* bytes);
int rmm_residual(rmm_handle h, rmm_dtype dt, int64_t m, int64_t d, const void* A,
                 int64_t lda, const void* b, const double* x, double* resid);
/* Exact solution x* = A^+ b (Sec. 4.1) by FP64 CholeskyQR2 of A itself: the
 * "plain" comparator. Same argument conventions as rmm_sketched_lsr. */
int rmm_plain_lsr_workspace(rmm_handle h, rmm_dtype dt, int64_t m, int64_t d,
                            size_t* bytes);
int rmm_plain_lsr(rmm_handle h, rmm_dtype dt, int64_t m, int64_t d,
                  const void* A, int64_t lda, const void* b, double* x,
                  double* resid, int32_t* status);

/* ---- Nystrom approximation of an RBF kernel matrix (Sec. 6.4; kernel of
 * Sec. 6.1.1) -----------------------------------------------------------------
 * X: n points of dimension d (row-major n x d fp32, ldx >= d, device).
 * K_ij = exp(-||x_i - x_j||^2 / (2 sigma^2)) is never formed.
 *   idx (c int64)     S, c sorted indices drawn uniformly without replacement
 *                     from [0, n) (stream tag 6)
 *   C (n x c fp32, ldc >= n, column-major)   K[:, S]
 *   evals (c doubles) eigenvalues of W = K[S, S] (computed in FP64), descending
 *   L (n x k fp32, ldl >= n)  C U_k Lam_k^{-1/2}, so that K ~ L L^T =
 *                     C W_k^+ C^T; eigenvalues <= c * 2^-52 * lambda_max give
 *                     zero columns; L = C F is an FP32 product with
 *                     F = U_k Lam_k^{-1/2} formed in FP64 and rounded once
 * The eigensolver of W is cyclic Jacobi in FP64 (one workgroup for c <= 128,
 * block Jacobi above).  For c > 128, outside stream capture, the call reads
 * each sweep's convergence flag on the host one sweep after enqueueing it
 * (so it returns once the sweeps are decided, with the last work still
 * queued); under capture it enqueues the maximum number of sweeps, of which
 * those after convergence return at once.
 * Requires 1 <= k <= c <= n; d <= 64 and c <= 1024 (RMM_ERR_UNSUPPORTED
 * beyond).  status: RMM_STATUS_NOT_CONVERGED from the eigensolver. */
int rmm_nystrom_workspace(rmm_handle h, int64_t n, int64_t d, int64_t c, int64_t k,
                          size_t* bytes);
int rmm_nystrom(rmm_handle h, int64_t n, int64_t d, const float* X, int64_t ldx,
                double sigma, int64_t c, int64_t k, uint64_t seed, int64_t* idx,
                float* C, int64_t ldc, float* L, int64_t ldl, double* evals,
                int32_t* status);

/* Gaussian-projection variant of the Nystrom method (the W = S^T K S form of
 * Sec. 6.4 with a Gaussian S): C = K Omega (n x c fp32, ldc >= n), Omega
 * (n x c, i.i.d. N(0,1), stream tag 7) regenerated from the seed,
 * W = Omega^T C (FP64), W = U Lam U^T, L = C U_k Lam_k^{-1/2} (n x k fp32,
 * ldl >= n) with the same zero-eigenvalue cut as rmm_nystrom.  K is formed
 * tile by tile only.  Same limits, eigensolver and host behaviour as
 * rmm_nystrom. */
int rmm_nystrom_gaussian_workspace(rmm_handle h, int64_t n, int64_t d, int64_t c,
                                   int64_t k, size_t* bytes);
int rmm_nystrom_gaussian(rmm_handle h, int64_t n, int64_t d, const float* X,
                         int64_t ldx, double sigma, int64_t c, int64_t k, uint64_t seed,
                         float* C, int64_t ldc, float* L, int64_t ldl, double* evals,
                         int32_t* status);

/* ---- faster SPSD sketching (Sec. 6.3, Alg. 6.1) of the RBF kernel ----------
 * K_ij = exp(-||x_i - x_j||^2 / (2 sigma^2)) on the rows of X (n x d, dtype
 * dt, row-major, ldx >= d, d <= 64, n <= 2^20), never formed:
 *   S  (s int64, device): sorted uniform sample of [n] without replacement
 *   C = K[:, S] (in dt), Q_C (n x s FP64, ldq >= n): its orthonormal basis
 *      by shifted CholeskyQR (three passes)
 *   q_i = ||Q_C[i, :]||^2 (the leverage scores of the columns of C^T,
 *      Sec. 3.3.2); p draws with replacement with probability ~ q_i, by an
 *      inverse CDF over the integer weights floor(q_i 2^32 + 1/2) (stream
 *      seed, see rmm_leverage_sample)
 *   P  (capacity p + s int64): unique([draws; S]), sorted, padded with -1;
 *      *np (one int64, device) its length
 *   Z (s x s FP64, ld s) = (Q_C[P, :])^+ K[P, P] ((Q_C[P, :])^+)^T, K[P, P]
 *      in FP64, the pseudo-inverse from CholeskyQR2 of Q_C[P, :]
 * so that K ~ Q_C Z Q_C^T.  status: RANK_DEFICIENT if Q_C[P, :] is
 * numerically rank deficient (then Z uses a generalized inverse),
 * QR_FALLBACK if C is.  Requires 1 <= s <= n, s <= 4096, 0 <= p <= 2^20. */
int rmm_spsd_faster_workspace(rmm_handle h, rmm_dtype dt, int64_t n, int64_t d, int64_t s,
                              int64_t p, size_t* bytes);
int rmm_spsd_faster(rmm_handle h, rmm_dtype dt, int64_t n, int64_t d, const void* X, int64_t ldx,
                    double sigma, int64_t s, int64_t p, uint64_t seed, int64_t* S, int64_t* P,
                    int64_t* np, double* Qc, int64_t ldq, double* Z, int32_t* status);

/* ---- faster CUR decomposition (Sec. 6.6.3) of the RBF kernel ------------------
 * A = K(Xtest, Xtrain) (m x n; Xtest m x d and Xtrain n x d row-major, dtype
 * dt, m, n <= 2^20, d <= 64), never formed:
 *   SC (c of n) and SR (r of m): sorted uniform samples (int64, device)
 *   C = A[:, SC] (m x c, dt, ldc >= m); Rt = A[SR, :]^T (n x r, dt,
 *      ldrt >= n: R returned transposed, column-major)
 *   P_C (capacity p_c + r) and P_R (capacity p_r + c): mode 0 (the curFaster
 *      listing) draws p_c of m and p_r of n uniformly without replacement;
 *      mode 1 (the remark) draws them with replacement by the leverage scores
 *      of C^T and R (as rmm_spsd_faster does); then P_C = unique([P_C; SR]),
 *      P_R = unique([P_R; SC]), sorted, padded with -1; lens[0], lens[1]
 *      (int64, device) their lengths
 *   U (c x r FP64, ldu >= c) = (C[P_C, :])^+ A[P_C, P_R] (R[:, P_R])^+, the
 *      block A[P_C, P_R] in FP64, pseudo-inverses from CholeskyQR2
 * so that A ~ C U R.  status as rmm_spsd_faster.  Requires 1 <= c <= n,
 * 1 <= r <= m, c, r <= 4096; mode 0 needs p_c <= m, p_r <= n. */
int rmm_cur_faster_workspace(rmm_handle h, rmm_dtype dt, int64_t m, int64_t n, int64_t d, int64_t c,
                             int64_t r, int64_t pc, int64_t pr, int mode, size_t* bytes);
int rmm_cur_faster(rmm_handle h, rmm_dtype dt, int64_t m, int64_t n, int64_t d, const void* Xtest,
                   int64_t ldte, const void* Xtrain, int64_t ldtr, double sigma, int64_t c,
                   int64_t r, int64_t pc, int64_t pr, int mode, uint64_t seed, int64_t* SC,
                   int64_t* SR, int64_t* PC, int64_t* PR, int64_t* lens, void* C, int64_t ldc,
                   double* U, int64_t ldu, void* Rt, int64_t ldrt, int32_t* status);

/* Leverage-score sampling (Sec. 3.3.2), test hook: out[j] (j < p) is drawn
 * with probability ~ q_i from q (n FP64 >= 0, device): weights w_i =
 * floor(q_i 2^32 + 1/2), target t_j = floor(r_j W / 2^64) with r_j the 64-bit
 * uniform (w0 << 32 | w1) of Philox at counter (j, tag, 0) and W = sum w_i,
 * out[j] = the first i with w_0 + ... + w_i > t_j.  Integer arithmetic
 * throughout, so the indices are exact.  Needs
 * rmm_leverage_sample_workspace bytes of workspace. */
int rmm_leverage_sample_workspace(rmm_handle h, int64_t n, size_t* bytes);
int rmm_leverage_sample(rmm_handle h, int64_t n, const double* q, int64_t p, int32_t tag,
                        uint64_t seed, int64_t* out);

/* ---- mixed-precision product (test hook for the BF16 / FP8 passes of rsvd) --
 * A (m x n fp32, lda >= m) is quantized per column (scale = max |A_ij| / QMAX,
 * QMAX = 1 for BF16 and 448 for FP8 e4m3, round to nearest even) and the
 * small operand X is quantized per column after the column scales of A are
 * folded in (mode 0) or not (mode 1); the MFMA product accumulates in FP32:
 *   mode 0: out (m x l, ldo >= m) = A X with X n x l (ldx >= n)
 *   mode 1: out (n x l, ldo >= n) = A^T X with X m x l (ldx >= m)
 * All pointers device; workspace from rmm_mixed_product_workspace. */
int rmm_mixed_product_workspace(rmm_handle h, rmm_precision prec, int64_t m, int64_t n,
                                int64_t l, size_t* bytes);
int rmm_mixed_product(rmm_handle h, rmm_precision prec, int mode, int64_t m, int64_t n,
                      const float* A, int64_t lda, const float* X, int64_t ldx, int64_t l,
                      float* out, int64_t ldo);

/* ---- random quantities (test hooks; Sec. 3.2, Alg. 3.1) ------------------- */
/* CountSketch buckets h_i in [0, s) for rows 0..m-1 (int32, device). */
int rmm_sketch_hashes(rmm_handle h, int64_t m, int64_t s, uint64_t seed,
                      int32_t* out);
/* Row signs (+1 / -1, int8, device) of CountSketch (kind = RMM_COUNTSKETCH)
 * or of the SRHT diagonal D (kind = RMM_SRHT). */
int rmm_sketch_signs(rmm_handle h, rmm_sketch_kind kind, int64_t m,
                     uint64_t seed, int8_t* out);
/* SRHT sample: s sorted distinct indices of [0, N), N = 2^ceil(log2 m),
 * int64, device.  Requires 1 <= s <= min(N, 8192). */
int rmm_srht_indices(rmm_handle h, int64_t m, int64_t s, uint64_t seed,
                     int64_t* out);
/* Gaussian matrix Omega (rows x cols, ld >= rows) of stream `stream`
 * (0: sketch, 1: rsvd, 2: Nystrom) in dtype dt. */
int rmm_gaussian(rmm_handle h, rmm_dtype dt, int stream, int64_t rows,
                 int64_t cols, uint64_t seed, void* out, int64_t ld);

#ifdef __cplusplus
}
#endif

#endif /* RMM_H */
