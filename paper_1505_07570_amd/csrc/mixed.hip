// Mixed-precision passes over A for the randomized SVD: BF16 or FP8 (e4m3)
// MFMA operands with per-column scales and FP32 accumulation.
//
// A (m x n, fp32) is quantized once, column by column: sc_j = max_i |A_ij| /
// QMAX and Aq = q(A / sc).  Two copies are written, column-major (Aq) and
// row-major (Aq^T stored column-major), so that both products of a
// subspace-iteration step are the same K-contiguous form C = X^T Y:
//     Z = A^T Q  = diag(sc) * (Aq^T Qq) * diag(uq)        X = Aq,   Y = Qq
//     Y = A Qz   = (Aq_t^T Xq) * diag(ux)                 X = Aq_t, Y = Xq,
// where Xq = q(diag(sc) Qz / ux) carries the column scales of A on its rows
// and Qq = q(Q / uq); uq, ux are per-column scales of the small operands.
// The orthonormalization and the small SVD stay in fp64 (drivers.hip).
#include <hip/hip_bf16.h>

#include "common.hpp"
#include "dense.hpp"
#include "mixed.hpp"

namespace rmm {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef short shortx4 __attribute__((ext_vector_type(4)));

// ---- element formats ----------------------------------------------------------------

struct Bf16Fmt {
  using store_t = uint16_t;
  static constexpr float QMAX = 1.0f;  // scaling keeps |x| <= 1; bf16 has fp32's range
  static constexpr int KPL = 4;        // K elements per lane per MFMA (16x16x16)
  static __device__ __forceinline__ uint16_t enc(float x) {
    // round to nearest even
    const uint32_t u = __float_as_uint(x);
    const uint32_t r = u + 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(r >> 16);
  }
};
struct Fp8Fmt {
  using store_t = uint8_t;
  static constexpr float QMAX = 448.0f;  // OCP e4m3 largest finite value
  static constexpr int KPL = 8;          // 16x16x32
  static __device__ __forceinline__ uint8_t enc(float x) {
    return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(x, 0.0f, 0, false) & 0xFF);
  }
};

template <typename F>
__device__ __forceinline__ floatx4 qmfma(uint64_t a, uint64_t b, floatx4 c);
template <>
__device__ __forceinline__ floatx4 qmfma<Bf16Fmt>(uint64_t a, uint64_t b, floatx4 c) {
  shortx4 x, y;
  __builtin_memcpy(&x, &a, 8);
  __builtin_memcpy(&y, &b, 8);
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(x, y, c, 0, 0, 0);
}
template <>
__device__ __forceinline__ floatx4 qmfma<Fp8Fmt>(uint64_t a, uint64_t b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8((long)a, (long)b, c, 0, 0, 0);
}

// ---- quantization ----------------------------------------------------------------

// four values encoded and packed into consecutive elements (little-endian)
template <typename F>
__device__ __forceinline__ void enc4(const float v[4], typename F::store_t out[4]) {
#pragma unroll
  for (int e = 0; e < 4; ++e) out[e] = F::enc(v[e]);
}

// sc[j] = max_i |A_ij| / QMAX (1 for an all-zero column); one workgroup per
// column, 16-byte loads when the column is aligned
template <typename F>
__global__ __launch_bounds__(256) void colscale_kernel(int64_t m, const float* __restrict__ A,
                                                       int64_t lda, float* __restrict__ sc) {
  __shared__ float red[256];
  const float* col = A + (int64_t)blockIdx.x * lda;
  float mx = 0.f;
  int64_t i0 = 0;
  if ((uintptr_t)col % 16 == 0) {
    const int64_t m4 = m / 4 * 4;
    for (int64_t i = 4 * (int64_t)threadIdx.x; i < m4; i += 1024) {
      const float4 x = *reinterpret_cast<const float4*>(col + i);
      mx = fmaxf(mx, fmaxf(fmaxf(fabsf(x.x), fabsf(x.y)), fmaxf(fabsf(x.z), fabsf(x.w))));
    }
    i0 = m4;
  }
  for (int64_t i = i0 + threadIdx.x; i < m; i += 256) mx = fmaxf(mx, fabsf(col[i]));
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) sc[blockIdx.x] = red[0] > 0.f ? red[0] / F::QMAX : 1.f;
}

// Aq (column-major, ld ldq) and Aq_t (A^T column-major, ld ldqt) of a 64 x 64
// tile of A.  Thread (tx, ty) loads rows 4 tx .. 4 tx + 3 of columns
// ty + 16 r with 16-byte loads, writes them packed into Aq, and through an
// LDS transpose writes 16 consecutive entries of one row of A into Aq_t.
template <typename F>
__global__ __launch_bounds__(256) void quantize_tile_kernel(int64_t m, int64_t n,
                                                            const float* __restrict__ A, int64_t lda,
                                                            const float* __restrict__ sc,
                                                            typename F::store_t* __restrict__ Aq,
                                                            int64_t ldq,
                                                            typename F::store_t* __restrict__ Aqt,
                                                            int64_t ldqt) {
  using S = typename F::store_t;
  __shared__ __align__(16) S tile[64][64 + 16 / sizeof(S)];
  const int64_t i0 = (int64_t)blockIdx.x * 64, j0 = (int64_t)blockIdx.y * 64;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const bool full = (i0 + 64 <= m) && (j0 + 64 <= n) && ((uintptr_t)A % 16 == 0) && (lda % 4 == 0);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int jj = ty + 16 * r;
    const int64_t j = j0 + jj, i = i0 + 4 * tx;
    float v[4] = {0.f, 0.f, 0.f, 0.f};
    if (full) {
      const float4 x = *reinterpret_cast<const float4*>(A + i + j * lda);
      const float s = sc[j];
      v[0] = x.x / s; v[1] = x.y / s; v[2] = x.z / s; v[3] = x.w / s;
    } else if (j < n) {
      const float s = sc[j];
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (i + e < m) v[e] = A[i + e + j * lda] / s;
    }
    S q[4];
    enc4<F>(v, q);
    if (!full) {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (!(i + e < m && j < n)) q[e] = (S)0;  // padding rows and columns are zero
    }
    if (i < ldq && j < n) {
      if constexpr (sizeof(S) == 1) {
        const uint32_t w = (uint32_t)q[0] | ((uint32_t)q[1] << 8) | ((uint32_t)q[2] << 16) | ((uint32_t)q[3] << 24);
        *reinterpret_cast<uint32_t*>(Aq + i + j * ldq) = w;
      } else {
        const uint2 w = make_uint2((uint32_t)q[0] | ((uint32_t)q[1] << 16), (uint32_t)q[2] | ((uint32_t)q[3] << 16));
        *reinterpret_cast<uint2*>(Aq + i + j * ldq) = w;
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) tile[4 * tx + e][jj] = q[e];
  }
  __syncthreads();
  // row ii of the tile: 16 consecutive columns per thread
  const int ii = threadIdx.x >> 2, jg = threadIdx.x & 3;
  const int64_t i = i0 + ii, j = j0 + 16 * jg;
  if (i < m && j < ldqt) {
    S* dst = Aqt + j + i * ldqt;
    const S* srcl = &tile[ii][16 * jg];
    if constexpr (sizeof(S) == 1) {
      uint32_t w[4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        w[q] = (uint32_t)srcl[4 * q] | ((uint32_t)srcl[4 * q + 1] << 8) | ((uint32_t)srcl[4 * q + 2] << 16) |
               ((uint32_t)srcl[4 * q + 3] << 24);
      *reinterpret_cast<uint4*>(dst) = make_uint4(w[0], w[1], w[2], w[3]);
    } else {
      uint32_t w[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) w[q] = (uint32_t)srcl[2 * q] | ((uint32_t)srcl[2 * q + 1] << 16);
      *reinterpret_cast<uint4*>(dst) = make_uint4(w[0], w[1], w[2], w[3]);
      *reinterpret_cast<uint4*>(dst + 8) = make_uint4(w[4], w[5], w[6], w[7]);
    }
  }
}

// Xq[:, c] = q(rs .* X[:, c] / u_c), u_c = max_k |rs_k X_kc| / QMAX; one workgroup per column
template <typename F>
__global__ __launch_bounds__(256) void quantize_cols_kernel(int64_t rows, const float* __restrict__ X,
                                                            int64_t ldx, const float* __restrict__ rs,
                                                            typename F::store_t* __restrict__ Xq,
                                                            float* __restrict__ u) {
  __shared__ float red[256];
  const float* col = X + (int64_t)blockIdx.x * ldx;
  float mx = 0.f;
  for (int64_t i = threadIdx.x; i < rows; i += 256) mx = fmaxf(mx, fabsf(col[i] * (rs ? rs[i] : 1.f)));
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + st]);
    __syncthreads();
  }
  const float uc = red[0] > 0.f ? red[0] / F::QMAX : 1.f;
  if (threadIdx.x == 0) u[blockIdx.x] = uc;
  const int64_t ldq = (rows + 15) / 16 * 16;
  typename F::store_t* out = Xq + (int64_t)blockIdx.x * ldq;
  for (int64_t i = threadIdx.x; i < ldq; i += 256)
    out[i] = i < rows ? F::enc(col[i] * (rs ? rs[i] : 1.f) / uc) : (typename F::store_t)0;
}

// ---- C = X^T Y with quantized, K-contiguous operands ----------------------------------
//
// X: K x M, Y: K x N (column-major, ld = K).  Workgroup tile 64 x 128, 4 waves
// (2 x 2), wave tile 32 x 64 = 2 x 4 MFMA tiles.  Stages of BK = 64 K through
// LDS, each operand row of the tile stored K-contiguous with an 8-byte pad.
template <typename F>
__global__ __launch_bounds__(256) void qgemm_tn_kernel(int M, int N, int64_t K,
                                                       const typename F::store_t* __restrict__ X,
                                                       const typename F::store_t* __restrict__ Y,
                                                       float* __restrict__ P, int64_t kchunk) {
  using S = typename F::store_t;
  constexpr int BM = 64, BN = 128, BK = 64;
  constexpr int KPL = F::KPL;                 // elements per lane per MFMA
  constexpr int KM = 4 * KPL;                 // K per MFMA
  constexpr int RB = BK * (int)sizeof(S);     // bytes per staged row
  constexpr int RP = RB + 8;                  // padded
  __shared__ __align__(16) unsigned char xs[BM * RP];
  __shared__ __align__(16) unsigned char ys[BN * RP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  const int64_t k0 = (int64_t)blockIdx.z * kchunk;
  int64_t k1 = k0 + kchunk;
  if (k1 > K) k1 = K;
  floatx4 acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = floatx4{0, 0, 0, 0};
  const int g = lane >> 4, c16 = lane & 15;
  constexpr int V16 = 16 / (int)sizeof(S);  // elements per 16-byte load
  constexpr int CPR = BK / V16;             // 16-byte chunks per staged row
  for (int64_t kb = k0; kb < k1; kb += BK) {
    const bool full = kb + BK <= k1;
    // stage X rows (m0 .. m0+BM) and Y rows (n0 .. n0+BN), K kb .. kb+BK
    for (int e = tid; e < (BM + BN) * CPR; e += 256) {
      const int row = e / CPR, ch = e % CPR;
      const bool isx = row < BM;
      const int r = isx ? row : row - BM;
      const int64_t gr = (isx ? m0 : n0) + r;
      const S* src = isx ? X : Y;
      const int lim = isx ? M : N;
      unsigned char* dst = (isx ? xs : ys) + r * RP + ch * 16;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (gr < lim) {
        const S* p = src + gr * K + kb + ch * V16;
        if (full) {
          v = *reinterpret_cast<const uint4*>(p);
        } else {
          S tmp[V16];
#pragma unroll
          for (int q = 0; q < V16; ++q) tmp[q] = (kb + ch * V16 + q < k1) ? p[q] : (S)0;
          __builtin_memcpy(&v, tmp, 16);
        }
      }
      *reinterpret_cast<uint2*>(dst) = make_uint2(v.x, v.y);
      *reinterpret_cast<uint2*>(dst + 8) = make_uint2(v.z, v.w);
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < BK; ks += KM) {
      uint64_t av[2], bv[4];
#pragma unroll
      for (int a = 0; a < 2; ++a)
        av[a] = *reinterpret_cast<const uint64_t*>(xs + (wm * 32 + a * 16 + c16) * RP +
                                                   (ks + g * KPL) * (int)sizeof(S));
#pragma unroll
      for (int b = 0; b < 4; ++b)
        bv[b] = *reinterpret_cast<const uint64_t*>(ys + (wn * 64 + b * 16 + c16) * RP +
                                                   (ks + g * KPL) * (int)sizeof(S));
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = qmfma<F>(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
  float* dst = P + (int64_t)blockIdx.z * M * N;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int j = n0 + wn * 64 + b * 16 + c16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = m0 + wm * 32 + a * 16 + 4 * g + v;
        if (i < M && j < N) dst[i + (int64_t)j * M] = acc[a][b][v];
      }
    }
}

__global__ void qgemm_reduce_kernel(int M, int N, const float* __restrict__ P, int splits,
                                    const float* __restrict__ rs, const float* __restrict__ cs,
                                    float* __restrict__ C, int64_t ldc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i >= M) return;
  double acc = 0.0;
  for (int z = 0; z < splits; ++z) acc += (double)P[(int64_t)z * M * N + i + j * M];
  acc *= (double)cs[j] * (rs ? (double)rs[i] : 1.0);
  C[i + j * ldc] = (float)acc;
}

namespace {

struct QShape {
  int splits;
  int64_t kchunk;
};

QShape qshape(const rmm_ctx* h, int M, int N, int64_t K) {
  const int64_t tiles = (int64_t)((M + 63) / 64) * ((N + 127) / 128);
  int64_t want = (4ll * h->cus + tiles - 1) / tiles;
  const int64_t maxsplit = (K + 2047) / 2048;
  if (want > maxsplit) want = maxsplit;
  if (want < 1) want = 1;
  int64_t kc = (K + want - 1) / want;
  kc = (kc + 63) / 64 * 64;
  QShape q;
  q.kchunk = kc;
  q.splits = (int)((K + kc - 1) / kc);
  if (q.splits < 1) q.splits = 1;
  return q;
}

}  // namespace

size_t qgemm_workspace(const rmm_ctx* h, int M, int N, int64_t K) {
  const QShape q = qshape(h, M, N, K);
  Carver c(nullptr, 0);
  c.take<float>((size_t)q.splits * M * N);
  return c.off;
}

template <typename F>
int qgemm_tn(rmm_ctx* h, int M, int N, int64_t K, const void* X, const void* Y, const float* rs,
             const float* cs, float* C, int64_t ldc, Carver& ws) {
  if (M == 0 || N == 0) return RMM_OK;
  if (K % (16 / sizeof(typename F::store_t)) != 0) return RMM_ERR_UNSUPPORTED;
  const QShape q = qshape(h, M, N, K);
  const size_t mark = ws.off;
  float* P = ws.take<float>((size_t)q.splits * M * N);
  if (!ws.fits()) return RMM_ERR_WORKSPACE_TOO_SMALL;
  dim3 grid((unsigned)((M + 63) / 64), (unsigned)((N + 127) / 128), (unsigned)q.splits);
  hipLaunchKernelGGL(qgemm_tn_kernel<F>, grid, dim3(256), 0, h->stream, M, N, K,
                     (const typename F::store_t*)X, (const typename F::store_t*)Y, P, q.kchunk);
  RMM_TRY(launch_status());
  dim3 g2((unsigned)((M + 255) / 256), (unsigned)N);
  hipLaunchKernelGGL(qgemm_reduce_kernel, g2, dim3(256), 0, h->stream, M, N, P, q.splits, rs, cs, C,
                     ldc);
  ws.off = mark;
  return launch_status();
}

template <typename F>
int quantize_matrix(const rmm_ctx* h, int64_t m, int64_t n, const float* A, int64_t lda, float* sc,
                    void* Aq, void* Aqt) {
  hipLaunchKernelGGL(colscale_kernel<F>, dim3((unsigned)n), dim3(256), 0, h->stream, m, A, lda, sc);
  RMM_TRY(launch_status());
  const int64_t ldq = mp_pad(m), ldqt = mp_pad(n);
  const int64_t gm = ldq > m ? ldq : m, gn = ldqt > n ? ldqt : n;
  dim3 grid((unsigned)((gm + 63) / 64), (unsigned)((gn + 63) / 64));
  hipLaunchKernelGGL(quantize_tile_kernel<F>, grid, dim3(256), 0, h->stream, m, n, A, lda, sc,
                     (typename F::store_t*)Aq, ldq, (typename F::store_t*)Aqt, ldqt);
  return launch_status();
}

template <typename F>
int quantize_cols(const rmm_ctx* h, int64_t rows, int64_t cols, const float* X, int64_t ldx,
                  const float* rs, void* Xq, float* u) {
  hipLaunchKernelGGL(quantize_cols_kernel<F>, dim3((unsigned)cols), dim3(256), 0, h->stream, rows, X,
                     ldx, rs, (typename F::store_t*)Xq, u);
  return launch_status();
}

// dispatch on the precision enum
int mp_quantize_matrix(const rmm_ctx* h, rmm_precision p, int64_t m, int64_t n, const float* A,
                       int64_t lda, float* sc, void* Aq, void* Aqt) {
  return p == RMM_PREC_BF16 ? quantize_matrix<Bf16Fmt>(h, m, n, A, lda, sc, Aq, Aqt)
                            : quantize_matrix<Fp8Fmt>(h, m, n, A, lda, sc, Aq, Aqt);
}
int mp_quantize_cols(const rmm_ctx* h, rmm_precision p, int64_t rows, int64_t cols, const float* X,
                     int64_t ldx, const float* rs, void* Xq, float* u) {
  return p == RMM_PREC_BF16 ? quantize_cols<Bf16Fmt>(h, rows, cols, X, ldx, rs, Xq, u)
                            : quantize_cols<Fp8Fmt>(h, rows, cols, X, ldx, rs, Xq, u);
}
int mp_gemm_tn(rmm_ctx* h, rmm_precision p, int M, int N, int64_t K, const void* X, const void* Y,
               const float* rs, const float* cs, float* C, int64_t ldc, Carver& ws) {
  return p == RMM_PREC_BF16 ? qgemm_tn<Bf16Fmt>(h, M, N, K, X, Y, rs, cs, C, ldc, ws)
                            : qgemm_tn<Fp8Fmt>(h, M, N, K, X, Y, rs, cs, C, ldc, ws);
}
size_t mp_elem_bytes(rmm_precision p) { return p == RMM_PREC_BF16 ? 2 : 1; }

// ---- test hook: one quantized product ----------------------------------------------------

size_t mp_product_workspace(const rmm_ctx* h, rmm_precision p, int64_t m, int64_t n, int l) {
  const size_t eb = mp_elem_bytes(p);
  const int64_t pm = mp_pad(m), pn = mp_pad(n);
  Carver c(nullptr, 0);
  c.take<float>((size_t)n);
  c.take<unsigned char>((size_t)pm * n * eb);
  c.take<unsigned char>((size_t)pn * m * eb);
  c.take<unsigned char>((size_t)(pm > pn ? pm : pn) * l * eb);
  c.take<float>((size_t)l);
  const size_t a = qgemm_workspace(h, (int)m, l, pn), b = qgemm_workspace(h, (int)n, l, pm);
  return c.off + (a > b ? a : b) + 4 * kAlign;
}

// mode 0: out (m x l) = A X, X n x l;  mode 1: out (n x l) = A^T X, X m x l
int mp_product(rmm_ctx* h, rmm_precision p, int mode, int64_t m, int64_t n, const float* A,
               int64_t lda, const float* X, int64_t ldx, int l, float* out, int64_t ldo) {
  const size_t eb = mp_elem_bytes(p);
  const int64_t pm = mp_pad(m), pn = mp_pad(n);
  Carver ws(h->ws, h->ws_bytes);
  float* sc = ws.take<float>((size_t)n);
  unsigned char* Aq = ws.take<unsigned char>((size_t)pm * n * eb);
  unsigned char* Aqt = ws.take<unsigned char>((size_t)pn * m * eb);
  unsigned char* Xq = ws.take<unsigned char>((size_t)(pm > pn ? pm : pn) * l * eb);
  float* u = ws.take<float>((size_t)l);
  if (!ws.fits()) return RMM_ERR_WORKSPACE_TOO_SMALL;
  RMM_TRY(mp_quantize_matrix(h, p, m, n, A, lda, sc, Aq, Aqt));
  if (mode == 0) {
    RMM_TRY(mp_quantize_cols(h, p, n, l, X, ldx, sc, Xq, u));
    return mp_gemm_tn(h, p, (int)m, l, pn, Aqt, Xq, nullptr, u, out, ldo, ws);
  }
  RMM_TRY(mp_quantize_cols(h, p, m, l, X, ldx, nullptr, Xq, u));
  return mp_gemm_tn(h, p, (int)n, l, pm, Aq, Xq, sc, u, out, ldo, ws);
}

}  // namespace rmm

using namespace rmm;

extern "C" {

int rmm_mixed_product_workspace(rmm_handle h, rmm_precision prec, int64_t m, int64_t n, int64_t l,
                                size_t* bytes) {
  if (!h || !bytes || (prec != RMM_PREC_BF16 && prec != RMM_PREC_FP8) || m < 1 || n < 1 || l < 1 ||
      l > 4096 || m >= (1ll << 31) || n >= (1ll << 31))
    return RMM_ERR_INVALID_ARG;
  *bytes = mp_product_workspace(h, prec, m, n, (int)l);
  return RMM_OK;
}

int rmm_mixed_product(rmm_handle h, rmm_precision prec, int mode, int64_t m, int64_t n,
                      const float* A, int64_t lda, const float* X, int64_t ldx, int64_t l,
                      float* out, int64_t ldo) {
  if (!h || (prec != RMM_PREC_BF16 && prec != RMM_PREC_FP8) || (mode != 0 && mode != 1) || m < 1 ||
      n < 1 || l < 1 || l > 4096 || !A || !X || !out || lda < m || ldx < (mode == 0 ? n : m) ||
      ldo < (mode == 0 ? m : n) || m >= (1ll << 31) || n >= (1ll << 31))
    return RMM_ERR_INVALID_ARG;
  return mp_product(h, prec, mode, m, n, A, lda, X, ldx, (int)l, out, ldo);
}

}  // extern "C"
