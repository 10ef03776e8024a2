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
  static __device__ __forceinline__ uint8_t enc(float x) {
    return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(x, 0.0f, 0, false) & 0xFF);
  }
};

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// One MFMA of each format: 16 x 16 outputs; each lane holds K-consecutive
// elements of one row of each operand, 16 bytes of BF16 (gfx950's 16x16x32
// BF16 MFMA, K = 32) or 32 bytes of FP8 (gfx950's 16x16x128 f8f6f4 MFMA with
// unit block scales, K = 128).  Both operands use the same lane-to-K
// assignment, so the sum over K does not depend on the order in which the
// instruction pairs them.
template <typename F>
struct QOp;
template <>
struct QOp<Bf16Fmt> {
  using op_t = uint4;
  static __device__ __forceinline__ floatx4 mfma(uint4 a, uint4 b, floatx4 c) {
    bf16x8 x, y;
    __builtin_memcpy(&x, &a, 16);
    __builtin_memcpy(&y, &b, 16);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, c, 0, 0, 0);
  }
};
struct alignas(16) U8x32 {
  uint4 lo, hi;
};
typedef int intx8 __attribute__((ext_vector_type(8)));
template <>
struct QOp<Fp8Fmt> {
  using op_t = U8x32;
  static __device__ __forceinline__ floatx4 mfma(const U8x32& a, const U8x32& b, floatx4 c) {
    intx8 x, y;
    __builtin_memcpy(&x, &a, 32);
    __builtin_memcpy(&y, &b, 32);
    // formats e4m3 / e4m3, block scales 2^(127 - 127) = 1
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(x, y, c, 0, 0, 0, 127, 0, 127);
  }
};

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
      const float4 x = ld_stream(reinterpret_cast<const float4*>(col + i));
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
      const float4 x = ld_stream(reinterpret_cast<const float4*>(A + i + j * lda));
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

// Xq[:, c] = q(rs .* X[:, c] / u_c), u_c = max_k |rs_k X_kc| / QMAX (1 for a
// zero column), in three launches spread over the whole device: clear the
// column maxima, take them with atomicMax on the bit patterns (non-negative
// floats order as their bits), then quantize element-parallel.
constexpr int kQcRows = 4096;  // rows per workgroup of the max pass

__global__ void colmax_clear_kernel(int cols, unsigned* __restrict__ umax) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < cols) umax[c] = 0u;
}

__global__ __launch_bounds__(256) void colmax_kernel(int64_t rows, const float* __restrict__ X, int64_t ldx,
                                                     const float* __restrict__ rs,
                                                     unsigned* __restrict__ umax) {
  __shared__ float red[256];
  const float* col = X + (int64_t)blockIdx.x * ldx;
  const int64_t r0 = (int64_t)blockIdx.y * kQcRows;
  const int64_t r1 = (r0 + kQcRows < rows) ? r0 + kQcRows : rows;
  float mx = 0.f;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += 256) mx = fmaxf(mx, fabsf(col[i] * (rs ? rs[i] : 1.f)));
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0 && red[0] > 0.f) atomicMax(&umax[blockIdx.x], __float_as_uint(red[0]));
}

template <typename F>
__global__ __launch_bounds__(256) void quantize_cols_kernel(int64_t rows, const float* __restrict__ X,
                                                            int64_t ldx, const float* __restrict__ rs,
                                                            const unsigned* __restrict__ umax,
                                                            typename F::store_t* __restrict__ Xq,
                                                            float* __restrict__ u) {
  const int64_t c = blockIdx.y;
  const float m = __uint_as_float(umax[c]);
  const float uc = m > 0.f ? m / F::QMAX : 1.f;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i == 0) u[c] = uc;
  const int64_t ldq = (rows + 15) / 16 * 16;
  if (i >= ldq) return;
  const float* col = X + c * ldx;
  Xq[c * ldq + i] = i < rows ? F::enc(col[i] * (rs ? rs[i] : 1.f) / uc) : (typename F::store_t)0;
}

// ---- C = X^T Y with quantized, K-contiguous operands ----------------------------------
//
// X: K x M, Y: K x N (column-major, ld = K).  Workgroup tile 256 x 128 (so
// the small operand Y is re-read once per 256 rows of A), 8 waves of 64 x 64
// (4 x 4 MFMA tiles).  Stages of 128 bytes of K per operand row go through
// two LDS buffers (rows padded to 144 bytes: the 16-byte operand reads of a
// quarter wave hit distinct banks); the 16-byte global loads of the next two
// stages sit in registers while the current stage is multiplied, and each
// stage needs one barrier (a buffer is rewritten two stages after its last
// reads, behind the barrier of the stage in between).  Split-K over blockIdx.z, partials reduced in FP64 by
// qgemm_reduce_kernel.
constexpr int kQBM = 256, kQBN = 128;
constexpr int kQRow = 128;  // bytes of K per staged row
constexpr int kQPad = 144;  // padded row pitch in LDS
constexpr int kQThreads = 512;
constexpr size_t kQLds = 2 * (size_t)(kQBM + kQBN) * kQPad;

template <typename F>
__global__ __launch_bounds__(kQThreads) void qgemm_tn_kernel(int M, int N, int64_t K,
                                                             const typename F::store_t* __restrict__ X,
                                                             const typename F::store_t* __restrict__ Y,
                                                             float* __restrict__ P, int64_t kchunk) {
  using S = typename F::store_t;
  using op_t = typename QOp<F>::op_t;
  constexpr int ES = (int)sizeof(S);
  constexpr int BK = kQRow / ES;                        // K elements per stage
  constexpr int V16 = 16 / ES;                          // elements per 16-byte chunk
  constexpr int CPR = kQRow / 16;                       // chunks per staged row
  constexpr int ROWS = kQBM + kQBN;
  constexpr int CH = ROWS * CPR / kQThreads;            // chunks per thread
  constexpr int KPL = (int)sizeof(op_t) / ES;           // elements per lane per MFMA
  constexpr int KM = 4 * KPL;                           // K per MFMA
  static_assert(ROWS * CPR % kQThreads == 0, "chunks per thread");
  extern __shared__ __align__(16) unsigned char qlds[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int g = lane >> 4, c16 = lane & 15;
  const int m0 = blockIdx.x * kQBM, n0 = blockIdx.y * kQBN;
  const int64_t k0 = (int64_t)blockIdx.z * kchunk;
  const int64_t k1 = (k0 + kchunk < K) ? k0 + kchunk : K;
  floatx4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = floatx4{0, 0, 0, 0};
  // chunk e = tid + q * kQThreads: staged row e / CPR (X rows first), chunk e % CPR
  const S* src[CH];
  int lds_off[CH];
  bool live[CH];
#pragma unroll
  for (int q = 0; q < CH; ++q) {
    const int e = tid + q * kQThreads;
    const int row = e / CPR, ch = e % CPR;
    const bool isx = row < kQBM;
    const int r = isx ? row : row - kQBM;
    const int64_t gr = (int64_t)(isx ? m0 : n0) + r;
    live[q] = gr < (isx ? M : N);
    src[q] = (isx ? X : Y) + (live[q] ? gr : 0) * K + ch * V16;
    lds_off[q] = row * kQPad + ch * 16;
  }
  // two stages of loads in flight: stage t + 2 is issued while stage t is
  // multiplied (the loop is unrolled by two so that both register sets keep
  // constant indices)
  uint4 pa[CH], pb[CH];
  auto load = [&](uint4 (&pre)[CH], int64_t kb) {
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int64_t ko = kb + (int64_t)((tid + q * kQThreads) % CPR) * V16;
      // chunks that hold rows of the streamed operand X (read once) take the
      // nontemporal hint; the small operand Y is re-read by every workgroup
      const bool xq = (q + 1) * kQThreads <= kQBM * CPR;
      const uint4* p = reinterpret_cast<const uint4*>(src[q] + kb);
      pre[q] = (live[q] && ko < k1) ? (xq ? ld_stream(p) : *p) : make_uint4(0, 0, 0, 0);
    }
  };
  auto stage = [&](uint4 (&pre)[CH], int64_t kb, int parity) {
    unsigned char* buf = qlds + (size_t)parity * ROWS * kQPad;
#pragma unroll
    for (int q = 0; q < CH; ++q) *reinterpret_cast<uint4*>(buf + lds_off[q]) = pre[q];
    __syncthreads();
    if (kb + 2 * BK < k1) load(pre, kb + 2 * BK);
    const unsigned char* xb = buf;
    const unsigned char* yb = buf + kQBM * kQPad;
#pragma unroll
    for (int ks = 0; ks < BK; ks += KM) {
      op_t av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
        av[a] = *reinterpret_cast<const op_t*>(xb + (wm * 64 + a * 16 + c16) * kQPad + (ks + g * KPL) * ES);
#pragma unroll
      for (int b = 0; b < 4; ++b)
        bv[b] = *reinterpret_cast<const op_t*>(yb + (wn * 64 + b * 16 + c16) * kQPad + (ks + g * KPL) * ES);
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = QOp<F>::mfma(av[a], bv[b], acc[a][b]);
    }
  };
  load(pa, k0);
  if (k0 + BK < k1) load(pb, k0 + BK);
  for (int64_t kb = k0; kb < k1; kb += 2 * BK) {
    stage(pa, kb, 0);
    if (kb + BK < k1) stage(pb, kb + BK, 1);
  }
  float* dst = P + (int64_t)blockIdx.z * M * N;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int j = n0 + wn * 64 + b * 16 + c16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = m0 + wm * 64 + a * 16 + 4 * g + v;
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

// one workgroup per CU (each holds 108 KB of LDS): split K until the tiles
// times the splits reach the CU count, with at least 2048 K per split
QShape qshape(const rmm_ctx* h, int M, int N, int64_t K) {
  const int64_t tiles = (int64_t)((M + kQBM - 1) / kQBM) * ((N + kQBN - 1) / kQBN);
  int64_t want = ((int64_t)h->cus + tiles - 1) / tiles;
  const int64_t maxsplit = (K + 2047) / 2048;
  if (want > maxsplit) want = maxsplit;
  if (want < 1) want = 1;
  int64_t kc = (K + want - 1) / want;
  kc = (kc + 127) / 128 * 128;  // whole stages of both formats
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
  dim3 grid((unsigned)((M + kQBM - 1) / kQBM), (unsigned)((N + kQBN - 1) / kQBN), (unsigned)q.splits);
  RMM_HIP(hipFuncSetAttribute((const void*)qgemm_tn_kernel<F>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kQLds));
  hipLaunchKernelGGL(qgemm_tn_kernel<F>, grid, dim3(kQThreads), kQLds, h->stream, M, N, K,
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
                  const float* rs, void* Xq, float* u, unsigned* umax) {
  if (cols == 0) return RMM_OK;
  hipLaunchKernelGGL(colmax_clear_kernel, dim3((unsigned)((cols + 255) / 256)), dim3(256), 0, h->stream,
                     (int)cols, umax);
  hipLaunchKernelGGL(colmax_kernel, dim3((unsigned)cols, (unsigned)((rows + kQcRows - 1) / kQcRows)),
                     dim3(256), 0, h->stream, rows, X, ldx, rs, umax);
  const int64_t ldq = (rows + 15) / 16 * 16;
  hipLaunchKernelGGL(quantize_cols_kernel<F>, dim3((unsigned)((ldq + 255) / 256), (unsigned)cols),
                     dim3(256), 0, h->stream, rows, X, ldx, rs, (const unsigned*)umax,
                     (typename F::store_t*)Xq, u);
  return launch_status();
}

// dispatch on the precision enum
int mp_quantize_matrix(const rmm_ctx* h, rmm_precision p, int64_t m, int64_t n, const float* A,
                       int64_t lda, float* sc, void* Aq, void* Aqt) {
  return p == RMM_PREC_BF16 ? quantize_matrix<Bf16Fmt>(h, m, n, A, lda, sc, Aq, Aqt)
                            : quantize_matrix<Fp8Fmt>(h, m, n, A, lda, sc, Aq, Aqt);
}
int mp_quantize_cols(const rmm_ctx* h, rmm_precision p, int64_t rows, int64_t cols, const float* X,
                     int64_t ldx, const float* rs, void* Xq, float* u, unsigned* umax) {
  return p == RMM_PREC_BF16 ? quantize_cols<Bf16Fmt>(h, rows, cols, X, ldx, rs, Xq, u, umax)
                            : quantize_cols<Fp8Fmt>(h, rows, cols, X, ldx, rs, Xq, u, umax);
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
  c.take<unsigned>((size_t)l);
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
  unsigned* umax = ws.take<unsigned>((size_t)l);
  if (!ws.fits()) return RMM_ERR_WORKSPACE_TOO_SMALL;
  RMM_TRY(mp_quantize_matrix(h, p, m, n, A, lda, sc, Aq, Aqt));
  if (mode == 0) {
    RMM_TRY(mp_quantize_cols(h, p, n, l, X, ldx, sc, Xq, u, umax));
    return mp_gemm_tn(h, p, (int)m, l, pn, Aqt, Xq, nullptr, u, out, ldo, ws);
  }
  RMM_TRY(mp_quantize_cols(h, p, m, l, X, ldx, nullptr, Xq, u, umax));
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
