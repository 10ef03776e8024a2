// SRHT sketch C = s^{-1/2} (H_N D [A; 0])[idx, :]  (Sec. 3.2.2).
//
// Random signs D on the m real rows, zero padding to N = 2^ceil(log2 m),
// the Sylvester-ordered Walsh-Hadamard transform along the rows, and the s
// sampled rows idx (sorted, drawn without replacement), scaled by 1/sqrt(s).
//
// Only s of the N transformed rows are needed, so the transform is split
// with the Kronecker structure of the Sylvester recursion: with L = 4096 and
// row index i = i_hi L + i_lo,
//     H_N[r, i] = H_{N/L}[r_hi, i_hi] * H_L[r_lo, i_lo],
//     (H_N x)[r] = sum_{i_hi} (-1)^popcount(r_hi & i_hi) (H_L x_{i_hi})[r_lo].
// A workgroup of WV waves (8 for fp32, 4 for fp64) takes WV consecutive
// L-row chunks of one column: each wave loads its chunk (16-byte loads, 4
// rows per lane), applies D (sign bits from a table generated once per call,
// since they depend on the row only), runs the 12-stage butterfly network in
// registers with one LDS transpose and leaves z = H_L x_chunk in its LDS
// buffer; the workgroup then adds the WV chunks' signed contributions to the
// s sampled rows, whose accumulators are spread over its threads.  N < L is
// handled by zero padding to L: (H_L [x; 0])[r] equals (H_N x)[r] for r < N.
// Per-workgroup partial sums are reduced in a fixed order.
#include "common.hpp"
#include "rng.hpp"

namespace rmm {

namespace {

constexpr int kLogL = 12;
constexpr int kL = 1 << kLogL;  // 4096 rows per chunk, 64 values per lane

// LDS word address of row r inside a wave's chunk buffer.  XOR-ing row bits
// 8..10 into bits 2..4 makes both the 16-byte stores of the load layout and
// the strided 4-byte loads of the transposed layout bank-conflict free.
__device__ __forceinline__ uint32_t swz(uint32_t r) { return r ^ (((r >> 8) & 7u) << 2); }

template <typename T>
__device__ __forceinline__ T flip(T x, uint32_t w);
// toggles the IEEE sign bit of x when bit 0 of w is set (higher bits of w
// are shifted out)
template <>
__device__ __forceinline__ float flip<float>(float x, uint32_t w) {
  return __uint_as_float(__float_as_uint(x) + (w << 31));
}
template <>
__device__ __forceinline__ double flip<double>(double x, uint32_t w) {
  const uint64_t u = (uint64_t)__double_as_longlong(x) + ((uint64_t)w << 63);
  return __longlong_as_double((long long)u);
}

template <typename T>
__device__ __forceinline__ void bfly(T& a, T& b) {
  const T x = a + b;
  const T y = a - b;
  a = x;
  b = y;
}

// LDS word address of row r of a chunk in the combine layout: after the
// second butterfly phase lane (a | b' << 2) holds rows a + 4 i + 256 b' in
// x[i]; x[4 j .. 4 j + 3] go to one 16-byte store at word
// 4 (lane + 64 j), so the wave's stores cover 1 KiB contiguously.
__device__ __forceinline__ uint32_t zaddr(uint32_t r) {
  const uint32_t a = r & 3u, i = (r >> 2) & 63u, bp = r >> 8;
  return (i & 3u) + 4u * ((a | (bp << 2)) + 64u * (i >> 2));
}

template <typename T>
__device__ __forceinline__ T xor_sign(T x, uint32_t mask);
template <>
__device__ __forceinline__ float xor_sign<float>(float x, uint32_t mask) {
  return __uint_as_float(__float_as_uint(x) ^ mask);
}
template <>
__device__ __forceinline__ double xor_sign<double>(double x, uint32_t mask) {
  return __longlong_as_double(__double_as_longlong(x) ^ ((long long)mask << 32));
}

// One workgroup = WV waves working on WV consecutive chunks ("a group") of
// the same column; unit = (column, group).  Wave w transforms chunk WV g + w
// into its own LDS buffer; then the threads add, for the samples they own
// (t = tid + 64 WV k), the group's contribution
//   sum_w (-1)^popcount(r_hi & (WV g + w)) z_w[r_lo]
//   = (-1)^popcount((r_hi >> LW) & g) * sum_w (-1)^popcount((r_hi mod WV) & w) z_w[r_lo],
// the inner sum a WV-point Walsh-Hadamard combination whose sign bits are
// fixed per sample.
template <typename T, int WV, int SPQ, bool VEC>
__device__ __forceinline__ void srht_body(const T* __restrict__ A, int64_t lda,
                                          const T* __restrict__ bcol, int n, PanelPlan plan,
                                          const uint32_t* __restrict__ idx,
                                          const uint32_t* __restrict__ signs,
                                          T* __restrict__ partials) {
  constexpr int LW = WV == 8 ? 3 : 2;
  constexpr int NT = 64 * WV;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  T* buf = reinterpret_cast<T*>(smem) + (size_t)wave * kL;  // this wave's chunk
  uint32_t* sgn = reinterpret_cast<uint32_t*>(smem + WV * kL * sizeof(T)) + wave * 128;
  const int64_t blk = blockIdx.x;
  const int64_t u0 = plan_start(plan, blk);
  const int64_t u1 = plan_start(plan, blk + 1);
  const int s = plan.s;
  const int64_t ngroups = plan.nchunks;  // plan chunk = WV L rows

  // owned samples: word address of z[r_lo] in the combine layout times 4
  // (bits 0..13), r_hi mod WV (bits 14 ..), r_hi >> LW (bits 14 + LW ..)
  uint32_t pk[SPQ];
  T acc[SPQ];
#pragma unroll
  for (int k = 0; k < SPQ; ++k) {
    const int t = tid + NT * k;
    const uint32_t r = t < s ? idx[t] : 0u;
    const uint32_t hi = r >> kLogL;
    pk[k] = ((hi >> LW) << (14 + LW)) | ((hi & (WV - 1u)) << 14) | (zaddr(r & (kL - 1)) * 4u);
    acc[k] = T(0);
  }
  // lane-constant parts of the swizzled transpose addresses (swz only touches bits 2..4)
  const uint32_t a = lane & 3u, bq = (uint32_t)lane >> 2;
  uint32_t woff[8], roff[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    woff[i] = 4u * ((uint32_t)lane ^ (uint32_t)i);
    roff[i] = a + 256u * bq + 4u * ((uint32_t)i ^ (bq & 7u));
  }

  T xa[64];
  auto load_chunk = [&](int64_t u, T (&x)[64]) {
    const int64_t j = u / ngroups;
    const int64_t c = (u - j * ngroups) * WV + wave;
    const int64_t r0 = c * kL;
    const T* col = (j < n) ? A + j * lda : bcol;
    if (VEC && r0 + kL <= plan.m) {
      const T* p = col + r0 + 4 * lane;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        if constexpr (sizeof(T) == 4) {
          const float4 q = ld_stream(reinterpret_cast<const float4*>(p + 256 * k));
          x[4 * k] = q.x; x[4 * k + 1] = q.y; x[4 * k + 2] = q.z; x[4 * k + 3] = q.w;
        } else {
          const double2 q0 = ld_stream(reinterpret_cast<const double2*>(p + 256 * k));
          const double2 q1 = ld_stream(reinterpret_cast<const double2*>(p + 256 * k + 2));
          x[4 * k] = q0.x; x[4 * k + 1] = q0.y; x[4 * k + 2] = q1.x; x[4 * k + 3] = q1.y;
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < 16; ++k)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t row = r0 + 256 * k + 4 * lane + e;
          x[4 * k + e] = (row < plan.m) ? col[row] : T(0);
        }
    }
  };

  // the 128 sign words of unit u's chunk, loaded along with its rows
  auto load_signs = [&](int64_t u) {
    const int64_t j = u / ngroups;
    const int64_t r0 = ((u - j * ngroups) * WV + wave) * kL;
    return lane < 32 ? reinterpret_cast<const uint4*>(signs + (r0 >> 5))[lane] : make_uint4(0u, 0u, 0u, 0u);
  };
  int64_t cur = -1;
  T (&x)[64] = xa;
  uint4 sw = make_uint4(0u, 0u, 0u, 0u);
  if (u0 < u1) {
    sw = load_signs(u0);
    load_chunk(u0, x);
  }
  for (int64_t u = u0; u < u1; ++u) {
    const int64_t j = u / ngroups;
    const int64_t g = u - j * ngroups;
    if (j != cur) {
      if (cur >= 0) {
        T* dst = partials + (blk + cur) * plan.slot_elems;
#pragma unroll
        for (int k = 0; k < SPQ; ++k) {
          const int t = tid + NT * k;
          if (t < s) dst[t] = acc[k];
          acc[k] = T(0);
        }
      }
      cur = j;
    }
    if (lane < 32) reinterpret_cast<uint4*>(sgn)[lane] = sw;
    wave_lds_sync();
    {
      // row 4 lane + e + 256 k: bit 4 (lane mod 8) + e of word 4 (2 k + lane / 32) + (lane mod 32) / 8;
      // (w >> e) << 31 keeps that bit alone at the sign position
      const int wsel = (lane & 31) >> 3;
      const uint32_t sh = 4u * (lane & 7);
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const uint32_t word = sgn[4 * (2 * k + (lane >> 5)) + wsel] >> sh;
#pragma unroll
        for (int e = 0; e < 4; ++e) x[4 * k + e] = flip<T>(x[4 * k + e], word >> e);
      }
    }
    // butterflies on row bits 0,1 (e) and 8..11 (k): register index bits 0..5
#pragma unroll
    for (int b = 0; b < 6; ++b) {
#pragma unroll
      for (int i = 0; i < 64; ++i)
        if (!(i & (1 << b))) bfly(x[i], x[i | (1 << b)]);
    }
    // transpose through LDS: afterwards lane (a | b' << 2) holds rows a + 4 i + 256 b'
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      T* p = buf + 256 * k + woff[k & 7];
      if constexpr (sizeof(T) == 4) {
        *reinterpret_cast<float4*>(p) = make_float4(x[4 * k], x[4 * k + 1], x[4 * k + 2], x[4 * k + 3]);
      } else {
        *reinterpret_cast<double2*>(p) = make_double2(x[4 * k], x[4 * k + 1]);
        *reinterpret_cast<double2*>(p + 2) = make_double2(x[4 * k + 2], x[4 * k + 3]);
      }
    }
    wave_lds_sync();
#pragma unroll
    for (int i = 0; i < 64; ++i) x[i] = buf[roff[i & 7] + 32 * (i >> 3)];
    // butterflies on row bits 2..7
#pragma unroll
    for (int b = 0; b < 6; ++b) {
#pragma unroll
      for (int i = 0; i < 64; ++i)
        if (!(i & (1 << b))) bfly(x[i], x[i | (1 << b)]);
    }
    wave_lds_sync();
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
      T* p = buf + 4 * (lane + 64 * jj);
      if constexpr (sizeof(T) == 4) {
        *reinterpret_cast<float4*>(p) =
            make_float4(x[4 * jj], x[4 * jj + 1], x[4 * jj + 2], x[4 * jj + 3]);
      } else {
        *reinterpret_cast<double2*>(p) = make_double2(x[4 * jj], x[4 * jj + 1]);
        *reinterpret_cast<double2*>(p + 2) = make_double2(x[4 * jj + 2], x[4 * jj + 3]);
      }
    }
    // the registers are free again: the next unit's loads fly during the combine
    if (u + 1 < u1) {
      sw = load_signs(u + 1);
      load_chunk(u + 1, x);
    }
    __syncthreads();
    const uint32_t gmask = (uint32_t)g << (14 + LW);
#pragma unroll
    for (int k = 0; k < SPQ; ++k) {
      const unsigned char* zb = smem + (pk[k] & 0x3FFFu) * (sizeof(T) / 4);
      T z[WV];
#pragma unroll
      for (int w = 0; w < WV; ++w) z[w] = *reinterpret_cast<const T*>(zb + (size_t)w * kL * sizeof(T));
#pragma unroll
      for (int e = 0; e < LW; ++e)
#pragma unroll
        for (int w = 0; w < WV; w += 2 << e)
          z[w] = z[w] + xor_sign<T>(z[w + (1 << e)], (pk[k] >> (14 + e)) << 31);
      const uint32_t par = __builtin_popcount(pk[k] & gmask);
      acc[k] += flip<T>(z[0], par);
    }
    __syncthreads();
  }
  if (cur >= 0) {
    T* dst = partials + (blk + cur) * plan.slot_elems;
#pragma unroll
    for (int k = 0; k < SPQ; ++k) {
      const int t = tid + NT * k;
      if (t < s) dst[t] = acc[k];
    }
  }
}

// fp32 with s <= 4096: two workgroups per CU (64 KiB of chunk buffers
// each), so that one workgroup's transforms overlap the other's combine;
// otherwise the registers of one wave per SIMD
template <typename T, int SPQ>
constexpr int srht_wpe() {
  return sizeof(T) == 4 && SPQ <= 16 ? 2 : 1;
}
template <typename T, int WV, int SPQ, bool VEC>
__global__ __launch_bounds__(64 * WV) __attribute__((amdgpu_waves_per_eu(srht_wpe<T, SPQ>(),
                                                                         srht_wpe<T, SPQ>()))) void srht_kernel(
    const T* __restrict__ A, int64_t lda, const T* __restrict__ bcol, int n, PanelPlan plan,
    const uint32_t* __restrict__ idx, const uint32_t* __restrict__ signs, T* __restrict__ partials) {
  srht_body<T, WV, SPQ, VEC>(A, lda, bcol, n, plan, idx, signs, partials);
}

// signs[4 b + w] = word w of Philox block (b, TAG_SRHT_SIGN, 0): bit t of
// word w is the sign bit of row 128 b + 32 w + t
__global__ void srht_signs_kernel(int64_t blocks, uint64_t seed, uint32_t* __restrict__ signs) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= blocks) return;
  const Words4 w = philox_at((uint64_t)b, TAG_SRHT_SIGN, 0, seed);
  reinterpret_cast<uint4*>(signs)[b] = make_uint4(w.w[0], w.w[1], w.w[2], w.w[3]);
}

template <typename T>
constexpr int srht_waves() {
  return 4;
}

template <typename T>
size_t srht_lds() {
  return (size_t)srht_waves<T>() * ((size_t)kL * sizeof(T) + 512);
}

PanelPlan srht_plan(const rmm_ctx* h, int64_t m, int ncols, int s, size_t tsize) {
  return make_plan(m, ncols, 1, s, s, 4 * (int64_t)kL, h->cus * (tsize == 4 ? 2 : 1));
}

// rows covered by the sign table: whole groups of chunks
int64_t srht_sign_rows(const PanelPlan& plan) { return plan.nchunks * plan.chunk; }

template <typename T, int SPQ, bool VEC>
int launch_srht(const rmm_ctx* h, const T* A, int64_t lda, const T* b, int n, const PanelPlan& plan,
                const uint32_t* idx, const uint32_t* signs, T* partials) {
  constexpr int WV = srht_waves<T>();
  auto kern = srht_kernel<T, WV, SPQ, VEC>;
  const size_t lds = srht_lds<T>();
  RMM_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds));
  ktime_mark(h, 0);
  hipLaunchKernelGGL(kern, dim3(plan.G), dim3(64 * WV), lds, h->stream, A, lda, b, n, plan, idx, signs,
                     partials);
  ktime_mark(h, 1);
  return launch_status();
}

}  // namespace

int launch_sample_indices_u32(const rmm_ctx* h, uint64_t domain, int k, int64_t s,
                              uint32_t tag, uint64_t seed, uint32_t* out);

template <typename T>
size_t srht_workspace(const rmm_ctx* h, int64_t m, int ncols, int64_t s) {
  const PanelPlan plan = srht_plan(h, m, ncols, (int)s, sizeof(T));
  Carver c(nullptr, 0);
  c.take<uint32_t>((size_t)s);
  c.take<uint32_t>((size_t)(srht_sign_rows(plan) / 32));
  c.take<T>((size_t)plan_slots(plan) * plan.slot_elems);
  return c.off;
}

template <typename T>
int srht_run(rmm_ctx* h, int64_t m, int n, const T* A, int64_t lda, const T* b, int64_t s,
             uint64_t seed, T* C, int64_t ldc, Carver& ws) {
  const int ncols = n + (b ? 1 : 0);
  if (ncols == 0) return RMM_OK;
  const int k = ceil_log2((uint64_t)(m > 0 ? m : 1));
  if (s > (1ll << k) || s > 8192) return s > (1ll << k) ? RMM_ERR_INVALID_ARG : RMM_ERR_UNSUPPORTED;
  if (k > 30) return RMM_ERR_UNSUPPORTED;  // r_hi >> 2 must fit the packed sample field
  if (m == 0) return launch_fill_zero<T>(C, s, ncols, ldc, h->stream);
  const PanelPlan plan = srht_plan(h, m, ncols, (int)s, sizeof(T));
  uint32_t* idx = ws.take<uint32_t>((size_t)s);
  const int64_t sblocks = srht_sign_rows(plan) / 128;
  uint32_t* signs = ws.take<uint32_t>((size_t)sblocks * 4);
  T* partials = ws.take<T>((size_t)plan_slots(plan) * plan.slot_elems);
  if (!ws.fits()) return RMM_ERR_WORKSPACE_TOO_SMALL;
  RMM_TRY(launch_sample_indices_u32(h, 1ull << k, k, s, TAG_SRHT_SAMPLE, seed, idx));
  hipLaunchKernelGGL(srht_signs_kernel, dim3((unsigned)((sblocks + 255) / 256)), dim3(256), 0, h->stream,
                     sblocks, seed, signs);
  RMM_TRY(launch_status());
  const bool vec = ((uintptr_t)A % 16 == 0) && (lda % 4 == 0) &&
                   (b == nullptr || (uintptr_t)b % 16 == 0);
  int rc;
#define RMM_SRHT_CASE(SPQ)                                                                 \
  rc = vec ? launch_srht<T, SPQ, true>(h, A, lda, b, n, plan, idx, signs, partials)        \
           : launch_srht<T, SPQ, false>(h, A, lda, b, n, plan, idx, signs, partials);
  // samples per thread: s over the workgroup's 64 WV threads
  const int nt = 64 * srht_waves<T>();
  if (s <= nt) {
    RMM_SRHT_CASE(1)
  } else if (s <= 4 * nt) {
    RMM_SRHT_CASE(4)
  } else if (s <= 16 * nt) {
    RMM_SRHT_CASE(16)
  } else {
    RMM_SRHT_CASE(32)
  }
#undef RMM_SRHT_CASE
  RMM_TRY(rc);
  return launch_panel_reduce<T>(plan, partials, 1.0 / sqrt((double)s), C, ldc, h->stream);
}

template size_t srht_workspace<float>(const rmm_ctx*, int64_t, int, int64_t);
template size_t srht_workspace<double>(const rmm_ctx*, int64_t, int, int64_t);
template int srht_run<float>(rmm_ctx*, int64_t, int, const float*, int64_t, const float*,
                             int64_t, uint64_t, float*, int64_t, Carver&);
template int srht_run<double>(rmm_ctx*, int64_t, int, const double*, int64_t, const double*,
                              int64_t, uint64_t, double*, int64_t, Carver&);

}  // namespace rmm
