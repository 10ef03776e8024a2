// Gaussian-projection sketch C = (Omega / sqrt(s))^T A  (Sec. 3.2.1).
//
// A GEMM with the long dimension m as its reduction:  C (s x n') =
// Omega^T (s x m) * A (m x n').  Omega is never stored in HBM: every stage
// of KS rows, the workgroup generates the KS x 128 block of Omega it needs
// from the counter-based generator (one Philox block -> four fp32 normals,
// or two fp64 normals) straight into LDS, so the only HBM traffic is one
// read of A and the split-K partials.
//
// Tiling (gfx950, 16x16x4 MFMA, fp32 or fp64):
//  * workgroup = 4 waves = 128 sketch rows x (16 NT) columns x one K range
//    of at most 16384 rows (fp32), so no fp32 running sum spans more than
//    4096 MFMA steps; the K ranges are reduced in a fixed order in fp64;
//  * wave w covers sketch rows 32 w .. 32 w + 31 of the block as two 16-row
//    MFMA tiles against all NT column tiles;
//  * A and Omega are staged through double-buffered LDS tiles: while the
//    MFMAs consume stage t, the loads of stage t+1 are in flight and its
//    Omega block is generated; two workgroups share a CU so that one
//    group's generator work overlaps the other's MFMAs.
#include "common.hpp"
#include "rng.hpp"

namespace rmm {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename T>
struct GaussCfg;
template <>
struct GaussCfg<float> {
  static constexpr int KS = 16;   // rows per LDS stage
  static constexpr int LDT = 18;  // padded stride (elements) of a staged A column
  static constexpr int64_t KMAX = 16384;
  using acc_t = floatx4;
};
template <>
struct GaussCfg<double> {
  static constexpr int KS = 16;
  static constexpr int LDT = 17;
  static constexpr int64_t KMAX = 1 << 20;
  using acc_t = doublex4;
};

__device__ __forceinline__ floatx4 mfma16(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ doublex4 mfma16(double a, double b, doublex4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// row of the 16x16 result held in register v by lane group g = lane >> 4
__device__ __forceinline__ int mfma_row(float, int g, int v) { return 4 * g + v; }
__device__ __forceinline__ int mfma_row(double, int g, int v) { return g + 4 * v; }

// MAT: the left operand is a stored matrix Qm (m x s, column-major, ld ldq)
// instead of generated Gaussians, i.e. the kernel computes Qm^T [A | b].
// XC: the last column tile carries one more column (ncols = 16 NT t + 1, the
// sketch of [A | b] with n a multiple of 256); its 128 dot products per stage
// run on the VALU (two threads per sketch row, 8 of the 16 rows of K each)
// instead of padding a whole 16-column MFMA tile.
template <typename T, int NT, bool VEC, bool MAT, bool XC = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void gauss_sketch_kernel(
    const T* __restrict__ A, int64_t lda, const T* __restrict__ bcol, int n, int ncols,
    int64_t m, int s, int64_t kchunk, uint32_t tag, uint64_t seed, const T* __restrict__ Qm,
    int64_t ldq, T* __restrict__ partials) {
  using Cfg = GaussCfg<T>;
  using acc_t = typename Cfg::acc_t;
  // fp32 with an even number of 16-column tiles: 32 x 32 x 2 MFMAs, each
  // B operand value serving 32 sketch rows (half the instructions and half
  // the B reads of the 16 x 16 x 4 form for the same flops)
  constexpr bool W32 = sizeof(T) == 4 && NT % 2 == 0;
  constexpr int KS = Cfg::KS;
  constexpr int LDT = Cfg::LDT;
  constexpr int NCOL = NT * 16;              // columns of the MFMA tiles
  constexpr int NSTG = NCOL + (XC ? 1 : 0);  // columns staged per stage
  constexpr int GROUPS = NSTG * (KS / 4);    // 4-row groups of A per stage
  constexpr int GPT = (GROUPS + 255) / 256;  // groups per thread
  constexpr int PER = sizeof(T) == 4 ? 4 : 2;            // normals per Philox block
  constexpr int CALLS = KS * 128 / PER;                  // Philox blocks per stage
  constexpr int CPT = CALLS / 256;                       // per thread
  __shared__ T tile[2][NSTG * LDT];
  __shared__ T om[2][KS * 128];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int mi = lane & 15;
  const int kk = lane >> 4;
  const int mblk = blockIdx.x * 128;
  const int nbase = blockIdx.y * NCOL;
  const int sp = blockIdx.z;
  const int64_t k0 = (int64_t)sp * kchunk;
  int64_t k1 = k0 + kchunk;
  if (k1 > m) k1 = m;

  acc_t acc[2][NT];
  floatx16 acc32[NT / 2 > 0 ? NT / 2 : 1];
  if constexpr (W32) {
#pragma unroll
    for (int q = 0; q < NT / 2; ++q)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc32[q][v] = 0.f;
  } else {
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int q = 0; q < NT; ++q) acc[t][q] = acc_t{0, 0, 0, 0};
  }
  const int lo = lane & 31, hi = lane >> 5;

  T stage_v[GPT][4];
  auto load_stage = [&](int64_t r0) {
    const bool full = VEC && (r0 + KS <= k1);
#pragma unroll
    for (int g = 0; g < GPT; ++g) {
      const int gi = tid + 256 * g;
      const int jc = gi / (KS / 4);
      const int rg = gi - jc * (KS / 4);
      const int64_t j = nbase + jc;
      const int64_t row = r0 + 4 * rg;
#pragma unroll
      for (int e = 0; e < 4; ++e) stage_v[g][e] = T(0);
      if (gi < GROUPS && j < ncols) {
        const T* col = j < n ? A + j * lda : bcol;
        if (full) {
          if constexpr (sizeof(T) == 4) {
            const float4 x = *reinterpret_cast<const float4*>(col + row);
            stage_v[g][0] = x.x; stage_v[g][1] = x.y; stage_v[g][2] = x.z; stage_v[g][3] = x.w;
          } else {
            const double2 x = *reinterpret_cast<const double2*>(col + row);
            const double2 y = *reinterpret_cast<const double2*>(col + row + 2);
            stage_v[g][0] = x.x; stage_v[g][1] = x.y; stage_v[g][2] = y.x; stage_v[g][3] = y.y;
          }
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (row + e < k1) stage_v[g][e] = col[row + e];
        }
      }
    }
  };
  auto store_stage = [&](int b) {
#pragma unroll
    for (int g = 0; g < GPT; ++g) {
      const int gi = tid + 256 * g;
      if (gi < GROUPS) {
        const int jc = gi / (KS / 4);
        const int rg = gi - jc * (KS / 4);
#pragma unroll
        for (int e = 0; e < 4; ++e) tile[b][jc * LDT + 4 * rg + e] = stage_v[g][e];
      }
    }
  };
  // stored left operand: thread = (column c, 4 consecutive rows), 16-byte
  // loads along a column when aligned
  constexpr int QG = 128 * (KS / 4);         // (column, 4-row group) pairs per stage
  constexpr int QPT = (QG + 255) / 256;
  T qv[QPT][4];
  auto load_q = [&](int64_t r0) {
#pragma unroll
    for (int u = 0; u < QPT; ++u) {
      const int gi = tid + 256 * u;
      const int c = gi / (KS / 4), kg = gi - c * (KS / 4);
      const int64_t row = r0 + 4 * kg;
      const int col = mblk + c;
#pragma unroll
      for (int e = 0; e < 4; ++e) qv[u][e] = T(0);
      if (gi < QG && col < s) {
        const T* qc = Qm + (int64_t)col * ldq;
        if (VEC && row + 4 <= k1) {
          if constexpr (sizeof(T) == 4) {
            const float4 x = *reinterpret_cast<const float4*>(qc + row);
            qv[u][0] = x.x; qv[u][1] = x.y; qv[u][2] = x.z; qv[u][3] = x.w;
          } else {
            const double2 x = *reinterpret_cast<const double2*>(qc + row);
            const double2 y = *reinterpret_cast<const double2*>(qc + row + 2);
            qv[u][0] = x.x; qv[u][1] = x.y; qv[u][2] = y.x; qv[u][3] = y.y;
          }
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (row + e < k1) qv[u][e] = qc[row + e];
        }
      }
    }
  };
  auto store_q = [&](int b) {
#pragma unroll
    for (int u = 0; u < QPT; ++u) {
      const int gi = tid + 256 * u;
      if (gi < QG) {
        const int c = gi / (KS / 4), kg = gi - c * (KS / 4);
#pragma unroll
        for (int e = 0; e < 4; ++e) om[b][(4 * kg + e) * 128 + c] = qv[u][e];
      }
    }
  };
  // Omega[r0 + k, mblk + c] for k < KS, c < 128, written to om[b][k * 128 + c].
  // Entries of rows past the K range are generated too (always finite): they
  // meet zero rows of the A tile.  Columns past s are zero without generation.
  auto gen_omega = [&](int64_t r0, int b) {
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      const int call = tid + 256 * u;
      const int k = call / (128 / PER);
      const int cq = call - k * (128 / PER);
      const int64_t i = r0 + k;
      const int c0 = mblk + PER * cq;
      T z[PER];
#pragma unroll
      for (int e = 0; e < PER; ++e) z[e] = T(0);
      if (c0 < s) {
        if constexpr (sizeof(T) == 4) gauss4_f32((uint64_t)i, (uint32_t)(c0 >> 2), tag, seed, z);
        else gauss2_f64((uint64_t)i, (uint32_t)(c0 >> 1), tag, seed, z);
      }
      T* o = &om[b][k * 128 + PER * cq];
      if constexpr (sizeof(T) == 4)
        *reinterpret_cast<float4*>(o) = make_float4(z[0], z[1], z[2], z[3]);
      else
        *reinterpret_cast<double2*>(o) = make_double2(z[0], z[1]);
    }
  };

  const int64_t nst = (k1 - k0 + KS - 1) / KS;
  if (nst > 0) {
    load_stage(k0);
    if constexpr (MAT) {
      load_q(k0);
      store_q(0);
    } else {
      gen_omega(k0, 0);
    }
    store_stage(0);
  }
  __syncthreads();
  const int arow = 32 * wave + mi;
  // extra column: this thread's sketch row and half of the stage's K rows
  const bool has_xc = XC && blockIdx.y + 1 == gridDim.y;
  const int xr = tid & 127, xh = tid >> 7;
  T xacc = T(0);
  const bool wave_rows = mblk + 32 * wave < s;  // uniform per wave
  for (int64_t st = 0; st < nst; ++st) {
    const int b = (int)(st & 1);
    const int64_t r0 = k0 + st * KS;
    const bool more = st + 1 < nst;
    if (more) {
      load_stage(r0 + KS);
      if constexpr (MAT) load_q(r0 + KS);
    }
    if constexpr (XC) {
      if (has_xc) {
        const T* tx = &tile[b][NCOL * LDT + 8 * xh];
        const T* ox = &om[b][8 * xh * 128 + xr];
#pragma unroll
        for (int k = 0; k < 8; ++k) xacc += ox[k * 128] * tx[k];
      }
    }
    // a wave whose 32 sketch rows all lie past s skips the MFMAs
    if (wave_rows && W32) {
      if constexpr (W32) {
#pragma unroll
        for (int ks = 0; ks < KS / 2; ++ks) {
          const float a = om[b][(2 * ks + hi) * 128 + 32 * wave + lo];
          const float* tb = &tile[b][lo * LDT + 2 * ks + hi];
#pragma unroll
          for (int q = 0; q < NT / 2; ++q)
            acc32[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, tb[q * 32 * LDT], acc32[q], 0, 0, 0);
        }
      }
    } else if (wave_rows) {
#pragma unroll
      for (int ks = 0; ks < KS / 4; ++ks) {
        const T a0 = om[b][(4 * ks + kk) * 128 + arow];
        const T a1 = om[b][(4 * ks + kk) * 128 + arow + 16];
        const T* tb = &tile[b][mi * LDT + 4 * ks + kk];
#pragma unroll
        for (int q = 0; q < NT; ++q) {
          const T bv = tb[q * 16 * LDT];
          acc[0][q] = mfma16(a0, bv, acc[0][q]);
          acc[1][q] = mfma16(a1, bv, acc[1][q]);
        }
      }
    }
    if (more) {
      if constexpr (MAT) store_q(b ^ 1);
      else gen_omega(r0 + KS, b ^ 1);
      store_stage(b ^ 1);
    }
    __syncthreads();
  }
  T* dst = partials + (int64_t)sp * ncols * s;
  if constexpr (XC) {
    if (has_xc) {
      // the two halves of each row meet in LDS (free after the last barrier)
      if (xh == 1) om[0][xr] = xacc;
      __syncthreads();
      const int r = mblk + xr;
      if (xh == 0 && r < s) dst[(int64_t)(nbase + NCOL) * s + r] = xacc + om[0][xr];
    }
  }
  if constexpr (W32) {
    // register v of the 32 x 32 result holds row 8 (v / 4) + 4 hi + v % 4,
    // column lo
#pragma unroll
    for (int q = 0; q < NT / 2; ++q) {
      const int64_t j = nbase + q * 32 + lo;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int r = mblk + 32 * wave + 8 * (v >> 2) + 4 * hi + (v & 3);
        if (j < ncols && r < s) dst[j * s + r] = acc32[q][v];
      }
    }
  } else {
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int q = 0; q < NT; ++q) {
        const int64_t j = nbase + q * 16 + mi;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = mblk + 32 * wave + 16 * t + mfma_row(T(0), kk, v);
          if (j < ncols && r < s) dst[j * s + r] = acc[t][q][v];
        }
      }
  }
}

// C[r + j * ldc] (TRANS: C[j + r * ldc]) = scale * (sum of the split
// partials) + beta C
template <typename T, bool TRANS>
__global__ void splitk_reduce_kernel(const T* __restrict__ partials, int splits, int64_t plane,
                                     double scale, double beta, int s, T* __restrict__ C, int64_t ldc) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (r >= s) return;
  double acc = 0.0;
  for (int p = 0; p < splits; ++p) acc += (double)partials[p * plane + j * s + r];
  T* dst = TRANS ? C + j + r * ldc : C + r + j * ldc;
  double v = acc * scale;
  if (beta != 0.0) v += beta * (double)*dst;
  *dst = (T)v;
}

// The transposed form for wide outputs (s >= 512) through a 64 x 64 LDS
// tile: the partials are read along r and C is written along j, both
// contiguous (the kernel above writes C^T with a stride of ldc between
// neighbouring threads); the splits are summed in the same order.
template <typename T>
__global__ __launch_bounds__(256) void splitk_reduce_t_kernel(const T* __restrict__ partials, int splits,
                                                              int64_t plane, double scale, double beta, int s,
                                                              int ncols, T* __restrict__ C, int64_t ldc) {
  __shared__ double tile[64][65];
  const int r0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll 4
  for (int k = 0; k < 16; ++k) {
    const int j = j0 + ty + 4 * k, r = r0 + tx;
    double acc = 0.0;
    if (r < s && j < ncols)
      for (int p = 0; p < splits; ++p) acc += (double)partials[p * plane + (int64_t)j * s + r];
    tile[ty + 4 * k][tx] = acc;
  }
  __syncthreads();
#pragma unroll 4
  for (int k = 0; k < 16; ++k) {
    const int r = r0 + ty + 4 * k, j = j0 + tx;
    if (r < s && j < ncols) {
      T* dst = C + j + (int64_t)r * ldc;
      double v = tile[tx][ty + 4 * k] * scale;
      if (beta != 0.0) v += beta * (double)*dst;
      *dst = (T)v;
    }
  }
}

namespace {

struct GaussShape {
  int NT;
  bool xc;  // one extra column in the last tile
  int ntiles;
  int mtiles;
  int splits;
  int64_t kchunk;
};

template <typename T>
GaussShape gauss_shape(const rmm_ctx* h, int64_t m, int ncols, int s) {
  GaussShape g;
  // fp64 accumulators for 17 column tiles do not fit two waves per SIMD
  const int ntmax = sizeof(T) == 4 ? 17 : 8;
  g.NT = ncols > 128 ? ntmax : ncols > 64 ? 8 : ncols > 16 ? 4 : 1;
  g.xc = false;
  // fp32: 256-column tiles without padding when ncols is 256 t or 256 t + 1
  if (sizeof(T) == 4 && ncols > 128 && (ncols % 256 == 0 || ncols % 256 == 1)) {
    g.NT = 16;
    g.xc = ncols % 256 == 1;
  }
  g.ntiles = (ncols - (g.xc ? 1 : 0) + g.NT * 16 - 1) / (g.NT * 16);
  g.mtiles = (s + 127) / 128;
  const int64_t KS = GaussCfg<T>::KS;
  // enough K splits for about four workgroups per CU, each at most KMAX rows
  // and at least 16 stages (a short problem is latency bound: its stages run
  // one after another inside a workgroup)
  int64_t want = (4ll * h->cus + (int64_t)g.mtiles * g.ntiles - 1) / ((int64_t)g.mtiles * g.ntiles);
  const int64_t minsplit = (m + GaussCfg<T>::KMAX - 1) / GaussCfg<T>::KMAX;
  const int64_t maxsplit = (m + 16 * KS - 1) / (16 * KS);
  if (want > maxsplit) want = maxsplit;
  if (want < minsplit) want = minsplit;
  if (want < 1) want = 1;
  int64_t kc = (m + want - 1) / want;
  kc = (kc + KS - 1) / KS * KS;
  if (kc < KS) kc = KS;
  g.kchunk = kc;
  g.splits = (int)((m + kc - 1) / kc);
  if (g.splits < 1) g.splits = 1;
  return g;
}

template <typename T, int NT, bool XC = false>
int launch_gauss(const rmm_ctx* h, const GaussShape& g, const T* A, int64_t lda, const T* b,
                 int n, int ncols, int64_t m, int s, uint32_t tag, uint64_t seed, const T* Qm,
                 int64_t ldq, T* partials) {
  dim3 grid((unsigned)g.mtiles, (unsigned)g.ntiles, (unsigned)g.splits);
  bool vec = ((uintptr_t)A % 16 == 0) && (lda % 4 == 0) && (b == nullptr || (uintptr_t)b % 16 == 0);
  if (Qm) vec = vec && ((uintptr_t)Qm % 16 == 0) && (ldq % 4 == 0);
#define RMM_GS_LAUNCH(V, M)                                                                    \
  hipLaunchKernelGGL((gauss_sketch_kernel<T, NT, V, M, XC>), grid, dim3(256), 0, h->stream, A, lda, b, \
                     n, ncols, m, s, g.kchunk, tag, seed, Qm, ldq, partials)
  ktime_mark(h, 0);
  if (Qm) {
    if (vec) RMM_GS_LAUNCH(true, true);
    else RMM_GS_LAUNCH(false, true);
  } else {
    if (vec) RMM_GS_LAUNCH(true, false);
    else RMM_GS_LAUNCH(false, false);
  }
  ktime_mark(h, 1);
#undef RMM_GS_LAUNCH
  return launch_status();
}

}  // namespace

template <typename T>
size_t gauss_sketch_workspace(const rmm_ctx* h, int64_t m, int ncols, int64_t s) {
  const GaussShape g = gauss_shape<T>(h, m, ncols, (int)s);
  Carver c(nullptr, 0);
  c.take<T>((size_t)g.splits * ncols * s);
  return c.off;
}

namespace {

// C (s x ncols, or its transpose) = scale * L^T [A | b] + beta C, L = Qm
// (m x s) when given, else Omega of stream `tag`.
template <typename T>
int project_any(rmm_ctx* h, int64_t m, int n, const T* A, int64_t lda, const T* b, int64_t s,
                uint32_t tag, uint64_t seed, const T* Qm, int64_t ldq, double scale, T* C,
                int64_t ldc, bool trans, Carver& ws, double beta = 0.0) {
  const int ncols = n + (b ? 1 : 0);
  if (ncols == 0) return RMM_OK;
  if (m == 0) {
    if (beta == 0.0) return launch_fill_zero<T>(C, s, ncols, ldc, h->stream);
    return beta == 1.0 ? RMM_OK : RMM_ERR_UNSUPPORTED;
  }
  const GaussShape g = gauss_shape<T>(h, m, ncols, (int)s);
  const size_t mark = ws.off;  // the partials are released on return
  T* partials = ws.take<T>((size_t)g.splits * ncols * s);
  if (!ws.fits()) return RMM_ERR_WORKSPACE_TOO_SMALL;
  int rc;
  switch (g.NT) {
    case 17:
      if constexpr (sizeof(T) == 4) {
        rc = launch_gauss<T, 17>(h, g, A, lda, b, n, ncols, m, (int)s, tag, seed, Qm, ldq, partials);
        break;
      }
      return RMM_ERR_UNSUPPORTED;
    case 16:
      if constexpr (sizeof(T) == 4) {
        rc = g.xc ? launch_gauss<T, 16, true>(h, g, A, lda, b, n, ncols, m, (int)s, tag, seed, Qm,
                                              ldq, partials)
                  : launch_gauss<T, 16, false>(h, g, A, lda, b, n, ncols, m, (int)s, tag, seed,
                                               Qm, ldq, partials);
        break;
      }
      return RMM_ERR_UNSUPPORTED;
    case 8: rc = launch_gauss<T, 8>(h, g, A, lda, b, n, ncols, m, (int)s, tag, seed, Qm, ldq, partials); break;
    case 4: rc = launch_gauss<T, 4>(h, g, A, lda, b, n, ncols, m, (int)s, tag, seed, Qm, ldq, partials); break;
    default: rc = launch_gauss<T, 1>(h, g, A, lda, b, n, ncols, m, (int)s, tag, seed, Qm, ldq, partials); break;
  }
  RMM_TRY(rc);
  dim3 grid((unsigned)((s + 255) / 256), (unsigned)ncols);
  if (trans && s >= 512)
    hipLaunchKernelGGL((splitk_reduce_t_kernel<T>), dim3((unsigned)((s + 63) / 64), (unsigned)((ncols + 63) / 64)),
                       dim3(256), 0, h->stream, partials, g.splits, (int64_t)ncols * s, scale, beta, (int)s,
                       ncols, C, ldc);
  else if (trans)
    hipLaunchKernelGGL((splitk_reduce_kernel<T, true>), grid, dim3(256), 0, h->stream, partials, g.splits,
                       (int64_t)ncols * s, scale, beta, (int)s, C, ldc);
  else
    hipLaunchKernelGGL((splitk_reduce_kernel<T, false>), grid, dim3(256), 0, h->stream, partials, g.splits,
                       (int64_t)ncols * s, scale, beta, (int)s, C, ldc);
  ws.off = mark;
  return launch_status();
}

}  // namespace

// Y (s x ncols) = Omega^T [A | b] * scale with Omega of stream `tag`.
template <typename T>
int gauss_project(rmm_ctx* h, int64_t m, int n, const T* A, int64_t lda, const T* b,
                  int64_t s, uint32_t tag, uint64_t seed, double scale, T* C, int64_t ldc,
                  Carver& ws) {
  return project_any<T>(h, m, n, A, lda, b, s, tag, seed, nullptr, 0, scale, C, ldc, false, ws);
}

// Z (ncols x s, ld ldz) = A^T Qm + beta Z for A (m x ncols) and Qm (m x s):
// the same kernel with the stored matrix as its left operand, written
// transposed.
template <typename T>
int project_tn(rmm_ctx* h, int64_t m, int ncols, const T* A, int64_t lda, const T* Qm, int64_t ldq,
               int64_t s, T* Z, int64_t ldz, Carver& ws, double beta) {
  return project_any<T>(h, m, ncols, A, lda, nullptr, s, 0, 0, Qm, ldq, 1.0, Z, ldz, true, ws, beta);
}

template <typename T>
int gauss_sketch_run(rmm_ctx* h, int64_t m, int n, const T* A, int64_t lda, const T* b,
                     int64_t s, uint64_t seed, T* C, int64_t ldc, Carver& ws) {
  return gauss_project<T>(h, m, n, A, lda, b, s, TAG_GAUSS_SKETCH, seed, 1.0 / sqrt((double)s), C,
                          ldc, ws);
}

template size_t gauss_sketch_workspace<float>(const rmm_ctx*, int64_t, int, int64_t);
template size_t gauss_sketch_workspace<double>(const rmm_ctx*, int64_t, int, int64_t);
template int gauss_sketch_run<float>(rmm_ctx*, int64_t, int, const float*, int64_t, const float*,
                                     int64_t, uint64_t, float*, int64_t, Carver&);
template int gauss_sketch_run<double>(rmm_ctx*, int64_t, int, const double*, int64_t,
                                      const double*, int64_t, uint64_t, double*, int64_t, Carver&);
template int project_tn<float>(rmm_ctx*, int64_t, int, const float*, int64_t, const float*, int64_t,
                               int64_t, float*, int64_t, Carver&, double);
template int project_tn<double>(rmm_ctx*, int64_t, int, const double*, int64_t, const double*, int64_t,
                                int64_t, double*, int64_t, Carver&, double);
template int gauss_project<float>(rmm_ctx*, int64_t, int, const float*, int64_t, const float*,
                                  int64_t, uint32_t, uint64_t, double, float*, int64_t, Carver&);
template int gauss_project<double>(rmm_ctx*, int64_t, int, const double*, int64_t, const double*,
                                   int64_t, uint32_t, uint64_t, double, double*, int64_t, Carver&);

}  // namespace rmm
