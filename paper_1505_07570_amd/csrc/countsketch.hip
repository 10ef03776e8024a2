// CountSketch C = S^T A (Sec. 3.2.3, Alg. 3.1, streaming fashion).
//
// S has one nonzero per row: row i of A is added, with sign g_i, into row
// h_i of C.  One pass over A; no scaling.
//
// Kernel layout (one workgroup of WAVES waves per column panel x row-chunk
// range, see PanelPlan):
//  * wave w owns column (panel start + w) and a private LDS accumulator of
//    ST buckets, so every LDS add to a bucket comes from one wave in program
//    order: the per-block sums are reproducible run to run;
//  * the CountSketch words of a chunk's rows are generated once per chunk
//    by the whole workgroup (one Philox block per 4 rows) into an LDS table
//    shared by the WAVES columns;
//  * A is streamed with 16-byte loads, 4 consecutive rows per lane, issued
//    before the hash generation so the loads are in flight meanwhile;
//  * at a panel change the accumulators are flushed to a partial slot and a
//    fixed-order reduction (reduce.hip) sums the slots into C.
#include <algorithm>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "rng.hpp"

namespace rmm {

template <typename T>
__device__ __forceinline__ T apply_sign(T v, uint32_t packed);
template <>
__device__ __forceinline__ float apply_sign<float>(float v, uint32_t packed) {
  return __uint_as_float(__float_as_uint(v) ^ (packed & 0x80000000u));
}
template <>
__device__ __forceinline__ double apply_sign<double>(double v, uint32_t packed) {
  return (packed >> 31) ? -v : v;
}

template <typename T, int WAVES, int UNROLL, bool VEC>
__global__ __launch_bounds__(WAVES * 64) void countsketch_kernel(
    const T* __restrict__ A, int64_t lda, const T* __restrict__ bcol, int n, PanelPlan plan,
    uint64_t seed, T* __restrict__ partials) {
  constexpr int CH = 256 * UNROLL;  // rows per chunk
  constexpr int NT = WAVES * 64;
  extern __shared__ __align__(16) unsigned char smem[];
  T* acc = reinterpret_cast<T*>(smem);
  uint32_t* hbuf = reinterpret_cast<uint32_t*>(smem + (size_t)WAVES * plan.ST * sizeof(T));

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int64_t blk = blockIdx.x;
  const int64_t u0 = plan_start(plan, blk);
  const int64_t u1 = plan_start(plan, blk + 1);
  const uint32_t s = (uint32_t)plan.s;
  const int ST = plan.ST;
  T* my_acc = acc + (size_t)wave * ST;

  // this wave's column for unit u (nullptr when the panel is narrower)
  auto column = [&](int64_t u) -> const T* {
    const int panel = (int)(u / plan.nchunks / plan.BT);
    const int64_t j = plan_col0(plan, panel) + wave;
    if (j >= plan_col0(plan, panel + 1)) return nullptr;
    return j < n ? A + j * lda : bcol;
  };
  auto load_unit = [&](int64_t u, T v[UNROLL][4]) {
    const T* col = column(u);
    const int64_t r0 = (u % plan.nchunks) * CH;
    if (col == nullptr) return;
    if (VEC && r0 + CH <= plan.m) {
#pragma unroll
      for (int k = 0; k < UNROLL; ++k) {
        const T* p = col + r0 + 256 * k + 4 * lane;
        if constexpr (sizeof(T) == 4) {
          const float4 x = ld_stream(reinterpret_cast<const float4*>(p));
          v[k][0] = x.x; v[k][1] = x.y; v[k][2] = x.z; v[k][3] = x.w;
        } else {
          const double2 x = ld_stream(reinterpret_cast<const double2*>(p));
          const double2 y = ld_stream(reinterpret_cast<const double2*>(p + 2));
          v[k][0] = x.x; v[k][1] = x.y; v[k][2] = y.x; v[k][3] = y.y;
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < UNROLL; ++k)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t row = r0 + 256 * k + 4 * lane + e;
          v[k][e] = row < plan.m ? col[row] : T(0);
        }
    }
  };

  T v[UNROLL][4], vn[UNROLL][4];
  if (u0 < u1) load_unit(u0, v);
  int64_t cur_vp = -1;
  int buf = 0;
  for (int64_t u = u0; u < u1; ++u) {
    const int64_t vp = u / plan.nchunks;
    const int64_t c = u - vp * plan.nchunks;
    const int panel = (int)(vp / plan.BT);
    const int bt = (int)(vp - (int64_t)panel * plan.BT);
    if (vp != cur_vp) {
      if (cur_vp >= 0) {
        __syncthreads();
        T* dst = partials + (blk + cur_vp) * plan.slot_elems;
        for (int i = tid; i < WAVES * ST; i += NT) dst[i] = acc[i];
      }
      __syncthreads();
      for (int i = tid; i < WAVES * ST; i += NT) acc[i] = T(0);
      cur_vp = vp;
    }
    const int64_t r0 = c * CH;
    const bool active = column(u) != nullptr;
    // CountSketch words of this chunk, packed as bucket | sign << 31
    uint32_t* hb = hbuf + buf * CH;
#pragma unroll
    for (int q = tid; q < CH / 4; q += NT) {
      const Words4 w = philox_at((uint64_t)(r0 >> 2) + q, TAG_COUNTSKETCH, 0, seed);
      uint4 pk;
      pk.x = cs_bucket(w.w[0], s) | (w.w[0] << 31);
      pk.y = cs_bucket(w.w[1], s) | (w.w[1] << 31);
      pk.z = cs_bucket(w.w[2], s) | (w.w[2] << 31);
      pk.w = cs_bucket(w.w[3], s) | (w.w[3] << 31);
      *reinterpret_cast<uint4*>(hb + 4 * q) = pk;
    }
    __syncthreads();
    // next unit's loads go out before this unit's scatter-adds
    if (u + 1 < u1) load_unit(u + 1, vn);
    if (active) {
      const bool fast = (r0 + CH <= plan.m) && (plan.BT == 1);
      if (fast) {
#pragma unroll
        for (int k = 0; k < UNROLL; ++k) {
          const uint4 pk = *reinterpret_cast<const uint4*>(hb + 256 * k + 4 * lane);
          atomicAdd(my_acc + (pk.x & 0x7FFFFFFFu), apply_sign<T>(v[k][0], pk.x));
          atomicAdd(my_acc + (pk.y & 0x7FFFFFFFu), apply_sign<T>(v[k][1], pk.y));
          atomicAdd(my_acc + (pk.z & 0x7FFFFFFFu), apply_sign<T>(v[k][2], pk.z));
          atomicAdd(my_acc + (pk.w & 0x7FFFFFFFu), apply_sign<T>(v[k][3], pk.w));
        }
      } else {
        const uint32_t tile0 = (uint32_t)bt * (uint32_t)ST;
#pragma unroll
        for (int k = 0; k < UNROLL; ++k) {
          const int off = 256 * k + 4 * lane;
          const uint4 pk = *reinterpret_cast<const uint4*>(hb + off);
          const uint32_t pw[4] = {pk.x, pk.y, pk.z, pk.w};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const uint32_t bucket = (pw[e] & 0x7FFFFFFFu) - tile0;
            if (r0 + off + e < plan.m && bucket < (uint32_t)ST)
              atomicAdd(my_acc + bucket, apply_sign<T>(v[k][e], pw[e]));
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < UNROLL; ++k)
#pragma unroll
      for (int e = 0; e < 4; ++e) v[k][e] = vn[k][e];
    buf ^= 1;
  }
  if (cur_vp >= 0) {
    __syncthreads();
    T* dst = partials + (blk + cur_vp) * plan.slot_elems;
    for (int i = tid; i < WAVES * ST; i += NT) dst[i] = acc[i];
  }
}

// ---- scheduled variant (s <= 16384) ------------------------------------------------
//
// LDS float atomics are slow and a dependent read-modify-write per row
// leaves the LDS idle for a round trip each time, so the scatter-add is made
// conflict free ahead of time and issued in batches.  Rows are taken in
// windows of 256 consecutive rows; lane l of a wave holds rows 4 l + e
// (e = 0..3) of each window.  A pre-pass records for every row its bucket,
// its sign and whether a row of smaller index in its window has the same
// bucket ("later").  The first row of every bucket in a window does a plain
// LDS read-modify-write: those buckets are pairwise distinct, so the four
// reads of a lane go out together, then the four writes.  A later row sends
// its plain read-modify-write to a scratch slot after the buckets instead and
// then adds its value atomically into its bucket, after the plain writes in
// program order (the LDS executes a wave's instructions in order).
// Entry (16 bits): bits 0-13 bucket, bit 14 later, bit 15 sign.  The table is
// padded to whole row chunks; rows past the end of A read 0x4000 (their
// values are zero).  Within a chunk of UN windows the entries are stored
// lane-major: the 4 UN entries that lane l uses (rows 256 k + 4 l + e) are
// contiguous, so a lane fetches them with a few 16-byte loads.

constexpr int kCsSchedMaxS = 1 << 14;
constexpr int kCsWindow = 256;

// rows per chunk (the unit of work): 8 windows, one 16-byte (fp32) or two
// (fp64) loads of A per lane and window.  Smaller units measured faster:
// three of them in flight per wave, each issued as one burst of loads.
template <typename T>
constexpr int sched_chunk() {
  return 2048;
}

// table entries (rows) for m rows: whole chunks of the widest type
__host__ __device__ inline int64_t cs_table_rows(int64_t m) {
  const int64_t c = sched_chunk<float>();
  return (m + c - 1) / c * c;
}
// the table is followed by kCsZeroBytes zero bytes, the load target of rows past m
constexpr int kCsZeroBytes = 256;
inline size_t cs_table_elems(int64_t m) { return (size_t)cs_table_rows(m) + kCsZeroBytes / 2; }

// one wave per 256-row window; un: windows per chunk; owner: this wave's s LDS words
__device__ __forceinline__ void cs_schedule_body(int64_t m, uint32_t s, uint64_t seed, int un,
                                                 uint16_t* __restrict__ table, int64_t win,
                                                 uint32_t* __restrict__ owner) {
  const int lane = threadIdx.x & 63;
  const int64_t row0 = win * kCsWindow + 4 * lane;
  const Words4 w = philox_at((uint64_t)(row0 >> 2), TAG_COUNTSKETCH, 0, seed);
  uint32_t b[4];
  bool ok[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    b[e] = cs_bucket(w.w[e], s);
    ok[e] = row0 + e < m;
  }
  // the smallest window position per bucket wins: set, min, read back
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (ok[e]) owner[b[e]] = 0xFFFFFFFFu;
  wave_lds_sync();
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (ok[e]) atomicMin(owner + b[e], (uint32_t)(4 * lane + e));
  wave_lds_sync();
  uint32_t o[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const uint32_t later = owner[b[e]] != (uint32_t)(4 * lane + e) ? 1u : 0u;
    o[e] = ok[e] ? (b[e] | (later << 14) | ((w.w[e] & 1u) << 15)) : 0x4000u;
  }
  if (win == 0 && lane < kCsZeroBytes / 16)
    reinterpret_cast<uint4*>(table + cs_table_rows(m))[lane] = make_uint4(0u, 0u, 0u, 0u);
  const int64_t c = win / un;
  const int64_t pos = c * kCsWindow * un + 4 * ((int64_t)lane * un + (win - c * un));
  *reinterpret_cast<uint2*>(table + pos) = make_uint2(o[0] | (o[1] << 16), o[2] | (o[3] << 16));
}

__global__ __launch_bounds__(64) void cs_schedule_kernel(int64_t m, uint32_t s, uint64_t seed,
                                                         int un, uint16_t* __restrict__ table) {
  extern __shared__ uint32_t cs_owner[];
  cs_schedule_body(m, s, seed, un, table, blockIdx.x, cs_owner);
}

// worker = one workgroup of WAVES waves; unit = (panel of up to WAVES
// columns, chunk of rows).  Wave w owns column (panel start + w) and a
// private LDS accumulator of s buckets plus the scratch slot; it loads its
// own copy of the chunk's table entries (the WAVES waves of a workgroup read
// the same entries at about the same time, mostly from cache), so the waves
// never wait for each other.  A and the entries are loaded one unit ahead.
template <typename T>
struct CsUnit {
  T v[sched_chunk<T>() / kCsWindow][4];
  uint4 t[sched_chunk<T>() / kCsWindow / 2];  // entries of windows 2 j and 2 j + 1
};

template <typename T, bool VEC, int WAVES>
__device__ __forceinline__ void cs_sched_body(const T* __restrict__ A, int64_t lda,
                                              const T* __restrict__ bcol, int n,
                                              const PanelPlan& plan,
                                              const uint16_t* __restrict__ table,
                                              T* __restrict__ partials, int64_t wk) {
  constexpr int CH = sched_chunk<T>();
  constexpr int UN = CH / kCsWindow;
  extern __shared__ __align__(16) unsigned char smem[];
  const int s = plan.s;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T* my = reinterpret_cast<T*>(smem) + (size_t)wave * (s + 4);
  const int64_t u0 = plan_start(plan, wk);
  const int64_t u1 = plan_start(plan, wk + 1);
  const int64_t nch = plan.nchunks;
  const int64_t m = plan.m;
  for (int i = lane; i < s + 4; i += 64) my[i] = T(0);

  // this wave's column of panel vp.  A wave without a column in a narrower
  // panel streams the panel's first column along with wave 0 (cache hits)
  // and adds it into its accumulator, which lands in a partial slot that no
  // reduction reads: every wave then runs the same loads and LDS work.
  auto column = [&](int64_t vp) -> const T* {
    const int64_t j0 = plan_col0(plan, (int)vp);
    int64_t j = j0 + wave;
    if (j >= plan_col0(plan, (int)vp + 1)) j = j0;
    return j < n ? A + j * lda : bcol;
  };
  // Rows past m load zeros from the bytes after the table.  Both branches
  // issue the same loads and no load result is touched here, so the wait
  // before a value's first use covers that value's own load only.
  const T* const zeros = reinterpret_cast<const T*>(table + cs_table_rows(m));
  // entries of windows 2 j and 2 j + 1 of the chunk at row r0
  auto load_tab = [&](int64_t r0, int j, CsUnit<T>& x) {
    x.t[j] = reinterpret_cast<const uint4*>(table + r0 + 4 * UN * lane)[j];
  };
  // A values of window k of column col, chunk at row r0
  auto load_win = [&](const T* col, int64_t r0, bool full, int k, CsUnit<T>& x) {
    const T* q = col + r0 + kCsWindow * k + 4 * lane;
    if (!full) {
      // VEC implies m % 4 == 0: a lane's 4 rows are all in range or all out
      if (VEC) q = r0 + kCsWindow * k + 4 * lane < m ? q : zeros;
    }
    if constexpr (VEC && sizeof(T) == 4) {
      const float4 v4 = ld_stream(reinterpret_cast<const float4*>(q));
      x.v[k][0] = v4.x; x.v[k][1] = v4.y; x.v[k][2] = v4.z; x.v[k][3] = v4.w;
    } else if constexpr (VEC) {
      const double2 q0 = ld_stream(reinterpret_cast<const double2*>(q));
      const double2 q1 = ld_stream(reinterpret_cast<const double2*>(q + 2));
      x.v[k][0] = q0.x; x.v[k][1] = q0.y; x.v[k][2] = q1.x; x.v[k][3] = q1.y;
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const T* qe = q + e;
        if (!full) qe = r0 + kCsWindow * k + 4 * lane + e < m ? qe : zeros;
        x.v[k][e] = *qe;
      }
    }
  };
  auto scatter_win = [&](const CsUnit<T>& x, int k) {
    const uint32_t w0 = (k & 1) ? x.t[k >> 1].z : x.t[k >> 1].x;
    const uint32_t w1 = (k & 1) ? x.t[k >> 1].w : x.t[k >> 1].y;
    const uint32_t ent[4] = {w0 & 0xFFFFu, w0 >> 16, w1 & 0xFFFFu, w1 >> 16};
    T val[4], old[4];
    uint32_t f[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      val[e] = apply_sign<T>(x.v[k][e], ent[e] << 16);
      f[e] = ent[e] & 0x7FFFu;  // bucket, plus 0x4000 for a later row
    }
    // the bucket, or the scratch slot s for a later row (0x4000 >= s)
#pragma unroll
    for (int e = 0; e < 4; ++e) old[e] = my[min(f[e], (uint32_t)s)];
    // all four reads go out before the first wait for their data
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int e = 0; e < 4; ++e) my[min(f[e], (uint32_t)s)] = old[e] + val[e];
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (f[e] >= 0x4000u) atomicAdd(my + (f[e] - 0x4000u), val[e]);
  };
  auto scatter = [&](const CsUnit<T>& x) {
#pragma unroll
    for (int k = 0; k < UN; ++k) scatter_win(x, k);
  };

  // all loads of a unit, issued together (a burst keeps more bytes in flight
  // than loads spread over the unit's additions, measured)
  auto load = [&](const T* lcol, int64_t r0, CsUnit<T>& x) {
#pragma unroll
    for (int k = 0; k < UN; ++k) {
      if ((k & 1) == 0) load_tab(r0, k >> 1, x);
      load_win(lcol, r0, r0 + CH <= m, k, x);
    }
    __builtin_amdgcn_sched_barrier(0);
  };
  // Units u = (panel, chunk) are loaded two ahead of their addition, into
  // three register buffers used in rotation.  Every step issues the same
  // loads in the same order, so the wait before a value's first use only
  // covers that value's own load.  Both cursors advance without divisions.
  int64_t lp = u0 / nch, lc = u0 - (u0 / nch) * nch;  // next unit to load
  const T* lcol = column(lp);
  int64_t ap = lp, ac = lc;  // next unit to add
  int64_t cur = ap;          // panel of the accumulator contents
  auto load_next = [&](CsUnit<T>& x) {
    load(lcol, lc * CH, x);
    if (++lc == nch) {
      lc = 0;
      lcol = column(++lp);
    }
  };
  auto add_next = [&](const CsUnit<T>& x) {
    if (ap != cur) {
      T* dst = partials + (wk + cur) * plan.slot_elems + (size_t)wave * s;
      for (int i = lane; i < s; i += 64) {
        dst[i] = my[i];
        my[i] = T(0);
      }
      cur = ap;
    }
    scatter(x);
    if (++ac == nch) {
      ac = 0;
      ++ap;
    }
  };
  const int64_t nu = u1 - u0;
  if (nu > 0) {
    CsUnit<T> xa, xb, xc;
    load_next(xa);
    if (nu > 1) load_next(xb);
    int64_t i = 0;  // units added
    for (; i + 5 <= nu; i += 3) {
      load_next(xc);
      add_next(xa);
      load_next(xa);
      add_next(xb);
      load_next(xb);
      add_next(xc);
    }
    const int64_t r = nu - i;  // 1..4 units left; xa (and xb if r > 1) loaded
    if (r == 1) {
      add_next(xa);
    } else if (r == 2) {
      add_next(xa);
      add_next(xb);
    } else if (r == 3) {
      load_next(xc);
      add_next(xa);
      add_next(xb);
      add_next(xc);
    } else {
      load_next(xc);
      add_next(xa);
      load_next(xa);
      add_next(xb);
      add_next(xc);
      add_next(xa);
    }
    T* dst = partials + (wk + cur) * plan.slot_elems + (size_t)wave * s;
    for (int i = lane; i < s; i += 64) dst[i] = my[i];
  }
}

template <typename T, bool VEC, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void countsketch_sched_kernel(
    const T* __restrict__ A, int64_t lda, const T* __restrict__ bcol, int n, PanelPlan plan,
    const uint16_t* __restrict__ table, T* __restrict__ partials) {
  cs_sched_body<T, VEC, WAVES>(A, lda, bcol, n, plan, table, partials, blockIdx.x);
}

// waves per workgroup of the scheduled kernel for sketch size s
template <typename T>
int cs_sched_waves(int64_t s) {
  int w = 8;
  while (w > 1 && (size_t)w * (s + 4) * sizeof(T) > 150 * 1024) w /= 2;
  return w;
}

template <typename T>
size_t cs_sched_lds(int64_t s, int waves) {
  return (size_t)waves * (s + 4) * sizeof(T);
}

// ---- grouped execution over a descriptor table ----------------------------------------
//
// A batch of CountSketch problems of different shapes runs as one launch per
// stage (schedule, scatter-add, reduction).  Each problem keeps exactly the
// work partition of its solo call, so its result is bitwise identical to
// rmm_sketch on it alone; the grids are the concatenation of the solo grids,
// and a workgroup finds its problem by binary search over the prefix offsets.
template <typename T>
struct CsGroupDesc {
  const T* A;
  const T* b;
  T* C;
  uint16_t* table;
  T* partials;
  int64_t lda, ldc, m;
  uint64_t seed;
  int64_t sblk0;  // first schedule window of this problem
  int64_t wk0;    // first scatter-add worker
  int64_t col0;   // first reduction column
  PanelPlan plan;
  int n;          // columns of A (the optional b column comes after)
  int vec;        // 16-byte loads allowed
};

template <typename T>
__device__ __forceinline__ int group_find(const CsGroupDesc<T>* __restrict__ d, int count,
                                          int64_t x, int which) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int64_t start = which == 0 ? d[mid].sblk0 : which == 1 ? d[mid].wk0 : d[mid].col0;
    if (start <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <typename T>
__global__ __launch_bounds__(64) void cs_schedule_group_kernel(const CsGroupDesc<T>* __restrict__ d,
                                                               int count) {
  extern __shared__ uint32_t cs_owner[];
  const int p = group_find(d, count, blockIdx.x, 0);
  cs_schedule_body(d[p].m, (uint32_t)d[p].plan.s, d[p].seed, sched_chunk<T>() / kCsWindow,
                   d[p].table, (int64_t)blockIdx.x - d[p].sblk0, cs_owner);
}

template <typename T, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void countsketch_group_kernel(
    const CsGroupDesc<T>* __restrict__ d, int count, int64_t wk_base) {
  const int64_t x = wk_base + blockIdx.x;
  const int p = group_find(d, count, x, 1);
  const CsGroupDesc<T>& g = d[p];
  const int64_t wk = x - g.wk0;
  if (g.vec)
    cs_sched_body<T, true, WAVES>(g.A, g.lda, g.b, g.n, g.plan, g.table, g.partials, wk);
  else
    cs_sched_body<T, false, WAVES>(g.A, g.lda, g.b, g.n, g.plan, g.table, g.partials, wk);
}

template <typename T>
__global__ void panel_reduce_group_kernel(const CsGroupDesc<T>* __restrict__ d, int count) {
  const int p = group_find(d, count, blockIdx.y, 2);
  const CsGroupDesc<T>& g = d[p];
  panel_reduce_body<T>(g.plan, g.partials, 1.0, g.C, g.ldc, (int64_t)blockIdx.y - g.col0);
}

namespace {

constexpr size_t kAccBudget = 128 * 1024;  // LDS bytes for the bucket accumulators

template <typename T>
int pick_unroll() {
  return sizeof(T) == 4 ? 8 : 4;
}

template <typename T>
void cs_shape(const rmm_ctx* h, int64_t m, int ncols, int s, int* waves, int* ST,
              PanelPlan* plan) {
  int st = s;
  const int max_st = (int)(kAccBudget / sizeof(T));
  if (st > max_st) st = max_st;
  int w = (int)(kAccBudget / ((size_t)st * sizeof(T)));
  if (w > 8) w = 8;
  int pw = 1;
  while (pw * 2 <= w) pw *= 2;
  while (pw > 1 && pw / 2 >= ncols) pw /= 2;
  *waves = pw;
  *ST = st;
  const int unroll = pick_unroll<T>();
  const size_t lds = (size_t)pw * st * sizeof(T) + 2 * 256 * unroll * 4;
  int per_cu = (int)(160 * 1024 / lds);
  if (per_cu < 1) per_cu = 1;
  if (per_cu > 8) per_cu = 8;
  *plan = make_plan(m, ncols, pw, s, st, 256 * unroll, h->cus * per_cu);
}

template <typename T, int WAVES, bool VEC>
int launch_cs(const rmm_ctx* h, const T* A, int64_t lda, const T* b, int n,
              const PanelPlan& plan, uint64_t seed, T* partials) {
  constexpr int UNROLL = sizeof(T) == 4 ? 8 : 4;
  const size_t lds = (size_t)WAVES * plan.ST * sizeof(T) + 2 * 256 * UNROLL * 4;
  auto kern = countsketch_kernel<T, WAVES, UNROLL, VEC>;
  RMM_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds));
  ktime_mark(h, 0);
  hipLaunchKernelGGL(kern, dim3(plan.G), dim3(WAVES * 64), lds, h->stream, A, lda, b, n, plan,
                     seed, partials);
  ktime_mark(h, 1);
  return launch_status();
}

}  // namespace

bool cs_use_sched(int64_t s, size_t tsize) {
  return s <= kCsSchedMaxS && (size_t)s * tsize <= 64 * 1024;
}

template <typename T>
PanelPlan cs_sched_plan(const rmm_ctx* h, int64_t m, int ncols, int s) {
  const int waves = cs_sched_waves<T>(s);
  const size_t lds = cs_sched_lds<T>(s, waves);
  int per_cu = (int)(160 * 1024 / lds);
  if (per_cu > 8) per_cu = 8;
  if (per_cu < 1) per_cu = 1;
  return make_plan(m, ncols, waves, s, s, sched_chunk<T>(), h->cus * per_cu);
}

template <typename T, bool VEC>
int launch_cs_sched(const rmm_ctx* h, const T* A, int64_t lda, const T* b, int n,
                    const PanelPlan& plan, const uint16_t* table, T* partials) {
  const size_t lds = cs_sched_lds<T>(plan.s, plan.width);
#define RMM_CSS_CASE(W)                                                                     \
  case W: {                                                                                 \
    auto kern = countsketch_sched_kernel<T, VEC, W>;                                        \
    RMM_HIP(hipFuncSetAttribute((const void*)kern,                                          \
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));     \
    ktime_mark(h, 0);                                                                       \
    hipLaunchKernelGGL(kern, dim3(plan.G), dim3(64 * W), lds, h->stream, A, lda, b, n, plan, \
                       table, partials);                                                    \
    ktime_mark(h, 1);                                                                       \
    return launch_status();                                                                 \
  }
  switch (plan.width) {
    RMM_CSS_CASE(1)
    RMM_CSS_CASE(2)
    RMM_CSS_CASE(4)
    RMM_CSS_CASE(8)
  }
#undef RMM_CSS_CASE
  return RMM_ERR_UNSUPPORTED;
}

template <typename T>
size_t countsketch_workspace(const rmm_ctx* h, int64_t m, int ncols, int64_t s) {
  Carver c(nullptr, 0);
  if (cs_use_sched(s, sizeof(T))) {
    const PanelPlan plan = cs_sched_plan<T>(h, m, ncols, (int)s);
    c.take<uint16_t>(cs_table_elems(m > 0 ? m : 1));
    c.take<T>((size_t)plan_slots(plan) * plan.slot_elems);
    return c.off;
  }
  int waves, ST;
  PanelPlan plan;
  cs_shape<T>(h, m, ncols, (int)s, &waves, &ST, &plan);
  c.take<T>((size_t)plan_slots(plan) * plan.slot_elems);
  return c.off;
}

template <typename T>
int countsketch_run(rmm_ctx* h, int64_t m, int n, const T* A, int64_t lda, const T* b,
                    int64_t s, uint64_t seed, T* C, int64_t ldc, Carver& ws) {
  const int ncols = n + (b ? 1 : 0);
  if (ncols == 0) return RMM_OK;
  if (m == 0) return launch_fill_zero<T>(C, s, ncols, ldc, h->stream);
  if (cs_use_sched(s, sizeof(T))) {
    const bool vecs = ((uintptr_t)A % 16 == 0) && (lda % 4 == 0) && (m % 4 == 0) &&
                      (b == nullptr || (uintptr_t)b % 16 == 0);
    const PanelPlan plan = cs_sched_plan<T>(h, m, ncols, (int)s);
    uint16_t* table = ws.take<uint16_t>(cs_table_elems(m));
    T* partials = ws.take<T>((size_t)plan_slots(plan) * plan.slot_elems);
    if (!ws.fits()) return RMM_ERR_WORKSPACE_TOO_SMALL;
    hipLaunchKernelGGL(cs_schedule_kernel, dim3((unsigned)(cs_table_rows(m) / kCsWindow)),
                       dim3(64), (size_t)s * sizeof(uint32_t), h->stream, m, (uint32_t)s, seed,
                       sched_chunk<T>() / kCsWindow, table);
    RMM_TRY(launch_status());
    const int rc = vecs ? launch_cs_sched<T, true>(h, A, lda, b, n, plan, table, partials)
                        : launch_cs_sched<T, false>(h, A, lda, b, n, plan, table, partials);
    RMM_TRY(rc);
    return launch_panel_reduce<T>(plan, partials, 1.0, C, ldc, h->stream);
  }
  int waves, ST;
  PanelPlan plan;
  cs_shape<T>(h, m, ncols, (int)s, &waves, &ST, &plan);
  T* partials = ws.take<T>((size_t)plan_slots(plan) * plan.slot_elems);
  if (!ws.fits()) return RMM_ERR_WORKSPACE_TOO_SMALL;
  const bool vec = ((uintptr_t)A % 16 == 0) && (lda % 4 == 0) &&
                   (b == nullptr || (uintptr_t)b % 16 == 0);
  int rc;
#define RMM_CS_CASE(W)                                                          \
  case W:                                                                       \
    rc = vec ? launch_cs<T, W, true>(h, A, lda, b, n, plan, seed, partials)     \
             : launch_cs<T, W, false>(h, A, lda, b, n, plan, seed, partials);   \
    break;
  switch (waves) {
    RMM_CS_CASE(1)
    RMM_CS_CASE(2)
    RMM_CS_CASE(4)
    RMM_CS_CASE(8)
    default:
      return RMM_ERR_UNSUPPORTED;
  }
#undef RMM_CS_CASE
  RMM_TRY(rc);
  return launch_panel_reduce<T>(plan, partials, 1.0, C, ldc, h->stream);
}

// ---- batch: host side ------------------------------------------------------------------

namespace {

// carve the per-problem buffers and fill the descriptor table (ws may have a
// null base: size query)
template <typename T>
int cs_batch_layout(const rmm_ctx* h, int count, const rmm_sketch_desc* d, Carver& ws,
                    std::vector<CsGroupDesc<T>>* out, int64_t* nsblk, int64_t* nwk, int64_t* ncol,
                    int* max_s) {
  int64_t sb = 0, wk = 0, col = 0;
  int ms = 1;
  // problems of equal workgroup width are contiguous (one launch per width)
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return cs_sched_waves<T>(d[a].s) > cs_sched_waves<T>(d[b].s);
  });
  for (int i : order) {
    const int ncols = (int)d[i].n + (d[i].b ? 1 : 0);
    if (d[i].m == 0 || ncols == 0) continue;
    const int s = (int)d[i].s;
    const PanelPlan plan = cs_sched_plan<T>(h, d[i].m, ncols, s);
    uint16_t* table = ws.take<uint16_t>(cs_table_elems(d[i].m));
    T* partials = ws.take<T>((size_t)plan_slots(plan) * plan.slot_elems);
    if (out) {
      CsGroupDesc<T> g{};
      g.A = (const T*)d[i].A;
      g.b = (const T*)d[i].b;
      g.C = (T*)d[i].C;
      g.table = table;
      g.partials = partials;
      g.lda = d[i].lda;
      g.ldc = d[i].ldc;
      g.m = d[i].m;
      g.seed = d[i].seed;
      g.sblk0 = sb;
      g.wk0 = wk;
      g.col0 = col;
      g.plan = plan;
      g.n = (int)d[i].n;
      g.vec = ((uintptr_t)d[i].A % 16 == 0) && (d[i].lda % 4 == 0) && (d[i].m % 4 == 0) &&
              (d[i].b == nullptr || (uintptr_t)d[i].b % 16 == 0);
      out->push_back(g);
    }
    sb += cs_table_rows(d[i].m) / kCsWindow;
    wk += plan.G;
    col += ncols;
    if (s > ms) ms = s;
  }
  *nsblk = sb;
  *nwk = wk;
  *ncol = col;
  *max_s = ms;
  return RMM_OK;
}

}  // namespace

template <typename T>
bool countsketch_batch_grouped(int count, const rmm_sketch_desc* d) {
  for (int i = 0; i < count; ++i)
    if (!cs_use_sched(d[i].s, sizeof(T))) return false;
  return true;
}

template <typename T>
size_t countsketch_batch_workspace(const rmm_ctx* h, int count, const rmm_sketch_desc* d) {
  Carver c(nullptr, 0);
  int64_t a, b, e;
  int ms;
  cs_batch_layout<T>(h, count, d, c, nullptr, &a, &b, &e, &ms);
  c.take<CsGroupDesc<T>>((size_t)count + 1);
  return c.off;
}

template <typename T>
int countsketch_batch_run(rmm_ctx* h, int count, const rmm_sketch_desc* d, Carver& ws) {
  std::vector<CsGroupDesc<T>> g;
  g.reserve(count);
  int64_t nsblk, nwk, ncol;
  int ms;
  RMM_TRY(cs_batch_layout<T>(h, count, d, ws, &g, &nsblk, &nwk, &ncol, &ms));
  CsGroupDesc<T>* dd = ws.take<CsGroupDesc<T>>((size_t)count + 1);
  if (!ws.fits()) return RMM_ERR_WORKSPACE_TOO_SMALL;
  for (int i = 0; i < count; ++i) {
    const int ncols = (int)d[i].n + (d[i].b ? 1 : 0);
    if (d[i].m == 0 && ncols > 0)
      RMM_TRY(launch_fill_zero<T>((T*)d[i].C, d[i].s, ncols, d[i].ldc, h->stream));
  }
  const int gc = (int)g.size();
  if (gc == 0) return RMM_OK;
  // the table is staged in the handle so the host bytes outlive the async copy
  h->table_host.resize(sizeof(CsGroupDesc<T>) * gc);
  std::memcpy(h->table_host.data(), g.data(), h->table_host.size());
  RMM_HIP(hipMemcpyAsync(dd, h->table_host.data(), h->table_host.size(), hipMemcpyHostToDevice,
                         h->stream));
  hipLaunchKernelGGL(cs_schedule_group_kernel<T>, dim3((unsigned)nsblk), dim3(64),
                     (size_t)ms * sizeof(uint32_t), h->stream, dd, gc);
  RMM_TRY(launch_status());
  // one scatter-add launch per workgroup width; problems of the same width
  // are contiguous in the table (sorted by width on the host)
  int i0 = 0;
  while (i0 < gc) {
    const int w = g[i0].plan.width;
    int i1 = i0;
    int s_max = 1;
    while (i1 < gc && g[i1].plan.width == w) {
      if (g[i1].plan.s > s_max) s_max = g[i1].plan.s;
      ++i1;
    }
    const int64_t wk_lo = g[i0].wk0;
    const int64_t wk_hi = (i1 < gc) ? g[i1].wk0 : nwk;
    const size_t lds = cs_sched_lds<T>(s_max, w);
#define RMM_CSG_CASE(W)                                                                       \
  case W: {                                                                                   \
    RMM_HIP(hipFuncSetAttribute((const void*)countsketch_group_kernel<T, W>,                  \
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));       \
    hipLaunchKernelGGL((countsketch_group_kernel<T, W>), dim3((unsigned)(wk_hi - wk_lo)),      \
                       dim3(64 * W), lds, h->stream, dd + i0, i1 - i0, wk_lo);                \
    break;                                                                                    \
  }
    switch (w) {
      RMM_CSG_CASE(1)
      RMM_CSG_CASE(2)
      RMM_CSG_CASE(4)
      RMM_CSG_CASE(8)
      default:
        return RMM_ERR_UNSUPPORTED;
    }
#undef RMM_CSG_CASE
    RMM_TRY(launch_status());
    i0 = i1;
  }
  hipLaunchKernelGGL(panel_reduce_group_kernel<T>, dim3((unsigned)((ms + 255) / 256), (unsigned)ncol),
                     dim3(256), 0, h->stream, dd, gc);
  return launch_status();
}

// ---- column count sketch C = A S (the first step of the faster k-SVD) --------------
//
// S is an n x s count sketch of the columns of A: column j of A goes, with
// sign g_j, into column h_j of C (the words of the count-sketch stream for
// index j).  A gather instead of a scatter: workgroup (row chunk, bucket c)
// lists the columns of bucket c in increasing j, 2048 at a time (wave
// ballots, one barrier per round), then sums them for its 4096 rows, 16 per
// thread in registers, with 16-byte loads when the columns allow them.  Every
// entry of C is a fixed-order sum, and A is read once.
constexpr int kColRows = 16;               // rows per thread
constexpr int kColChunk = 256 * kColRows;  // rows per workgroup
constexpr int kColSeg = 8;                 // columns scanned per thread per segment

__global__ void colcs_hash_kernel(int64_t n, uint32_t s, uint64_t seed, uint32_t* __restrict__ hs) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const uint32_t w = cs_word((uint64_t)j, seed);
  hs[j] = cs_bucket(w, s) | ((w & 1u) << 31);
}

template <typename T, bool VEC>
__global__ __launch_bounds__(256) void colcs_kernel(int64_t m, int64_t n, const T* __restrict__ A,
                                                    int64_t lda, const uint32_t* __restrict__ hs,
                                                    T* __restrict__ C, int64_t ldc) {
  __shared__ int32_t list[256 * kColSeg];
  __shared__ int32_t wcount[4];
  __shared__ int32_t total;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t c = blockIdx.y;
  const int64_t r0 = (int64_t)blockIdx.x * kColChunk;
  T acc[4][4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[q][e] = T(0);
  for (int64_t seg = 0; seg < n; seg += 256 * kColSeg) {
    if (tid == 0) total = 0;
    __syncthreads();
#pragma unroll 1
    for (int i = 0; i < kColSeg; ++i) {
      const int64_t j = seg + (int64_t)i * 256 + tid;
      const uint32_t w = j < n ? hs[j] : 0xFFFFFFFFu;
      const bool hit = j < n && (w & 0x7FFFFFFFu) == c;
      const uint64_t bal = __ballot(hit);
      if (lane == 0) wcount[wave] = __popcll(bal);
      __syncthreads();
      int off = total;
      for (int v = 0; v < wave; ++v) off += wcount[v];
      if (hit) {
        const int pos = off + __popcll(bal & ((1ull << lane) - 1ull));
        list[pos] = (int32_t)((j - seg) | ((w >> 31) << 30));
      }
      __syncthreads();
      if (tid == 0) total += wcount[0] + wcount[1] + wcount[2] + wcount[3];
      __syncthreads();
    }
    const int cnt = total;
    for (int t = 0; t < cnt; ++t) {
      const int32_t ent = list[t];
      const int64_t j = seg + (ent & 0x3FFFFFFF);
      const T sg = (ent >> 30) & 1 ? T(-1) : T(1);
      const T* col = A + j * lda;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t r = r0 + q * 1024 + 4 * tid;
        if (VEC) {
          if (r < m) {
            if constexpr (sizeof(T) == 4) {
              const float4 x = ld_stream(reinterpret_cast<const float4*>(col + r));
              acc[q][0] += sg * x.x; acc[q][1] += sg * x.y; acc[q][2] += sg * x.z; acc[q][3] += sg * x.w;
            } else {
              const double2 x = ld_stream(reinterpret_cast<const double2*>(col + r));
              const double2 y = ld_stream(reinterpret_cast<const double2*>(col + r + 2));
              acc[q][0] += sg * x.x; acc[q][1] += sg * x.y; acc[q][2] += sg * y.x; acc[q][3] += sg * y.y;
            }
          }
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (r + e < m) acc[q][e] += sg * col[r + e];
        }
      }
    }
    __syncthreads();  // the list is rewritten by the next segment
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t r = r0 + q * 1024 + 4 * tid + e;
      if (r < m) C[r + (int64_t)c * ldc] = acc[q][e];
    }
}

size_t countsketch_cols_workspace(int64_t n) {
  Carver c(nullptr, 0);
  c.take<uint32_t>((size_t)(n > 0 ? n : 1));
  return c.off + kAlign;
}

template <typename T>
int countsketch_cols_run(rmm_ctx* h, int64_t m, int64_t n, const T* A, int64_t lda, int64_t s,
                         uint64_t seed, T* C, int64_t ldc, Carver& ws) {
  if (m == 0 || s == 0) return RMM_OK;
  if (n == 0) return launch_fill_zero<T>(C, m, s, ldc, h->stream);
  const size_t mark = ws.off;
  uint32_t* hs = ws.take<uint32_t>((size_t)n);
  if (!ws.fits()) return RMM_ERR_WORKSPACE_TOO_SMALL;
  hipLaunchKernelGGL(colcs_hash_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, h->stream, n,
                     (uint32_t)s, seed, hs);
  RMM_TRY(launch_status());
  const bool vec = (uintptr_t)A % 16 == 0 && lda % 4 == 0 && m % 4 == 0;
  dim3 grid((unsigned)((m + kColChunk - 1) / kColChunk), (unsigned)s);
  if (vec)
    hipLaunchKernelGGL((colcs_kernel<T, true>), grid, dim3(256), 0, h->stream, m, n, A, lda, hs, C, ldc);
  else
    hipLaunchKernelGGL((colcs_kernel<T, false>), grid, dim3(256), 0, h->stream, m, n, A, lda, hs, C, ldc);
  ws.off = mark;
  return launch_status();
}

template int countsketch_cols_run<float>(rmm_ctx*, int64_t, int64_t, const float*, int64_t, int64_t,
                                         uint64_t, float*, int64_t, Carver&);
template int countsketch_cols_run<double>(rmm_ctx*, int64_t, int64_t, const double*, int64_t,
                                          int64_t, uint64_t, double*, int64_t, Carver&);

template bool countsketch_batch_grouped<float>(int, const rmm_sketch_desc*);
template bool countsketch_batch_grouped<double>(int, const rmm_sketch_desc*);
template size_t countsketch_batch_workspace<float>(const rmm_ctx*, int, const rmm_sketch_desc*);
template size_t countsketch_batch_workspace<double>(const rmm_ctx*, int, const rmm_sketch_desc*);
template int countsketch_batch_run<float>(rmm_ctx*, int, const rmm_sketch_desc*, Carver&);
template int countsketch_batch_run<double>(rmm_ctx*, int, const rmm_sketch_desc*, Carver&);

template size_t countsketch_workspace<float>(const rmm_ctx*, int64_t, int, int64_t);
template size_t countsketch_workspace<double>(const rmm_ctx*, int64_t, int, int64_t);
template int countsketch_run<float>(rmm_ctx*, int64_t, int, const float*, int64_t, const float*,
                                    int64_t, uint64_t, float*, int64_t, Carver&);
template int countsketch_run<double>(rmm_ctx*, int64_t, int, const double*, int64_t,
                                     const double*, int64_t, uint64_t, double*, int64_t,
                                     Carver&);

}  // namespace rmm
