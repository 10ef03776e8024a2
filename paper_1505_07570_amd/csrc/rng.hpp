// Counter-based random numbers on the device.
//
// Every random quantity used by the sketches is a pure function of
// (seed, stream tag, index), so any thread can produce any entry of S in
// registers.  Generator: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11),
// key = (lo32(seed), hi32(seed)), counter = (lo32(i), hi32(i), tag, j).
//
//  CountSketch (Alg. 3.1)      w = philox(i>>2, TAG_COUNTSKETCH, 0)[i&3];
//                              bucket = (w * s) >> 32, sign = -1 if w odd
//  SRHT diagonal (Sec. 3.2.2)  d_i = bit (i & 127) of the 128-bit block
//                              philox(i>>7, TAG_SRHT_SIGN, 0); bit b lives in
//                              word b>>5 at position b&31; set bit = -1
//  Row sampling                6-round Feistel bijection of [0, 2^k),
//                              F_r(v) = philox(v, tag, r)[0], cycle walking
//                              for domains that are not powers of two
//  Gaussians (Sec. 3.2.1)      Box-Muller; fp32: philox(i, tag, q) gives
//                              entries (i, 4q..4q+3); fp64: entries
//                              (i, 2q), (i, 2q+1) from 53-bit uniforms
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rmm {

enum : uint32_t {
  TAG_COUNTSKETCH = 1,
  TAG_SRHT_SIGN = 2,
  TAG_SRHT_SAMPLE = 3,
  TAG_GAUSS_SKETCH = 4,
  TAG_GAUSS_RSVD = 5,
  TAG_NYSTROM_SAMPLE = 6,
  TAG_GAUSS_NYSTROM = 7,
  TAG_SPSD_SAMPLE = 8,
  TAG_LEVERAGE = 9,
  TAG_CUR_COLS = 10,
  TAG_CUR_ROWS = 11,
  TAG_CUR_PC = 12,
  TAG_CUR_PR = 13,
};

struct Words4 {
  uint32_t w[4];
};

__host__ __device__ __forceinline__ Words4 philox(uint32_t c0, uint32_t c1,
                                                  uint32_t c2, uint32_t c3,
                                                  uint64_t seed) {
  uint32_t k0 = (uint32_t)seed;
  uint32_t k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // both halves of each 64-bit product come from one v_mad_u64_u32
    const uint64_t pa = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t pb = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    c0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
    c1 = (uint32_t)pb;
    c2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
    c3 = (uint32_t)pa;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  Words4 o;
  o.w[0] = c0;
  o.w[1] = c1;
  o.w[2] = c2;
  o.w[3] = c3;
  return o;
}

__host__ __device__ __forceinline__ Words4 philox_at(uint64_t i, uint32_t tag,
                                                     uint32_t j, uint64_t seed) {
  return philox((uint32_t)i, (uint32_t)(i >> 32), tag, j, seed);
}

// CountSketch word of row i.
__host__ __device__ __forceinline__ uint32_t cs_word(uint64_t i, uint64_t seed) {
  Words4 b = philox_at(i >> 2, TAG_COUNTSKETCH, 0, seed);
  return b.w[i & 3];
}

__host__ __device__ __forceinline__ uint32_t cs_bucket(uint32_t w, uint32_t s) {
  return (uint32_t)(((uint64_t)w * (uint64_t)s) >> 32);
}

// SRHT sign bit (1 means -1) of row i.
__host__ __device__ __forceinline__ uint32_t srht_sign_bit(uint64_t i, uint64_t seed) {
  Words4 b = philox_at(i >> 7, TAG_SRHT_SIGN, 0, seed);
  const uint32_t bit = (uint32_t)(i & 127);
  return (b.w[bit >> 5] >> (bit & 31)) & 1u;
}

// Keyed Feistel bijection of [0, 2^k).
__host__ __device__ __forceinline__ uint64_t feistel(uint64_t x, int k, uint32_t tag,
                                                     uint64_t seed) {
  const int a = k >> 1;
  const int b = k - a;
  const uint64_t lo_mask = (a >= 64) ? ~0ull : ((1ull << a) - 1);
  const uint64_t hi_mask = (b >= 64) ? ~0ull : ((1ull << b) - 1);
  uint64_t hi = (a >= 64) ? 0 : (x >> a);
  uint64_t lo = x & lo_mask;
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    if ((r & 1) == 0) {
      hi ^= (uint64_t)philox_at(lo, tag, (uint32_t)r, seed).w[0] & hi_mask;
    } else {
      lo ^= (uint64_t)philox_at(hi, tag, (uint32_t)r, seed).w[0] & lo_mask;
    }
  }
  return (hi << a) | lo;
}

// Bijection of [0, n) by cycle walking; k = ceil(log2 n).  The walk from
// x < n returns to [0, n) within at most 2^k steps because the Feistel map
// is a permutation whose cycle through x contains x itself.
__host__ __device__ __forceinline__ uint64_t permute_domain(uint64_t x, uint64_t n, int k,
                                                            uint32_t tag, uint64_t seed) {
  uint64_t y = feistel(x, k, tag, seed);
  const uint64_t limit = 1ull << k;
  for (uint64_t step = 0; y >= n && step < limit; ++step) y = feistel(y, k, tag, seed);
  return y;
}

__host__ __device__ __forceinline__ int ceil_log2(uint64_t n) {
  int k = 0;
  while ((1ull << k) < n) ++k;
  return k;
}

// Four fp32 normals: entries (i, 4q .. 4q+3) of the Gaussian stream `tag`.
// Transcendentals use the hardware units: v_log_f32 (log2), v_sqrt_f32 and
// v_sin/v_cos_f32, which take their argument in revolutions.
__device__ __forceinline__ void gauss4_f32(uint64_t i, uint32_t q, uint32_t tag,
                                           uint64_t seed, float z[4]) {
  Words4 b = philox_at(i, tag, q, seed);
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const float u = (float)((b.w[2 * p] >> 8) + 1u) * 0x1p-24f;   // (0, 1]
    const float v = (float)(b.w[2 * p + 1] >> 8) * 0x1p-24f;      // [0, 1)
    // -2 ln u = -2 ln2 * log2 u
    const float r = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u));
    z[2 * p] = r * __builtin_amdgcn_cosf(v);
    z[2 * p + 1] = r * __builtin_amdgcn_sinf(v);
  }
}

// Two fp64 normals: entries (i, 2q), (i, 2q+1).
__device__ __forceinline__ void gauss2_f64(uint64_t i, uint32_t q, uint32_t tag,
                                           uint64_t seed, double z[2]) {
  Words4 b = philox_at(i, tag, q, seed);
  const uint64_t iu = (((uint64_t)b.w[0] << 21) | (b.w[1] >> 11)) + 1ull;
  const uint64_t iv = ((uint64_t)b.w[2] << 21) | (b.w[3] >> 11);
  const double u = (double)iu * 0x1p-53;
  const double v = (double)iv * 0x1p-53;
  const double r = sqrt(-2.0 * log(u));
  double sn, cs;
  sincospi(2.0 * v, &sn, &cs);
  z[0] = r * cs;
  z[1] = r * sn;
}

}  // namespace rmm
