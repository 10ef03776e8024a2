// Streaming-read reference: reads a device buffer once with 16-byte
// nontemporal loads, sixteen in flight per lane, one contiguous range per workgroup, and writes
// one float per workgroup (so the loads cannot be dropped).  It is what every
// HBM-bound pass of the library does with A, minus all arithmetic: its rate
// is the practical read ceiling against which those passes are judged, next
// to the rated peak.
#include "common.hpp"

namespace rmm {
namespace {

constexpr int kProbeGroups = 4096;
constexpr int kProbeUnroll = 16;

__global__ __launch_bounds__(256) void stream_read_kernel(const float4* __restrict__ x, int64_t n4,
                                                          float* __restrict__ sink) {
  const int64_t per = (n4 + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = (int64_t)blockIdx.x * per;
  const int64_t b1 = b0 + per < n4 ? b0 + per : n4;
  float acc = 0.f;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += 256 * kProbeUnroll) {
    float4 v[kProbeUnroll];
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) {
      const int64_t j = i + 256 * u;
      v[u] = j < b1 ? ld_stream(x + j) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
  }
  __shared__ float red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) sink[blockIdx.x] = red[0];
}

}  // namespace
}  // namespace rmm

using namespace rmm;

extern "C" int rmm_stream_read(rmm_handle h, const void* x, int64_t bytes, float* sink) {
  if (!h || !x || !sink || bytes < 16 || bytes % 16 != 0 || (uintptr_t)x % 16 != 0) return RMM_ERR_INVALID_ARG;
  const int64_t n4 = bytes / 16;
  hipLaunchKernelGGL(stream_read_kernel, dim3(kProbeGroups), dim3(256), 0, h->stream,
                     reinterpret_cast<const float4*>(x), n4, sink);
  return launch_status();
}
