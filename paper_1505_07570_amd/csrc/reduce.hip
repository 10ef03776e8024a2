// Fixed-order reduction of per-worker partial sketches, and small fills.
//
// Partial slot (worker w, panel p) holds width x ST values laid out
// [column-in-panel][bucket-in-tile].  Every output element sums the slots of
// the contiguous run of workers that touched its panel, in increasing worker
// order and in fp64, so the result does not depend on scheduling.
#include "common.hpp"

namespace rmm {

PanelPlan make_plan(int64_t m, int ncols, int width, int s, int ST, int64_t chunk, int G) {
  PanelPlan p{};
  p.m = m;
  p.chunk = chunk;
  p.nchunks = m > 0 ? (m + chunk - 1) / chunk : 0;
  p.ncols = ncols;
  p.width = width;
  p.P = (ncols + width - 1) / width;
  p.s = s;
  p.ST = ST;
  p.BT = (s + ST - 1) / ST;
  p.units = (int64_t)p.P * p.BT * p.nchunks;
  int64_t g = G;
  if (g > p.units) g = p.units;
  if (g < 1) g = 1;
  p.G = (int)g;
  p.slot_elems = width * ST;
  return p;
}

template <typename T>
__global__ void panel_reduce_kernel(PanelPlan plan, const T* __restrict__ partials,
                                    double scale, T* __restrict__ C, int64_t ldc) {
  panel_reduce_body<T>(plan, partials, scale, C, ldc, blockIdx.y);
}

template <typename T>
int launch_panel_reduce(const PanelPlan& plan, const T* partials, double scale, T* C,
                        int64_t ldc, hipStream_t st) {
  if (plan.ncols == 0 || plan.s == 0) return RMM_OK;
  dim3 grid((unsigned)((plan.s + 255) / 256), (unsigned)plan.ncols);
  hipLaunchKernelGGL(panel_reduce_kernel<T>, grid, dim3(256), 0, st, plan, partials, scale, C,
                     ldc);
  return launch_status();
}

template <typename T>
__global__ void fill_zero_kernel(T* __restrict__ C, int64_t rows, int64_t ldc) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < rows) C[r + (int64_t)blockIdx.y * ldc] = T(0);
}

template <typename T>
int launch_fill_zero(T* C, int64_t rows, int64_t cols, int64_t ldc, hipStream_t st) {
  if (rows == 0 || cols == 0) return RMM_OK;
  dim3 grid((unsigned)((rows + 255) / 256), (unsigned)cols);
  hipLaunchKernelGGL(fill_zero_kernel<T>, grid, dim3(256), 0, st, C, rows, ldc);
  return launch_status();
}

template int launch_panel_reduce<float>(const PanelPlan&, const float*, double, float*, int64_t,
                                        hipStream_t);
template int launch_panel_reduce<double>(const PanelPlan&, const double*, double, double*,
                                         int64_t, hipStream_t);
template int launch_fill_zero<float>(float*, int64_t, int64_t, int64_t, hipStream_t);
template int launch_fill_zero<double>(double*, int64_t, int64_t, int64_t, hipStream_t);

}  // namespace rmm
