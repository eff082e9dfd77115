// amr_stream.hip - the streaming ceiling the stage kernels are measured against
// (amr_stream_ceiling in include/amr_hydro.h): out = (a + b) / 2 over n doubles, the
// HBM access pattern of the second RK stage (two arrays read and one written, each
// element once), with nothing else in the kernel.  Each lane moves 16-byte vectors,
// four per array per iteration, so that many loads are in flight per wavefront.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "../../include/amr_hydro.h"

namespace {

constexpr int NT = 256;
constexpr int UNROLL = 4;

__global__ __launch_bounds__(NT) void stream_avg(const double2* __restrict__ a, const double2* __restrict__ b,
                                                 double2* __restrict__ o, int64_t n2) {
  const int64_t step = (int64_t)gridDim.x * NT * UNROLL;
  for (int64_t base = (int64_t)blockIdx.x * NT * UNROLL + threadIdx.x; base < n2; base += step) {
    double2 x[UNROLL], y[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      const int64_t i = base + (int64_t)u * NT;
      if (i < n2) {
        x[u] = a[i];
        y[u] = b[i];
      }
    }
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      const int64_t i = base + (int64_t)u * NT;
      if (i < n2) o[i] = make_double2(0.5 * (x[u].x + y[u].x), 0.5 * (x[u].y + y[u].y));
    }
  }
}

__global__ void stream_tail(const double* a, const double* b, double* o, int64_t i) {
  if (threadIdx.x == 0 && blockIdx.x == 0) o[i] = 0.5 * (a[i] + b[i]);
}

}  // namespace

extern "C" amr_status amr_stream_ceiling(const double* a, const double* b, double* out, int64_t n,
                                         int32_t wg_per_cu, hipStream_t stream) {
  if (!a || !b || !out || n < 1 || wg_per_cu < 0 || wg_per_cu > 64) return AMR_EINVAL;
  if (((uintptr_t)a | (uintptr_t)b | (uintptr_t)out) & 15) return AMR_EINVAL;
  const int64_t n2 = n / 2;
  if (n2 > 0) {
    const int64_t full = (n2 + (int64_t)NT * UNROLL - 1) / ((int64_t)NT * UNROLL);
    int64_t grid = full;
    if (wg_per_cu > 0) {
      int dev = 0, ncu = 0;
      if (hipGetDevice(&dev) != hipSuccess ||
          hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return AMR_EHIP;
      grid = std::min<int64_t>(full, (int64_t)wg_per_cu * ncu);
    }
    if (grid > 0x7fffffff) grid = 0x7fffffff;
    hipLaunchKernelGGL(stream_avg, dim3((unsigned)grid), dim3(NT), 0, stream, reinterpret_cast<const double2*>(a),
                       reinterpret_cast<const double2*>(b), reinterpret_cast<double2*>(out), n2);
    if (hipGetLastError() != hipSuccess) return AMR_EHIP;
  }
  if (n & 1) {
    hipLaunchKernelGGL(stream_tail, dim3(1), dim3(64), 0, stream, a, b, out, n - 1);
    if (hipGetLastError() != hipSuccess) return AMR_EHIP;
  }
  return AMR_OK;
}
