// testhooks.hip -- device-side probes of the arithmetic the kernels rely on
// (own elementary functions, binary64 sqrt and division, Philox, normals),
// so their bit patterns can be compared with a CPU implementation.
#include "devmath.h"
#include "trk_internal.h"

namespace trk {

__global__ void k_elementary(int fn, const double *__restrict__ x, const double *__restrict__ y,
                             double *__restrict__ out, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double a = x[i];
    double r;
    switch (fn) {
      case 0: r = dm::own_sin(a); break;
      case 1: r = dm::own_cos(a); break;
      case 2: r = dm::own_log(a); break;
      case 3: r = dm::own_exp(a); break;
      case 4: r = sqrt(a); break;
      default: r = a / y[i]; break;
    }
    out[i] = r;
  }
}

__global__ void k_philox(const uint32_t *__restrict__ ctr, const uint32_t *__restrict__ key,
                         uint32_t *__restrict__ out, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    dm::U4 c;
    for (int k = 0; k < 4; ++k) c.v[k] = ctr[4 * i + k];
    const dm::U4 o = dm::philox4x32_10(c, key[2 * i], key[2 * i + 1]);
    for (int k = 0; k < 4; ++k) out[4 * i + k] = o.v[k];
  }
}

__global__ void k_gauss(const uint32_t *__restrict__ id, uint32_t step, uint32_t tag, uint32_t klo,
                        uint32_t khi, double *__restrict__ out, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    out[i] = dm::gauss(id[i], step, tag, klo, khi);
}

static int grid_for(int64_t n) {
  const int64_t g = (n + 255) / 256;
  return static_cast<int>(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

hipError_t launch_elementary(int fn, const double *x, const double *y, double *out, int64_t n,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_elementary, dim3(grid_for(n)), dim3(256), 0, st, fn, x, y, out, n);
  return hipGetLastError();
}

hipError_t launch_philox(const uint32_t *ctr, const uint32_t *key, uint32_t *out, int64_t n,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_philox, dim3(grid_for(n)), dim3(256), 0, st, ctr, key, out, n);
  return hipGetLastError();
}

hipError_t launch_gauss(const uint32_t *id, uint32_t step, uint32_t tag, uint64_t seed,
                        double *out, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_gauss, dim3(grid_for(n)), dim3(256), 0, st, id, step, tag,
                     static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32), out, n);
  return hipGetLastError();
}

}  // namespace trk
