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

// ---------------------------------------------------------------- machine probes
// Streaming ceiling: mode 0 copies (dst = src + 1: n doubles read, n
// written), mode 1 only reads (per-workgroup sums into dst[blockIdx.x]),
// mode 2 copies with non-temporal loads and stores.  Four loads in flight
// per lane, grid-stride over 8-byte elements.
__global__ __launch_bounds__(256) void k_probe_stream(const double *__restrict__ src,
                                                      double *__restrict__ dst, int64_t n,
                                                      int mode) {
  const int64_t nthr = static_cast<int64_t>(gridDim.x) * 256;
  double acc = 0.0;
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; base < n;
       base += 4 * nthr) {
    double v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t i = base + q * nthr;
      v[q] = i < n ? (mode == 2 ? __builtin_nontemporal_load(src + i) : src[i]) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t i = base + q * nthr;
      if (mode == 0) {
        if (i < n) dst[i] = v[q] + 1.0;
      } else if (mode == 2) {
        if (i < n) __builtin_nontemporal_store(v[q] + 1.0, dst + i);
      } else {
        acc += v[q];
      }
    }
  }
  if (mode == 1) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
    __shared__ double part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) dst[blockIdx.x] = (part[0] + part[1]) + (part[2] + part[3]);
  }
}

// FP64 FMA ceiling: 8 independent chains of `iters` fmas per lane (2 flops
// each); one result per lane is stored so nothing is dead.
__global__ __launch_bounds__(256) void k_probe_fma(double *__restrict__ out, int iters) {
  double a[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) a[k] = 1.0 + 1e-3 * (threadIdx.x + k);
  const double b = 0.999999, c = 1e-7;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = fma(a[k], b, c);
  }
  double r = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) r += a[k];
  out[static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x] = r;
}

hipError_t launch_probe_stream(const double *src, double *dst, int64_t n, int mode, int grid,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_probe_stream, dim3(grid), dim3(256), 0, st, src, dst, n, mode);
  return hipGetLastError();
}

hipError_t launch_probe_fma(double *out, int iters, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_probe_fma, dim3(grid), dim3(256), 0, st, out, iters);
  return hipGetLastError();
}

}  // namespace trk
