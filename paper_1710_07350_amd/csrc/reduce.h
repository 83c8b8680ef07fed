// reduce.h -- deterministic block reductions for 256-thread blocks.
//
// Sums use a fixed butterfly inside each 64-lane wavefront (xor 32, 16, ...,
// 1), then the four wave totals are added in wave order, so a result depends
// only on the data and the block size, never on scheduling.  Min/max are
// exact and order-free.
#pragma once
#include <hip/hip_runtime.h>

#include "trk_internal.h"

namespace trk {

constexpr int kWaves = kBlock / 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Block totals of v[0..N); returns a shared array holding them (valid for all
// threads until the next call).
template <int N>
__device__ __forceinline__ const double *block_sum(double (&v)[N]) {
  __shared__ double part[kWaves][N];
  __shared__ double tot[N];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) part[wave][k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x < N) {
    double s = part[0][threadIdx.x];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) s += part[w][threadIdx.x];
    tot[threadIdx.x] = s;
  }
  __syncthreads();
  return tot;
}

// Block totals of (w, d_k, d_k d_l for k <= l), written to row[0..28).  The
// 28 components are reduced one at a time so that only d stays live.
__device__ __forceinline__ void block_moment_row(double w, const double (&d)[6], double *row) {
  __shared__ double part[kWaves][28];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll 1
  for (int c = 0; c < 28; ++c) {
    double v;
    if (c == 0) {
      v = w;
    } else if (c < 7) {
      v = d[0];
#pragma unroll
      for (int k = 1; k < 6; ++k)
        if (c - 1 == k) v = d[k];
    } else {
      // c -> (k, l), k <= l, row-major upper triangle
      int k = 0, r = c - 7;
      while (r >= 6 - k) {
        r -= 6 - k;
        ++k;
      }
      const int l = k + r;
      double dk = d[0], dl = d[0];
#pragma unroll
      for (int q = 1; q < 6; ++q) {
        if (q == k) dk = d[q];
        if (q == l) dl = d[q];
      }
      v = dk * dl;
    }
    v = wave_sum(v);
    if (lane == 0) part[wave][c] = v;
  }
  __syncthreads();
  if (threadIdx.x < 28) {
    double s = part[0][threadIdx.x];
#pragma unroll
    for (int w2 = 1; w2 < kWaves; ++w2) s += part[w2][threadIdx.x];
    row[threadIdx.x] = s;
  }
  __syncthreads();
}

// As block_moment_row for kP particles per thread: (count, sum z_k,
// sum z_k z_l) over the alive ones, written to row[0..28).
template <int kP>
__device__ __forceinline__ void block_moment_row_multi(const bool (&al)[kP],
                                                       const double (&z)[kP][6], double *row) {
  __shared__ double part[kWaves][28];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll 1
  for (int c = 0; c < 28; ++c) {
    int k = 0, l = 0;
    if (c >= 1 && c < 7) {
      k = c - 1;
    } else if (c >= 7) {
      int r = c - 7;
      while (r >= 6 - k) {
        r -= 6 - k;
        ++k;
      }
      l = k + r;
    }
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < kP; ++q) {
      double zk = z[q][0], zl = z[q][0];
#pragma unroll
      for (int j = 1; j < 6; ++j) {
        if (j == k) zk = z[q][j];
        if (j == l) zl = z[q][j];
      }
      const double term = c == 0 ? 1.0 : (c < 7 ? zk : zk * zl);
      if (al[q]) v += term;
    }
    v = wave_sum(v);
    if (lane == 0) part[wave][c] = v;
  }
  __syncthreads();
  if (threadIdx.x < 28) {
    double s = part[0][threadIdx.x];
#pragma unroll
    for (int w2 = 1; w2 < kWaves; ++w2) s += part[w2][threadIdx.x];
    row[threadIdx.x] = s;
  }
  __syncthreads();
}

__device__ __forceinline__ void block_minmax(double &mn, double &mx) {
  __shared__ double pm[kWaves][2];
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    mn = fmin(mn, __shfl_xor(mn, m, 64));
    mx = fmax(mx, __shfl_xor(mx, m, 64));
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    pm[wave][0] = mn;
    pm[wave][1] = mx;
  }
  __syncthreads();
  mn = pm[0][0];
  mx = pm[0][1];
#pragma unroll
  for (int w = 1; w < kWaves; ++w) {
    mn = fmin(mn, pm[w][0]);
    mx = fmax(mx, pm[w][1]);
  }
  __syncthreads();
}

// exclusive block scan of a per-thread integer count; returns the block total
__device__ __forceinline__ int block_exclusive_scan(int v, int &total) {
  __shared__ int wsum[kWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int incl = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int t = __shfl_up(incl, d, 64);
    if (lane >= d) incl += t;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  int off = 0;
  total = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    if (w < wave) off += wsum[w];
    total += wsum[w];
  }
  __syncthreads();
  return off + incl - v;
}

}  // namespace trk
