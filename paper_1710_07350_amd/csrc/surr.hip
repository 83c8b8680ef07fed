// surr.hip -- particle-side kernels of the section surrogate: the admission
// gate with a stable split into admitted and rejected index lists, the
// gathers and scatters around the plain-tracking fallback, the training
// pairs, the residual scale reduction and the rejection sampler of the
// training inputs.  Every list keeps the particles' order (block counts,
// one scan, in-block ranks), so results never depend on scheduling.
#include "reduce.h"
#include "surrdev.h"

namespace trk {

namespace {

__device__ __forceinline__ void load6(const BeamPtrs6 &b, int64_t i, double (&z)[6]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) z[k] = b.z[k][i];
}

// exclusive scan over 1024 threads (int64)
__device__ __forceinline__ int64_t scan1024(int64_t v, int64_t &total) {
  __shared__ int64_t ws[16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t incl = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int64_t t = __shfl_up(incl, d, 64);
    if (lane >= d) incl += t;
  }
  if (lane == 63) ws[wave] = incl;
  __syncthreads();
  int64_t off = 0;
  total = 0;
  for (int w = 0; w < 16; ++w) {
    if (w < wave) off += ws[w];
    total += ws[w];
  }
  __syncthreads();
  return off + incl - v;
}

}  // namespace

// In-place exclusive scan of per-block counts blk[nblk][NC]; totals[NC].
template <int NC>
__global__ __launch_bounds__(1024) void k_scan_cols(int64_t *__restrict__ blk, int64_t nblk,
                                                    int64_t *__restrict__ totals) {
  const int64_t chunk = (nblk + 1023) / 1024;
  const int64_t b0 = threadIdx.x * chunk;
  const int64_t b1 = b0 + chunk < nblk ? b0 + chunk : nblk;
  for (int c = 0; c < NC; ++c) {
    int64_t s = 0;
    for (int64_t b = b0; b < b1; ++b) s += blk[b * NC + c];
    int64_t tot;
    int64_t off = scan1024(s, tot);
    for (int64_t b = b0; b < b1; ++b) {
      const int64_t v = blk[b * NC + c];
      blk[b * NC + c] = off;
      off += v;
    }
    if (threadIdx.x == 0) totals[c] = tot;
  }
}

__global__ __launch_bounds__(kBlock) void k_gate_count(const BeamPtrs6 b, const int64_t *__restrict__ n_alive,
                                                       int64_t n_total, const SurrDev c,
                                                       uint8_t *__restrict__ flags, int64_t *__restrict__ blk) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t na = min(*n_alive, n_total);
  int f = 0, rej = 0;
  if (i < n_total) {
    if (i < na) {
      double z[6];
      load6(b, i, z);
      f = surr_gate(c, z) ? 1 : 0;
      rej = 1 - f;
    }
    flags[i] = static_cast<uint8_t>(f);
  }
  const int ca = __syncthreads_count(f);
  const int cr = __syncthreads_count(rej);
  if (blk != nullptr && threadIdx.x == 0) {
    blk[2 * blockIdx.x] = ca;
    blk[2 * blockIdx.x + 1] = cr;
  }
}

__global__ __launch_bounds__(kBlock) void k_gate_split(const uint8_t *__restrict__ flags,
                                                       const int64_t *__restrict__ n_alive,
                                                       int64_t n_total, const int64_t *__restrict__ blk,
                                                       uint32_t *__restrict__ adm, uint32_t *__restrict__ rej) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t na = min(*n_alive, n_total);
  const int f = (i < n_total) ? flags[i] : 0;
  const int r = (i < na && f == 0) ? 1 : 0;
  int ta, tr;
  const int ra = block_exclusive_scan(f, ta);
  const int rr = block_exclusive_scan(r, tr);
  if (f) adm[blk[2 * blockIdx.x] + ra] = static_cast<uint32_t>(i);
  if (r) rej[blk[2 * blockIdx.x + 1] + rr] = static_cast<uint32_t>(i);
}

__global__ __launch_bounds__(kBlock) void k_gather(const BeamPtrs6 src, const uint32_t *__restrict__ list,
                                                   const int64_t *__restrict__ count, const BeamPtrs6 dst,
                                                   int64_t *__restrict__ dst_n, double *zin0, double *zin1, double *zin2, double *zin3,
                                                   double *zin4, double *zin5, int id_mode) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t n = *count;
  if (j == 0 && dst_n != nullptr) *dst_n = n;
  if (j >= n) return;
  const uint32_t i = list[j];
  double *zin[6] = {zin0, zin1, zin2, zin3, zin4, zin5};
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double v = src.z[k][i];
    dst.z[k][j] = v;
    if (zin0 != nullptr) zin[k][j] = v;
  }
  dst.id[j] = id_mode ? i : static_cast<uint32_t>(j);
  dst.lost_at[j] = src.lost_at[i];
}

__global__ __launch_bounds__(kBlock) void k_scatter_back(const BeamPtrs6 stage,
                                                         const int64_t *__restrict__ count,
                                                         const BeamPtrs6 beam) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (j >= *count) return;
  const uint32_t p = stage.id[j];
#pragma unroll
  for (int k = 0; k < 6; ++k) beam.z[k][p] = stage.z[k][j];
  beam.lost_at[p] = stage.lost_at[j];
}

__global__ __launch_bounds__(kBlock) void k_pairs(const BeamPtrs6 stage, const int64_t *__restrict__ n_stage,
                                                  const double *z0, const double *z1, const double *z2,
                                                  const double *z3, const double *z4, const double *z5,
                                                  const SurrDev c, float *__restrict__ u,
                                                  float *__restrict__ r, int64_t *__restrict__ n_pairs) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t n = *n_stage;
  if (j == 0) *n_pairs = n;
  if (j >= n) return;
  const uint32_t k = stage.id[j];
  const double *zin[6] = {z0, z1, z2, z3, z4, z5};
  double zi[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) zi[q] = zin[q][k];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    float uv = 0.0f, rv = 0.0f;
    if (q < 6 && q != kMlpSCol) uv = static_cast<float>(zi[q] * c.inv_nw[q]);
    if (q < kMlpDCol) rv = static_cast<float>(stage.z[q][j] - surr_linear(c, zi, q));
    u[j * 8 + q] = uv;
    r[j * 8 + q] = rv;
  }
}

__global__ __launch_bounds__(kBlock) void k_sumsq_part(const float *__restrict__ r, int64_t n,
                                                       double *__restrict__ part) {
  double acc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) acc[k] = 0.0;
  for (int64_t j = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; j < n;
       j += static_cast<int64_t>(gridDim.x) * kBlock) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const double v = static_cast<double>(r[j * 8 + k]);
      acc[k] += v * v;
    }
  }
  const double *t = block_sum<8>(acc);
  if (threadIdx.x < 8) part[blockIdx.x * 8 + threadIdx.x] = t[threadIdx.x];
}

__global__ __launch_bounds__(kBlock) void k_sumsq_final(const double *__restrict__ part, int nblk,
                                                        double *__restrict__ out) {
  double acc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) acc[k] = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kBlock)
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] += part[b * 8 + k];
  const double *t = block_sum<8>(acc);
  if (threadIdx.x < 8) out[threadIdx.x] = t[threadIdx.x];
}

__global__ __launch_bounds__(kBlock) void k_sample_count(const SurrDev c, uint64_t seed, uint64_t c0,
                                                         int64_t M, int64_t *__restrict__ blk) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  int f = 0;
  if (j < M) {
    double z[6];
    surr_draw(c, seed, c0 + static_cast<uint64_t>(j), z);
    f = surr_gate(c, z) ? 1 : 0;
  }
  const int cnt = __syncthreads_count(f);
  if (threadIdx.x == 0) blk[blockIdx.x] = cnt;
}

__global__ __launch_bounds__(kBlock) void k_sample_write(const SurrDev c, uint64_t seed, uint64_t c0,
                                                         int64_t M, const int64_t *__restrict__ blk,
                                                         const BeamPtrs6 out, const int64_t *__restrict__ base,
                                                         int64_t cap) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  double z[6];
  int f = 0;
  if (j < M) {
    surr_draw(c, seed, c0 + static_cast<uint64_t>(j), z);
    f = surr_gate(c, z) ? 1 : 0;
  }
  int tot;
  const int rank = block_exclusive_scan(f, tot);
  const int64_t pos = *base + blk[blockIdx.x] + rank;
  if (f && pos < cap) {
#pragma unroll
    for (int k = 0; k < 6; ++k) out.z[k][pos] = z[k];
    out.id[pos] = static_cast<uint32_t>(pos);
    out.lost_at[pos] = -1;
  }
}

__global__ void k_sample_advance(int64_t *base, const int64_t *total, int64_t cap) {
  const int64_t v = *base + *total;
  *base = v < cap ? v : cap;
}

// ------------------------------------------------------------------ launchers
static int grid_of(int64_t n) { return static_cast<int>(n > 0 ? (n + kBlock - 1) / kBlock : 1); }

hipError_t launch_gate_flags(const BeamPtrs6 &b, const int64_t *n_alive, int64_t n_total,
                             const SurrDev &c, uint8_t *flags, hipStream_t st) {
  hipLaunchKernelGGL(k_gate_count, dim3(grid_of(n_total)), dim3(kBlock), 0, st, b, n_alive, n_total, c,
                     flags, static_cast<int64_t *>(nullptr));
  return hipGetLastError();
}

hipError_t launch_gate_split(const BeamPtrs6 &b, const int64_t *n_alive, int64_t n_total,
                             const SurrDev &c, uint8_t *flags, int64_t *blk, uint32_t *adm,
                             uint32_t *rej, int64_t *counts, hipStream_t st) {
  const int g = grid_of(n_total);
  hipLaunchKernelGGL(k_gate_count, dim3(g), dim3(kBlock), 0, st, b, n_alive, n_total, c, flags, blk);
  hipLaunchKernelGGL(k_scan_cols<2>, dim3(1), dim3(1024), 0, st, blk, static_cast<int64_t>(g), counts);
  hipLaunchKernelGGL(k_gate_split, dim3(g), dim3(kBlock), 0, st, flags, n_alive, n_total, blk, adm, rej);
  return hipGetLastError();
}

hipError_t launch_gather(const BeamPtrs6 &src, const uint32_t *list, const int64_t *count,
                         int64_t n_total, const BeamPtrs6 &dst, int64_t *dst_n, double *const *zin,
                         int id_mode, hipStream_t st) {
  double *zz[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  if (zin != nullptr)
    for (int k = 0; k < 6; ++k) zz[k] = zin[k];
  hipLaunchKernelGGL(k_gather, dim3(grid_of(n_total)), dim3(kBlock), 0, st, src, list, count, dst, dst_n,
                     zz[0], zz[1], zz[2], zz[3], zz[4], zz[5], id_mode);
  return hipGetLastError();
}

hipError_t launch_scatter_back(const BeamPtrs6 &stage, const int64_t *count, int64_t n_total,
                               const BeamPtrs6 &beam, hipStream_t st) {
  hipLaunchKernelGGL(k_scatter_back, dim3(grid_of(n_total)), dim3(kBlock), 0, st, stage, count, beam);
  return hipGetLastError();
}

hipError_t launch_pairs(const BeamPtrs6 &stage, const int64_t *n_stage, int64_t n_total,
                        double *const *zin, const SurrDev &c, float *u, float *r, int64_t *n_pairs,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_pairs, dim3(grid_of(n_total)), dim3(kBlock), 0, st, stage, n_stage, zin[0], zin[1],
                     zin[2], zin[3], zin[4], zin[5], c, u, r, n_pairs);
  return hipGetLastError();
}

hipError_t launch_sumsq(const float *r, int64_t n, double *part, int nblk, double *sumsq,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_sumsq_part, dim3(nblk), dim3(kBlock), 0, st, r, n, part);
  hipLaunchKernelGGL(k_sumsq_final, dim3(1), dim3(kBlock), 0, st, part, nblk, sumsq);
  return hipGetLastError();
}

hipError_t launch_sample(const SurrDev &c, uint64_t seed, uint64_t c0, int64_t M, int64_t *blk,
                         const BeamPtrs6 &out, int64_t *base, int64_t cap, hipStream_t st) {
  const int g = grid_of(M);
  hipLaunchKernelGGL(k_sample_count, dim3(g), dim3(kBlock), 0, st, c, seed, c0, M, blk);
  hipLaunchKernelGGL(k_scan_cols<1>, dim3(1), dim3(1024), 0, st, blk, static_cast<int64_t>(g), blk + g);
  hipLaunchKernelGGL(k_sample_write, dim3(g), dim3(kBlock), 0, st, c, seed, c0, M, blk, out, base, cap);
  hipLaunchKernelGGL(k_sample_advance, dim3(1), dim3(1), 0, st, base, blk + g, cap);
  return hipGetLastError();
}

}  // namespace trk
