// batch.hip -- many lattice variants with uneven particle counts in one
// persistent launch.
//
// The variants' beams are concatenated segments of one structure-of-arrays
// beam and their element records are concatenated tables of equal length.
// Work is split into (variant, chunk) tickets of kBlock*kP particles; a grid
// of a few blocks per compute unit pulls tickets from an atomic counter until
// none are left (every block leaves the loop when the counter passes the
// ticket count), so small and large variants balance across the machine.
// A chunk runs all its passes in registers, exactly as the fused run kernel
// does for one lattice, so every particle's trajectory equals that of its
// variant tracked alone.  Per-chunk, per-pass moment rows are reduced per
// variant in fixed order afterwards; they are sums of coordinates shifted by
// the variant's mean at the entry of the call, so that an offset beam (a
// closed-orbit offset, a large s) does not cancel in the central moments.
// Particles stay in place; lost ones are marked in lost_at.
#include <utility>

#include "apply.h"
#include "reduce.h"

namespace trk {

template <uint32_t kFeat, int kP>
__global__ __launch_bounds__(kBlock) void k_batch(const BatchArgs a) {
  const ConstPool pool = (ConstPool)a.pool;
  __shared__ int64_t tick_sh;
  __shared__ int var_sh;
  for (;;) {
    if (threadIdx.x == 0) {
      const int64_t t = static_cast<int64_t>(atomicAdd(a.ticket, 1u));
      int lo = 0, hi = a.nvar;  // chunk_off[lo] <= t < chunk_off[hi]
      if (t < a.total) {
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (a.chunk_off[mid] <= t)
            lo = mid;
          else
            hi = mid;
        }
      }
      tick_sh = t;
      var_sh = lo;
    }
    __syncthreads();
    const int64_t t = tick_sh;
    const int v = var_sh;
    __syncthreads();
    if (t >= a.total) break;  // uniform across the block

    const int64_t s1 = a.seg_off[v + 1];
    const int64_t base = a.seg_off[v] + (t - a.chunk_off[v]) * (static_cast<int64_t>(kBlock) * kP) +
                         threadIdx.x;
    const uint64_t seed = a.seeds[v];
    const ElemCtx cx{nullptr, 0, 0, nullptr, nullptr, static_cast<uint32_t>(seed),
                     static_cast<uint32_t>(seed >> 32)};
    const ConstElems elems = (ConstElems)(a.elems + static_cast<int64_t>(v) * a.nelem);

    double z[kP][6];
    bool act[kP], alive[kP];
    int64_t rec[kP];
    uint32_t pid[kP];
#pragma unroll
    for (int q = 0; q < kP; ++q) {
      const int64_t i = base + q * kBlock;
      act[q] = i < s1;
#pragma unroll
      for (int k = 0; k < 6; ++k) z[q][k] = (act[q] && ((a.ldmask >> k) & 1u)) ? a.z[k][i] : 0.0;
      pid[q] = (act[q] && ((a.ldmask >> 6) & 1u)) ? a.id[i] : 0u;
      alive[q] = act[q] && a.lost_at[i] < 0;
      act[q] = alive[q];
      rec[q] = -1;
    }
    for (int p = 0; p < a.npass; ++p) {
      const uint32_t gp = static_cast<uint32_t>(a.pass0 + p);
      for (int e = 0; e < a.nelem; ++e) {
        const DevElem E = elems[e];
#pragma unroll
        for (int q = 0; q < kP; ++q) apply<kFeat>(E, pool, cx, p, gp, e, z[q], alive[q], rec[q], pid[q]);
      }
      if (a.mom_part != nullptr) {
        const double *sh = a.mom_shift + static_cast<int64_t>(v) * 6;
        double d[kP][6];
#pragma unroll
        for (int q = 0; q < kP; ++q)
#pragma unroll
          for (int k = 0; k < 6; ++k) d[q][k] = alive[q] ? z[q][k] - sh[k] : 0.0;
        block_moment_row_multi<kP>(alive, d, a.mom_part + (t * a.npass + p) * 28);
      }
    }
#pragma unroll
    for (int q = 0; q < kP; ++q) {
      if (!act[q]) continue;
      const int64_t i = base + q * kBlock;
#pragma unroll
      for (int k = 0; k < 6; ++k)
        if ((a.stmask >> k) & 1u) a.z[k][i] = z[q][k];
      if (rec[q] >= 0) a.lost_at[i] = rec[q];
    }
  }
}

// Mean at entry of each variant (the shift of its moment rows): one block
// per chunk of kBlock*kP slots sums (n, z_k) over its alive particles, then
// one block per variant adds its chunks' rows in order; 0 when none is alive.
template <int kP>
__global__ __launch_bounds__(kBlock) void k_batch_mean_partial(const BatchArgs a) {
  const int64_t t = blockIdx.x;
  int lo = 0, hi = a.nvar;  // chunk_off[lo] <= t < chunk_off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (a.chunk_off[mid] <= t)
      lo = mid;
    else
      hi = mid;
  }
  const int v = lo;
  const int64_t s1 = a.seg_off[v + 1];
  const int64_t base =
      a.seg_off[v] + (t - a.chunk_off[v]) * (static_cast<int64_t>(kBlock) * kP) + threadIdx.x;
  double acc[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) acc[k] = 0.0;
#pragma unroll
  for (int q = 0; q < kP; ++q) {
    const int64_t i = base + q * kBlock;
    if (i < s1 && a.lost_at[i] < 0) {
      acc[0] += 1.0;
#pragma unroll
      for (int k = 0; k < 6; ++k) acc[1 + k] += a.z[k][i];
    }
  }
  const double *tot = block_sum<7>(acc);
  if (threadIdx.x < 7) a.mean_part[t * 7 + threadIdx.x] = tot[threadIdx.x];
}

__global__ __launch_bounds__(kBlock) void k_batch_mean_finalize(const double *__restrict__ part,
                                                                const int64_t *__restrict__ chunk_off,
                                                                double *__restrict__ shift) {
  const int v = blockIdx.x;
  double acc[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) acc[k] = 0.0;
  for (int64_t c = chunk_off[v] + threadIdx.x; c < chunk_off[v + 1]; c += kBlock) {
#pragma unroll
    for (int k = 0; k < 7; ++k) acc[k] += part[c * 7 + k];
  }
  const double *tot = block_sum<7>(acc);
  if (threadIdx.x < 6) {
    const double n = tot[0];
    shift[static_cast<int64_t>(v) * 6 + threadIdx.x] = n > 0.0 ? tot[1 + threadIdx.x] / n : 0.0;
  }
}

// One block per (variant, pass): rows of the variant's chunks in order, then
// mean_k = shift_k + S_k/n, cov_kl = S_kl/n - (S_k/n)(S_l/n) on the shifted
// sums; every output 0 for a variant with nobody alive.
__global__ __launch_bounds__(kBlock) void k_batch_mom_finalize(const double *__restrict__ part,
                                                               const int64_t *__restrict__ chunk_off,
                                                               const double *__restrict__ shift,
                                                               int npass, double *__restrict__ out,
                                                               int out_pass0, int out_passes) {
  const int v = blockIdx.x / npass, p = blockIdx.x % npass;
  double acc[28];
#pragma unroll
  for (int k = 0; k < 28; ++k) acc[k] = 0.0;
  for (int64_t c = chunk_off[v] + threadIdx.x; c < chunk_off[v + 1]; c += kBlock) {
    const double *row = part + (c * npass + p) * 28;
#pragma unroll
    for (int k = 0; k < 28; ++k) acc[k] += row[k];
  }
  const double *tot = block_sum<28>(acc);
  if (threadIdx.x == 0) {
    double *o = out + (static_cast<int64_t>(v) * out_passes + out_pass0 + p) * 28;
    const double n = tot[0];
    if (n == 0.0) {
      for (int k = 0; k < 28; ++k) o[k] = 0.0;
      return;
    }
    const double *sh = shift + static_cast<int64_t>(v) * 6;
    double m[6];
    for (int k = 0; k < 6; ++k) m[k] = tot[1 + k] / n;
    o[0] = n;
    for (int k = 0; k < 6; ++k) o[1 + k] = sh[k] + m[k];
    int idx = 7;
    for (int k = 0; k < 6; ++k)
      for (int l = k; l < 6; ++l, ++idx) o[idx] = tot[idx] / n - m[k] * m[l];
  }
}

template <uint32_t kFeat>
void launch_batch_feat(const BatchArgs &a, int ppt, int grid, hipStream_t st) {
  if (ppt >= 4)
    hipLaunchKernelGGL((k_batch<kFeat, 4>), dim3(grid), dim3(kBlock), 0, st, a);
  else if (ppt == 2)
    hipLaunchKernelGGL((k_batch<kFeat, 2>), dim3(grid), dim3(kBlock), 0, st, a);
  else
    hipLaunchKernelGGL((k_batch<kFeat, 1>), dim3(grid), dim3(kBlock), 0, st, a);
}

template <uint32_t... kF>
void batch_dispatch(uint32_t feat, const BatchArgs &a, int ppt, int grid, hipStream_t st,
                    std::integer_sequence<uint32_t, kF...>) {
  // families without RF cavities and wakes: F_KD | F_RNG | F_GEN subsets
  ((feat == ((kF & 1u) * F_KD | ((kF >> 1) & 1u) * F_RNG | ((kF >> 2) & 1u) * F_GEN)
        ? (launch_batch_feat<((kF & 1u) * F_KD | ((kF >> 1) & 1u) * F_RNG |
                              ((kF >> 2) & 1u) * F_GEN)>(a, ppt, grid, st),
           0)
        : 0),
   ...);
}

hipError_t launch_batch(const BatchArgs &a, uint32_t feat, int ppt, int grid, hipStream_t st) {
  batch_dispatch(feat, a, ppt, grid, st, std::make_integer_sequence<uint32_t, 8>{});
  return hipGetLastError();
}

hipError_t launch_batch_mean(const BatchArgs &a, int ppt, hipStream_t st) {
  const int64_t total = a.total;
  if (ppt >= 4)
    hipLaunchKernelGGL((k_batch_mean_partial<4>), dim3(total), dim3(kBlock), 0, st, a);
  else if (ppt == 2)
    hipLaunchKernelGGL((k_batch_mean_partial<2>), dim3(total), dim3(kBlock), 0, st, a);
  else
    hipLaunchKernelGGL((k_batch_mean_partial<1>), dim3(total), dim3(kBlock), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_batch_mean_finalize, dim3(a.nvar), dim3(kBlock), 0, st, a.mean_part,
                     a.chunk_off, const_cast<double *>(a.mom_shift));
  return hipGetLastError();
}

hipError_t launch_batch_mom_finalize(const double *part, const int64_t *chunk_off,
                                     const double *shift, int nvar, int npass, double *out,
                                     int out_pass0, int out_passes, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_mom_finalize, dim3(nvar * npass), dim3(kBlock), 0, st, part,
                     chunk_off, shift, npass, out, out_pass0, out_passes);
  return hipGetLastError();
}

}  // namespace trk
