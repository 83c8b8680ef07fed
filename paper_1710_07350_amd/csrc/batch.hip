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
// variant in fixed order afterwards.  Particles stay in place; lost ones are
// marked in lost_at.
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
      if (a.mom_part != nullptr)
        block_moment_row_multi<kP>(alive, z, a.mom_part + (t * a.npass + p) * 28);
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

// One block per (variant, pass): rows of the variant's chunks in order.
__global__ __launch_bounds__(kBlock) void k_batch_mom_finalize(const double *__restrict__ part,
                                                               const int64_t *__restrict__ chunk_off,
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
    double m[6];
    for (int k = 0; k < 6; ++k) m[k] = tot[1 + k] / n;
    o[0] = n;
    for (int k = 0; k < 6; ++k) o[1 + k] = m[k];
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

hipError_t launch_batch_mom_finalize(const double *part, const int64_t *chunk_off, int nvar,
                                     int npass, double *out, int out_pass0, int out_passes,
                                     hipStream_t st) {
  hipLaunchKernelGGL(k_batch_mom_finalize, dim3(nvar * npass), dim3(kBlock), 0, st, part,
                     chunk_off, npass, out, out_pass0, out_passes);
  return hipGetLastError();
}

}  // namespace trk
