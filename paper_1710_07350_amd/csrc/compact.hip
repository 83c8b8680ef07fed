// compact.hip -- stable particle-loss compaction.
//
// The paper's loss algorithm (Sec. 2.5) flags lost particles, sums the flags
// (skipping the rest when nothing was lost), scans them and moves the lost
// particles behind the survivors.  This version keeps every order stable so
// the result does not depend on when compaction runs:
//   survivors   -> [0, n_new) in their previous order;
//   newly lost  -> [n_new, n_old) by loss record descending (latest first),
//                  ties in their previous order;
//   older lost  -> untouched beyond n_old.
// Kernels (all launched unconditionally; after `count`/`scan` they return at
// once when nothing was lost):
//   count   per-block survivor/loss counts and the extent of the loss records
//   scan    one block: exclusive block offsets, header, *n_alive update
//   gather  newly lost (dense rank of (pass, element), position) in position order
//   sort    one block: stable LSD radix sort of that list, 8 bits per pass
//   scatter survivors and the sorted lost ones into a staging copy
//   copy    staging copy -> beam for the positions that changed
#include "reduce.h"

namespace trk {

enum Hdr { H_NOLD = 0, H_NNEW, H_NLOST, H_LO, H_PMIN, H_PMAX, H_EMIN, H_EMAX, H_BITS, H_WHICH };
enum Blk { B_ALIVE = 0, B_LOST, B_LO, B_PMIN, B_NPMAX, B_EMIN, B_NEMAX, B_AOFF, B_LOFF };
constexpr int kBlkStride = 10;
constexpr int64_t kI64Max = 0x7fffffffffffffffLL;

__device__ __forceinline__ int64_t wave_min_i64(int64_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const int64_t o = __shfl_xor(v, m, 64);
    v = o < v ? o : v;
  }
  return v;
}

template <int N, int kThreads>
__device__ __forceinline__ void block_min_i64(int64_t (&v)[N]) {
  __shared__ int64_t part[kThreads / 64][N];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = wave_min_i64(v[k]);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) part[wave][k] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < N; ++k) {
    int64_t m = part[0][k];
    for (int w = 1; w < kThreads / 64; ++w) m = part[w][k] < m ? part[w][k] : m;
    v[k] = m;
  }
  __syncthreads();
}

__global__ __launch_bounds__(kBlock) void k_cmp_count(const int64_t *__restrict__ lost_at,
                                                      const int64_t *__restrict__ n_alive,
                                                      int64_t *__restrict__ blk) {
  const int64_t n = *n_alive;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t rec = i < n ? lost_at[i] : -1;
  const bool lost = rec >= 0;
  const bool alive = i < n && !lost;
  const int na = __syncthreads_count(alive);
  const int nl = __syncthreads_count(lost);
  int64_t m[5];
  const int64_t pass = rec >> 32, elem = rec & 0xffffffffLL;
  m[0] = lost ? i : kI64Max;
  m[1] = lost ? pass : kI64Max;
  m[2] = lost ? -pass : kI64Max;
  m[3] = lost ? elem : kI64Max;
  m[4] = lost ? -elem : kI64Max;
  block_min_i64<5, kBlock>(m);
  if (threadIdx.x == 0) {
    int64_t *b = blk + static_cast<int64_t>(blockIdx.x) * kBlkStride;
    b[B_ALIVE] = na;
    b[B_LOST] = nl;
    b[B_LO] = m[0];
    b[B_PMIN] = m[1];
    b[B_NPMAX] = m[2];
    b[B_EMIN] = m[3];
    b[B_NEMAX] = m[4];
  }
}

__device__ __forceinline__ int64_t block_scan_i64_1024(int64_t v, int64_t &total) {
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

__global__ __launch_bounds__(1024) void k_cmp_scan(int64_t *__restrict__ blk, int64_t nblk,
                                                   int64_t *__restrict__ hdr,
                                                   int64_t *__restrict__ n_alive) {
  const int64_t chunk = (nblk + 1023) / 1024;
  const int64_t b0 = threadIdx.x * chunk;
  const int64_t b1 = b0 + chunk < nblk ? b0 + chunk : nblk;
  int64_t sa = 0, sl = 0;
  int64_t m[5] = {kI64Max, kI64Max, kI64Max, kI64Max, kI64Max};
  for (int64_t b = b0; b < b1; ++b) {
    const int64_t *r = blk + b * kBlkStride;
    sa += r[B_ALIVE];
    sl += r[B_LOST];
    for (int k = 0; k < 5; ++k) m[k] = r[B_LO + k] < m[k] ? r[B_LO + k] : m[k];
  }
  int64_t ta, tl;
  int64_t oa = block_scan_i64_1024(sa, ta);
  int64_t ol = block_scan_i64_1024(sl, tl);
  for (int64_t b = b0; b < b1; ++b) {
    int64_t *r = blk + b * kBlkStride;
    r[B_AOFF] = oa;
    r[B_LOFF] = ol;
    oa += r[B_ALIVE];
    ol += r[B_LOST];
  }
  block_min_i64<5, 1024>(m);
  if (threadIdx.x == 0) {
    const int64_t n_old = *n_alive;
    hdr[H_NOLD] = n_old;
    hdr[H_NNEW] = n_old - tl;
    hdr[H_NLOST] = tl;
    hdr[H_LO] = tl > 0 ? m[0] : n_old;
    hdr[H_PMIN] = m[1];
    hdr[H_PMAX] = -m[2];
    hdr[H_EMIN] = m[3];
    hdr[H_EMAX] = -m[4];
    int bits = 0;
    if (tl > 0) {
      const uint64_t range = static_cast<uint64_t>(-m[2] - m[1] + 1) *
                             static_cast<uint64_t>(-m[4] - m[3] + 1);
      bits = range > 1 ? 64 - __builtin_clzll(range - 1) : 0;
    }
    hdr[H_BITS] = bits;
    hdr[H_WHICH] = 0;
    *n_alive = n_old - tl;
  }
}

// dense rank ascending == loss record descending
__global__ __launch_bounds__(kBlock) void k_cmp_gather(const int64_t *__restrict__ lost_at,
                                                       const int64_t *__restrict__ blk,
                                                       const int64_t *__restrict__ hdr,
                                                       uint64_t *__restrict__ key,
                                                       uint32_t *__restrict__ pos) {
  if (hdr[H_NLOST] == 0) return;
  const int64_t n = hdr[H_NOLD];
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t rec = i < n ? lost_at[i] : -1;
  const bool lost = rec >= 0;
  int tot;
  const int rank = block_exclusive_scan(lost ? 1 : 0, tot);
  if (lost) {
    const int64_t pmax = hdr[H_PMAX], emin = hdr[H_EMIN], emax = hdr[H_EMAX];
    const int64_t pass = rec >> 32, elem = rec & 0xffffffffLL;
    const uint64_t r = static_cast<uint64_t>(pmax - pass) * static_cast<uint64_t>(emax - emin + 1) +
                       static_cast<uint64_t>(emax - elem);
    const int64_t dst = blk[static_cast<int64_t>(blockIdx.x) * kBlkStride + B_LOFF] + rank;
    key[dst] = r;
    pos[dst] = static_cast<uint32_t>(i);
  }
}

// Single-workgroup stable LSD radix sort, 8-bit digits.  Within a 1024-item
// tile, lanes with equal digits find each other with eight ballots (a wave
// multi-split); per-wave digit counts are scanned across waves in wave order,
// so equal keys keep their input order.
__global__ __launch_bounds__(1024) void k_cmp_sort(int64_t *__restrict__ hdr, uint64_t *ka,
                                                   uint32_t *pa, uint64_t *kb, uint32_t *pb) {
  __shared__ uint32_t base[256];
  __shared__ uint32_t wcnt[16][256];
  const int64_t nl = hdr[H_NLOST];
  if (nl == 0) return;
  const int npass = static_cast<int>((hdr[H_BITS] + 7) / 8);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const uint64_t lt_mask = (1ull << lane) - 1ull;
  uint64_t *sk = ka, *dk = kb;
  uint32_t *sp = pa, *dp = pb;
  for (int ps = 0; ps < npass; ++ps) {
    const int shift = 8 * ps;
    if (t < 256) base[t] = 0u;
    for (int j = t; j < 16 * 256; j += 1024) (&wcnt[0][0])[j] = 0u;
    __syncthreads();
    for (int64_t j = t; j < nl; j += 1024) atomicAdd(&base[(sk[j] >> shift) & 255u], 1u);
    __syncthreads();
    if (t == 0) {
      uint32_t run = 0;
      for (int d = 0; d < 256; ++d) {
        const uint32_t c = base[d];
        base[d] = run;
        run += c;
      }
    }
    __syncthreads();
    for (int64_t tile = 0; tile < nl; tile += 1024) {
      const int64_t j = tile + t;
      const bool valid = j < nl;
      const uint64_t k = valid ? sk[j] : 0ull;
      const uint32_t p = valid ? sp[j] : 0u;
      const uint32_t dg = static_cast<uint32_t>((k >> shift) & 255u);
      uint64_t peers = __ballot(valid);
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const bool bit = (dg >> b) & 1u;
        const uint64_t m = __ballot(bit);
        peers &= bit ? m : ~m;
      }
      const uint32_t rank = static_cast<uint32_t>(__popcll(peers & lt_mask));
      if (valid && rank == 0) wcnt[wave][dg] = static_cast<uint32_t>(__popcll(peers));
      __syncthreads();
      if (t < 256) {
        uint32_t run = base[t];
        for (int w = 0; w < 16; ++w) {
          const uint32_t c = wcnt[w][t];
          wcnt[w][t] = run;
          run += c;
        }
        base[t] = run;
      }
      __syncthreads();
      if (valid) {
        const uint32_t d = wcnt[wave][dg] + rank;
        dk[d] = k;
        dp[d] = p;
      }
      __syncthreads();
      for (int q = t; q < 16 * 256; q += 1024) (&wcnt[0][0])[q] = 0u;
      __syncthreads();
    }
    uint64_t *tk = sk; sk = dk; dk = tk;
    uint32_t *tp = sp; sp = dp; dp = tp;
  }
  if (t == 0) hdr[H_WHICH] = npass & 1;
}

struct BeamPtrs {
  double *z[6];
  uint32_t *id;
  int64_t *lost_at;
};

__device__ __forceinline__ void move_particle(const BeamPtrs &src, int64_t i, const BeamPtrs &dst,
                                              int64_t j) {
#pragma unroll
  for (int k = 0; k < 6; ++k) dst.z[k][j] = src.z[k][i];
  dst.id[j] = src.id[i];
  dst.lost_at[j] = src.lost_at[i];
}

__global__ __launch_bounds__(kBlock) void k_cmp_scatter(BeamPtrs beam, BeamPtrs stage,
                                                        const int64_t *__restrict__ blk,
                                                        const int64_t *__restrict__ hdr,
                                                        const uint32_t *__restrict__ pa,
                                                        const uint32_t *__restrict__ pb) {
  const int64_t nl = hdr[H_NLOST];
  if (nl == 0) return;
  const int64_t n_old = hdr[H_NOLD], n_new = hdr[H_NNEW], lo = hdr[H_LO];
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const bool alive = i < n_old && beam.lost_at[i] < 0;
  int tot;
  const int rank = block_exclusive_scan(alive ? 1 : 0, tot);
  if (alive && i >= lo) {
    const int64_t dst = blk[static_cast<int64_t>(blockIdx.x) * kBlkStride + B_AOFF] + rank;
    move_particle(beam, i, stage, dst);
  }
  const uint32_t *sorted = hdr[H_WHICH] ? pb : pa;
  for (int64_t t = i; t < nl; t += static_cast<int64_t>(gridDim.x) * kBlock)
    move_particle(beam, sorted[t], stage, n_new + t);
}

__global__ __launch_bounds__(kBlock) void k_cmp_copy(BeamPtrs beam, BeamPtrs stage,
                                                     const int64_t *__restrict__ hdr) {
  if (hdr[H_NLOST] == 0) return;
  const int64_t n_old = hdr[H_NOLD], lo = hdr[H_LO];
  for (int64_t i = lo + static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n_old;
       i += static_cast<int64_t>(gridDim.x) * kBlock)
    move_particle(stage, i, beam, i);
}

hipError_t launch_compact(double *const z[6], uint32_t *id, int64_t *lost_at, int64_t *n_alive,
                          int64_t n_total, const Workspace &w, hipStream_t st) {
  const int64_t nb = nblocks(n_total);
  if (nb < 1) return hipSuccess;
  const int grid = static_cast<int>(nb);
  BeamPtrs beam, stage;
  for (int k = 0; k < 6; ++k) {
    beam.z[k] = z[k];
    stage.z[k] = w.tz[k];
  }
  beam.id = id;
  beam.lost_at = lost_at;
  stage.id = w.tid;
  stage.lost_at = w.tlost;
  hipLaunchKernelGGL(k_cmp_count, dim3(grid), dim3(kBlock), 0, st, lost_at, n_alive, w.cmp_blk);
  hipLaunchKernelGGL(k_cmp_scan, dim3(1), dim3(1024), 0, st, w.cmp_blk, nb, w.cmp_hdr, n_alive);
  hipLaunchKernelGGL(k_cmp_gather, dim3(grid), dim3(kBlock), 0, st, lost_at, w.cmp_blk, w.cmp_hdr,
                     w.key_a, w.pos_a);
  hipLaunchKernelGGL(k_cmp_sort, dim3(1), dim3(1024), 0, st, w.cmp_hdr, w.key_a, w.pos_a, w.key_b,
                     w.pos_b);
  hipLaunchKernelGGL(k_cmp_scatter, dim3(grid), dim3(kBlock), 0, st, beam, stage, w.cmp_blk,
                     w.cmp_hdr, w.pos_a, w.pos_b);
  const int cgrid = grid < kMaxGridStride ? grid : kMaxGridStride;
  hipLaunchKernelGGL(k_cmp_copy, dim3(cgrid), dim3(kBlock), 0, st, beam, stage, w.cmp_hdr);
  return hipGetLastError();
}

}  // namespace trk
