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
//   count   per-tile survivor/loss counts and the extent of the loss records
//   scan    one block: exclusive tile offsets, header, *n_alive update
//   gather  newly lost (dense rank of (pass, element), position) in position order
//   sort    stable LSD radix sort of that list by the rank, 8 bits per pass:
//           one workgroup for short lists, else count / scan / scatter
//           kernels over 4096-item tiles
//   scatter survivors and the sorted lost ones into a staging copy
//   copy    staging copy -> beam for the positions that changed
// A tile is 4096 consecutive slots: each wave of a 256-thread block takes
// 1024 of them in 16 rounds of 64, so loads stay coalesced and ranks inside
// a round come from one ballot.
#include <mutex>

#include <hipcub/hipcub.hpp>

#include "reduce.h"

namespace trk {

enum Hdr {
  H_NOLD = 0, H_NNEW, H_NLOST, H_LO, H_PMIN, H_PMAX, H_EMIN, H_EMAX, H_BITS, H_WHICH, H_NHOLE
};
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

constexpr int kCmpRounds = 16;
constexpr int kCmpTile = kBlock * kCmpRounds;  // 4096 slots per block

// slot of (round r, this lane) in this block's tile
__device__ __forceinline__ int64_t tile_slot(int r) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return static_cast<int64_t>(blockIdx.x) * kCmpTile + wave * (64 * kCmpRounds) + r * 64 + lane;
}
__device__ __forceinline__ uint64_t lanes_below() { return (1ull << (threadIdx.x & 63)) - 1ull; }

// The tile's loss records (-1 at and beyond n <= n_total), every load issued
// before the first is used: a ballot on each record as it arrives would wait
// for the loads one by one.  Slots at and beyond n read slot 0 (present in
// any launched grid) and drop it, so no branch separates the loads.
__device__ __forceinline__ void load_records(const int64_t *__restrict__ lost_at, int64_t n,
                                             int64_t (&rec)[kCmpRounds]) {
  int64_t v[kCmpRounds];
#pragma unroll
  for (int r = 0; r < kCmpRounds; ++r) {
    const int64_t i = tile_slot(r);
    v[r] = lost_at[i < n ? i : 0];
  }
#pragma unroll
  for (int r = 0; r < kCmpRounds; ++r) rec[r] = tile_slot(r) < n ? v[r] : -1;
}

// Exclusive offsets of the four waves' totals (in wave order), for two
// counters at once; returns the block totals through tot.
__device__ __forceinline__ void wave_offsets(int a, int b, int &oa, int &ob, int &ta, int &tb) {
  __shared__ int wt[kWaves][2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    wt[wave][0] = a;
    wt[wave][1] = b;
  }
  __syncthreads();
  oa = ob = ta = tb = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    if (w < wave) {
      oa += wt[w][0];
      ob += wt[w][1];
    }
    ta += wt[w][0];
    tb += wt[w][1];
  }
  __syncthreads();
}

__global__ __launch_bounds__(kBlock) void k_cmp_count(const int64_t *__restrict__ lost_at,
                                                      const int64_t *__restrict__ n_alive,
                                                      int64_t n_total, int64_t *__restrict__ blk) {
  const int64_t n = min(*n_alive, n_total);
  int64_t rec[kCmpRounds];
  load_records(lost_at, n, rec);
  int na = 0, nl = 0;  // per wave
  int64_t m[5] = {kI64Max, kI64Max, kI64Max, kI64Max, kI64Max};
#pragma unroll
  for (int r = 0; r < kCmpRounds; ++r) {
    const int64_t i = tile_slot(r);
    const bool lost = rec[r] >= 0;
    const bool alive = i < n && !lost;
    na += __popcll(__ballot(alive));
    nl += __popcll(__ballot(lost));
    if (lost) {
      const int64_t pass = rec[r] >> 32, elem = rec[r] & 0xffffffffLL;
      m[0] = i < m[0] ? i : m[0];
      m[1] = pass < m[1] ? pass : m[1];
      m[2] = -pass < m[2] ? -pass : m[2];
      m[3] = elem < m[3] ? elem : m[3];
      m[4] = -elem < m[4] ? -elem : m[4];
    }
  }
  int oa, ol, ta, tl;
  wave_offsets(na, nl, oa, ol, ta, tl);
  block_min_i64<5, kBlock>(m);
  if (threadIdx.x == 0) {
    int64_t *b = blk + static_cast<int64_t>(blockIdx.x) * kBlkStride;
    b[B_ALIVE] = ta;
    b[B_LOST] = tl;
    b[B_LO] = m[0];
    b[B_PMIN] = m[1];
    b[B_NPMAX] = m[2];
    b[B_EMIN] = m[3];
    b[B_NEMAX] = m[4];
  }
}

// exclusive scan of one int64 per thread over a kScanThreads block, in
// thread order; total receives the block sum
constexpr int kScanThreads = 256;
__device__ __forceinline__ int64_t block_scan_i64(int64_t v, int64_t &total) {
  __shared__ int64_t ws[kScanThreads / 64];
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
#pragma unroll
  for (int w = 0; w < kScanThreads / 64; ++w) {
    if (w < wave) off += ws[w];
    total += ws[w];
  }
  __syncthreads();
  return off + incl - v;
}

__global__ __launch_bounds__(kScanThreads) void k_cmp_scan(int64_t *__restrict__ blk, int64_t nblk,
                                                           int64_t *__restrict__ hdr,
                                                           int64_t *__restrict__ n_alive,
                                                           int64_t n_total) {
  const int64_t chunk = (nblk + kScanThreads - 1) / kScanThreads;
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
  int64_t oa = block_scan_i64(sa, ta);
  int64_t ol = block_scan_i64(sl, tl);
  for (int64_t b = b0; b < b1; ++b) {
    int64_t *r = blk + b * kBlkStride;
    r[B_AOFF] = oa;
    r[B_LOFF] = ol;
    oa += r[B_ALIVE];
    ol += r[B_LOST];
  }
  block_min_i64<5, kScanThreads>(m);
  if (threadIdx.x == 0) {
    const int64_t n_old = min(*n_alive, n_total);
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
    hdr[H_NHOLE] = 0;
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
  int64_t rec[kCmpRounds];
  load_records(lost_at, n, rec);
  int cnt = 0;
#pragma unroll
  for (int r = 0; r < kCmpRounds; ++r) cnt += __popcll(__ballot(rec[r] >= 0));
  int off, o2, tot, t2;
  wave_offsets(cnt, 0, off, o2, tot, t2);
  if (tot == 0) return;
  const int64_t pmax = hdr[H_PMAX], emin = hdr[H_EMIN], emax = hdr[H_EMAX];
  int64_t dst = blk[static_cast<int64_t>(blockIdx.x) * kBlkStride + B_LOFF] + off;
#pragma unroll
  for (int r = 0; r < kCmpRounds; ++r) {
    const bool lost = rec[r] >= 0;
    const uint64_t mask = __ballot(lost);
    if (lost) {
      const int64_t pass = rec[r] >> 32, elem = rec[r] & 0xffffffffLL;
      const uint64_t rk = static_cast<uint64_t>(pmax - pass) * static_cast<uint64_t>(emax - emin + 1) +
                          static_cast<uint64_t>(emax - elem);
      const int64_t d = dst + __popcll(mask & lanes_below());
      key[d] = rk;
      pos[d] = static_cast<uint32_t>(tile_slot(r));
    }
    dst += __popcll(mask);
  }
}

// Lists longer than this are sorted by the multi-block kernels (keys of at
// most 32 bits); shorter ones, and wider keys, by one workgroup.
constexpr int64_t kSmallSort = 16384;
__device__ __forceinline__ bool multi_sort(const int64_t *hdr) {
  return hdr[H_NLOST] > kSmallSort && hdr[H_BITS] <= 32;
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
  if (nl == 0 || multi_sort(hdr)) return;
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

// A particle's eight fields, loaded together before any is stored (the
// source and destination arrays are never the same memory, but the compiler
// cannot know, so a field-by-field copy would serialise the loads).
struct Particle {
  double z[6];
  uint32_t id;
  int64_t lost_at;
};
__device__ __forceinline__ Particle load_particle(const BeamPtrs &src, int64_t i) {
  Particle q;
#pragma unroll
  for (int k = 0; k < 6; ++k) q.z[k] = src.z[k][i];
  q.id = src.id[i];
  q.lost_at = src.lost_at[i];
  return q;
}
__device__ __forceinline__ void store_particle(const BeamPtrs &dst, int64_t j, const Particle &q) {
#pragma unroll
  for (int k = 0; k < 6; ++k) dst.z[k][j] = q.z[k];
  dst.id[j] = q.id;
  dst.lost_at[j] = q.lost_at;
}
__device__ __forceinline__ void move_particle(const BeamPtrs &src, int64_t i, const BeamPtrs &dst,
                                              int64_t j) {
  store_particle(dst, j, load_particle(src, i));
}

__global__ __launch_bounds__(kBlock) void k_cmp_scatter(BeamPtrs beam, BeamPtrs stage,
                                                        const int64_t *__restrict__ blk,
                                                        const int64_t *__restrict__ hdr,
                                                        const uint32_t *__restrict__ pa,
                                                        const uint32_t *__restrict__ pb) {
  const int64_t nl = hdr[H_NLOST];
  if (nl == 0) return;
  const int64_t n_old = hdr[H_NOLD], n_new = hdr[H_NNEW], lo = hdr[H_LO];
  int64_t rec[kCmpRounds];
  load_records(beam.lost_at, n_old, rec);
  bool alive[kCmpRounds];
  int cnt = 0;
#pragma unroll
  for (int r = 0; r < kCmpRounds; ++r) {
    alive[r] = tile_slot(r) < n_old && rec[r] < 0;
    cnt += __popcll(__ballot(alive[r]));
  }
  int off, o2, tot, t2;
  wave_offsets(cnt, 0, off, o2, tot, t2);
  int64_t dst = blk[static_cast<int64_t>(blockIdx.x) * kBlkStride + B_AOFF] + off;
  constexpr int kBatch = 4;  // particles in flight per thread
#pragma unroll
  for (int r0 = 0; r0 < kCmpRounds; r0 += kBatch) {
    Particle q[kBatch];
    int64_t to[kBatch];
    bool mv[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int r = r0 + u;
      const uint64_t mask = __ballot(alive[r]);
      const int64_t i = tile_slot(r);
      mv[u] = alive[r] && i >= lo;
      to[u] = dst + __popcll(mask & lanes_below());
      dst += __popcll(mask);
      if (mv[u]) q[u] = load_particle(beam, i);
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
      if (mv[u]) store_particle(stage, to[u], q[u]);
  }
  const uint32_t *sorted = hdr[H_WHICH] ? pb : pa;
  for (int64_t q = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; q < nl;
       q += static_cast<int64_t>(gridDim.x) * kBlock)
    move_particle(beam, sorted[q], stage, n_new + q);
}

// ------------------------------------------------------------------ multi-block radix sort
// Stable LSD radix sort of the lost list (nl = hdr[H_NLOST] items, keys of
// at most 32 bits), 8 bits per pass, for lists longer than kSmallSort.  The
// host launches four passes; a pass beyond the key width returns at once.
// Per pass: per-tile digit counts (digit-major table), a scan of each digit's
// row over the tiles, and a scatter in which every item lands at
//   (items of smaller digits) + (same digit in earlier tiles)
//   + (same digit earlier in this tile),
// the last term from ballots (equal-digit peers in a round) and per-wave
// running counts, waves taking consecutive quarters of the tile.
__device__ __forceinline__ bool rs_active(const int64_t *hdr, int pass) {
  return multi_sort(hdr) && 8 * pass < hdr[H_BITS];
}

__global__ __launch_bounds__(kBlock) void k_rs_count(const int64_t *__restrict__ hdr,
                                                     const uint64_t *__restrict__ ka,
                                                     const uint64_t *__restrict__ kb,
                                                     uint32_t *__restrict__ cnt, int pass,
                                                     int ntiles) {
  if (!rs_active(hdr, pass)) return;
  const int64_t nl = hdr[H_NLOST];
  if (static_cast<int64_t>(blockIdx.x) * kCmpTile >= nl) return;
  __shared__ uint32_t hist[256];
  hist[threadIdx.x] = 0u;
  __syncthreads();
  const uint64_t *src = (pass & 1) ? kb : ka;
  const int shift = 8 * pass;
  // every key load issued before the first atomic (slot 0 stands in past nl)
  uint64_t key[kCmpRounds];
#pragma unroll
  for (int r = 0; r < kCmpRounds; ++r) {
    const int64_t j = tile_slot(r);
    key[r] = src[j < nl ? j : 0];
  }
#pragma unroll
  for (int r = 0; r < kCmpRounds; ++r)
    if (tile_slot(r) < nl) atomicAdd(&hist[(key[r] >> shift) & 255u], 1u);
  __syncthreads();
  cnt[static_cast<int64_t>(threadIdx.x) * ntiles + blockIdx.x] = hist[threadIdx.x];
}

// block d: exclusive scan of digit d's counts over the active tiles
__global__ __launch_bounds__(kBlock) void k_rs_scan(const int64_t *__restrict__ hdr,
                                                    uint32_t *__restrict__ cnt,
                                                    uint32_t *__restrict__ rowtot, int pass,
                                                    int ntiles) {
  if (!rs_active(hdr, pass)) return;
  const int64_t nl = hdr[H_NLOST];
  const int act = static_cast<int>((nl + kCmpTile - 1) / kCmpTile);
  uint32_t *row = cnt + static_cast<int64_t>(blockIdx.x) * ntiles;
  uint32_t run = 0;
  for (int t0 = 0; t0 < act; t0 += kBlock) {
    const int t = t0 + threadIdx.x;
    const int v = t < act ? static_cast<int>(row[t]) : 0;
    int tot;
    const int ex = block_exclusive_scan(v, tot);
    if (t < act) row[t] = run + static_cast<uint32_t>(ex);
    run += static_cast<uint32_t>(tot);
  }
  if (threadIdx.x == 0) rowtot[blockIdx.x] = run;
}

__global__ __launch_bounds__(kBlock) void k_rs_scatter(int64_t *__restrict__ hdr, uint64_t *ka,
                                                       uint32_t *pa, uint64_t *kb, uint32_t *pb,
                                                       const uint32_t *__restrict__ cnt,
                                                       const uint32_t *__restrict__ rowtot,
                                                       int pass, int ntiles) {
  if (!rs_active(hdr, pass)) return;
  const int64_t nl = hdr[H_NLOST];
  if (static_cast<int64_t>(blockIdx.x) * kCmpTile >= nl) return;
  __shared__ uint32_t wcnt[kWaves][256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t *sk = (pass & 1) ? kb : ka;
  const uint32_t *sp = (pass & 1) ? pb : pa;
  uint64_t *dk = (pass & 1) ? ka : kb;
  uint32_t *dp = (pass & 1) ? pa : pb;
  const int shift = 8 * pass;
  // base of digit d in this tile: all smaller digits, then this digit's
  // items in earlier tiles
  int tot;
  const int below = block_exclusive_scan(static_cast<int>(rowtot[threadIdx.x]), tot);
  const uint32_t base =
      static_cast<uint32_t>(below) + cnt[static_cast<int64_t>(threadIdx.x) * ntiles + blockIdx.x];
#pragma unroll
  for (int w = 0; w < kWaves; ++w) wcnt[w][threadIdx.x] = 0u;
  __syncthreads();
  uint64_t key[kCmpRounds];
  uint32_t val[kCmpRounds];
  int rank[kCmpRounds], grp[kCmpRounds];
  const uint64_t lt = lanes_below();
#pragma unroll
  for (int r = 0; r < kCmpRounds; ++r) {
    const int64_t j = tile_slot(r);
    key[r] = sk[j < nl ? j : 0];  // all loads before the first ballot
    val[r] = sp[j < nl ? j : 0];
  }
#pragma unroll
  for (int r = 0; r < kCmpRounds; ++r) {
    const bool valid = tile_slot(r) < nl;
    if (!valid) key[r] = 0ull;
    const uint32_t dg = static_cast<uint32_t>((key[r] >> shift) & 255u);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (dg >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    rank[r] = valid ? static_cast<int>(__popcll(peers & lt)) : -1;
    grp[r] = static_cast<int>(__popcll(peers));
    if (valid && rank[r] == 0) wcnt[wave][dg] += static_cast<uint32_t>(grp[r]);
  }
  __syncthreads();
  {
    // per digit: the waves' offsets in wave order, after the tile's base
    uint32_t run = base;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      const uint32_t c = wcnt[w][threadIdx.x];
      wcnt[w][threadIdx.x] = run;
      run += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kCmpRounds; ++r) {
    const uint32_t dg = static_cast<uint32_t>((key[r] >> shift) & 255u);
    if (rank[r] >= 0) {
      const uint32_t d = wcnt[wave][dg] + static_cast<uint32_t>(rank[r]);
      dk[d] = key[r];
      dp[d] = val[r];
    }
    // the wave's lanes all read before its group leaders advance the count
    __builtin_amdgcn_wave_barrier();
    if (rank[r] == 0) wcnt[wave][dg] += static_cast<uint32_t>(grp[r]);
    __builtin_amdgcn_wave_barrier();
  }
  (void)lane;
  if (blockIdx.x == 0 && threadIdx.x == 0 && 8 * (pass + 1) >= hdr[H_BITS])
    hdr[H_WHICH] = (pass + 1) & 1;
}

__global__ __launch_bounds__(kBlock) void k_cmp_copy(BeamPtrs beam, BeamPtrs stage,
                                                     const int64_t *__restrict__ hdr) {
  if (hdr[H_NLOST] == 0) return;
  const int64_t n_old = hdr[H_NOLD], lo = hdr[H_LO];
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  constexpr int kBatch = 4;
  for (int64_t i0 = lo + static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i0 < n_old;
       i0 += kBatch * stride) {
    Particle q[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
      if (i0 + u * stride < n_old) q[u] = load_particle(stage, i0 + u * stride);
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
      if (i0 + u * stride < n_old) store_particle(beam, i0 + u * stride, q[u]);
  }
}

int64_t compact_tiles(int64_t n_total) { return (n_total + kCmpTile - 1) / kCmpTile; }

hipError_t launch_compact(double *const z[6], uint32_t *id, int64_t *lost_at, int64_t *n_alive,
                          int64_t n_total, const Workspace &w, hipStream_t st) {
  const int64_t nb = compact_tiles(n_total);
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
  hipLaunchKernelGGL(k_cmp_count, dim3(grid), dim3(kBlock), 0, st, lost_at, n_alive, n_total,
                     w.cmp_blk);
  hipLaunchKernelGGL(k_cmp_scan, dim3(1), dim3(kScanThreads), 0, st, w.cmp_blk, nb, w.cmp_hdr,
                     n_alive, n_total);
  hipLaunchKernelGGL(k_cmp_gather, dim3(grid), dim3(kBlock), 0, st, lost_at, w.cmp_blk, w.cmp_hdr,
                     w.key_a, w.pos_a);
  hipLaunchKernelGGL(k_cmp_sort, dim3(1), dim3(1024), 0, st, w.cmp_hdr, w.key_a, w.pos_a, w.key_b,
                     w.pos_b);
  for (int pass = 0; pass < 4; ++pass) {
    hipLaunchKernelGGL(k_rs_count, dim3(grid), dim3(kBlock), 0, st, w.cmp_hdr, w.key_a, w.key_b,
                       w.rs_cnt, pass, grid);
    hipLaunchKernelGGL(k_rs_scan, dim3(256), dim3(kBlock), 0, st, w.cmp_hdr, w.rs_cnt, w.rs_tot,
                       pass, grid);
    hipLaunchKernelGGL(k_rs_scatter, dim3(grid), dim3(kBlock), 0, st, w.cmp_hdr, w.key_a, w.pos_a,
                       w.key_b, w.pos_b, w.rs_cnt, w.rs_tot, pass, grid);
  }
  hipLaunchKernelGGL(k_cmp_scatter, dim3(grid), dim3(kBlock), 0, st, beam, stage, w.cmp_blk,
                     w.cmp_hdr, w.pos_a, w.pos_b);
  const int cgrid = static_cast<int>(nblocks(n_total) < kMaxGridStride ? nblocks(n_total)
                                                                        : kMaxGridStride);
  hipLaunchKernelGGL(k_cmp_copy, dim3(cgrid), dim3(kBlock), 0, st, beam, stage, w.cmp_hdr);
  return hipGetLastError();
}

// ------------------------------------------------------------------ the paper's variants
// Sparse swap (the paper's loss algorithm, Sec. 2.5): after count and scan,
// every block lists the holes of the head [0, n_new) -- lost particles, in
// index order -- and the survivors of the tail [n_new, n_old), in reverse
// index order; then the k-th hole swaps with the k-th tail survivor.  Only
// the 2H moved particles are read and written.  Survivors lose their order.
__global__ __launch_bounds__(kBlock) void k_swap_list(const int64_t *__restrict__ lost_at,
                                                      const int64_t *__restrict__ blk,
                                                      int64_t *__restrict__ hdr,
                                                      uint32_t *__restrict__ holes,
                                                      uint32_t *__restrict__ drev) {
  if (hdr[H_NLOST] == 0) return;
  const int64_t n_old = hdr[H_NOLD], n_new = hdr[H_NNEW];
  int64_t rec[kCmpRounds];
  load_records(lost_at, n_old, rec);
  int cl = 0, ca = 0, ch = 0;
#pragma unroll
  for (int r = 0; r < kCmpRounds; ++r) {
    const int64_t i = tile_slot(r);
    cl += __popcll(__ballot(rec[r] >= 0));
    ca += __popcll(__ballot(i < n_old && rec[r] < 0));
    ch += __popcll(__ballot(rec[r] >= 0 && i < n_new));
  }
  int ol, oa, tl, ta;
  wave_offsets(cl, ca, ol, oa, tl, ta);
  int oh, o2, th, t2;
  wave_offsets(ch, 0, oh, o2, th, t2);
  const int64_t *b = blk + static_cast<int64_t>(blockIdx.x) * kBlkStride;
  int64_t lr = b[B_LOFF] + ol, ar = b[B_AOFF] + oa;
  const uint64_t lt = lanes_below();
#pragma unroll
  for (int r = 0; r < kCmpRounds; ++r) {
    const int64_t i = tile_slot(r);
    const bool lost = rec[r] >= 0;
    const bool alive = i < n_old && !lost;
    const uint64_t ml = __ballot(lost), ma = __ballot(alive);
    if (lost && i < n_new) holes[lr + __popcll(ml & lt)] = static_cast<uint32_t>(i);
    if (alive && i >= n_new) drev[n_new - 1 - (ar + __popcll(ma & lt))] = static_cast<uint32_t>(i);
    lr += __popcll(ml);
    ar += __popcll(ma);
  }
  if (threadIdx.x == 0 && th > 0)
    atomicAdd(reinterpret_cast<unsigned long long *>(hdr + H_NHOLE),
              static_cast<unsigned long long>(th));
}

__device__ __forceinline__ void swap_particles(const BeamPtrs &b, int64_t i, int64_t j) {
  const Particle pi = load_particle(b, i), pj = load_particle(b, j);
  store_particle(b, i, pj);
  store_particle(b, j, pi);
}

__global__ __launch_bounds__(kBlock) void k_swap_move(BeamPtrs beam, const int64_t *__restrict__ hdr,
                                                      const uint32_t *__restrict__ holes,
                                                      const uint32_t *__restrict__ drev) {
  const int64_t h = hdr[H_NHOLE];
  for (int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; k < h;
       k += static_cast<int64_t>(gridDim.x) * kBlock)
    swap_particles(beam, holes[k], drev[h - 1 - k]);
}

// Sort by key (the straightforward algorithm the paper compares against):
// key = i for a survivor, i + N for a lost particle (N = n_total; slots
// beyond n_old get i + 2N and stay in place), a device-wide radix sort of
// (key, i), then every slot below n_old gathers its particle.
__global__ __launch_bounds__(kBlock) void k_sortkey_fill(const int64_t *__restrict__ lost_at,
                                                         const int64_t *__restrict__ hdr,
                                                         int64_t n_total, uint64_t *__restrict__ key,
                                                         uint32_t *__restrict__ val) {
  const int64_t n_old = hdr[H_NOLD];
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n_total;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    const uint64_t u = static_cast<uint64_t>(i);
    key[i] = i >= n_old ? u + 2 * static_cast<uint64_t>(n_total)
                        : (lost_at[i] >= 0 ? u + static_cast<uint64_t>(n_total) : u);
    val[i] = static_cast<uint32_t>(i);
  }
}

__global__ __launch_bounds__(kBlock) void k_sortkey_gather(BeamPtrs beam, BeamPtrs stage,
                                                           const int64_t *__restrict__ hdr,
                                                           const uint32_t *__restrict__ perm) {
  if (hdr[H_NLOST] == 0) return;
  const int64_t n_old = hdr[H_NOLD];
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  constexpr int kBatch = 4;
  for (int64_t j0 = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; j0 < n_old;
       j0 += kBatch * stride) {
    Particle q[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
      if (j0 + u * stride < n_old) q[u] = load_particle(beam, perm[j0 + u * stride]);
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
      if (j0 + u * stride < n_old) store_particle(stage, j0 + u * stride, q[u]);
  }
}

__global__ __launch_bounds__(kBlock) void k_sortkey_copy(BeamPtrs beam, BeamPtrs stage,
                                                         const int64_t *__restrict__ hdr) {
  if (hdr[H_NLOST] == 0) return;
  const int64_t n_old = hdr[H_NOLD];
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  constexpr int kBatch = 4;
  for (int64_t j0 = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; j0 < n_old;
       j0 += kBatch * stride) {
    Particle q[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
      if (j0 + u * stride < n_old) q[u] = load_particle(stage, j0 + u * stride);
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
      if (j0 + u * stride < n_old) store_particle(beam, j0 + u * stride, q[u]);
  }
}

static int key_bits(int64_t n_total) {
  const uint64_t top = 3 * static_cast<uint64_t>(n_total);
  return top > 1 ? 64 - __builtin_clzll(top - 1) : 1;
}

size_t sortkey_temp_bytes(int64_t n_total) {
  // the size query asks the runtime for device properties: remember the last answer
  static std::mutex mu;
  static int64_t last_n = -1;
  static size_t last_bytes = 0;
  std::lock_guard<std::mutex> lock(mu);
  if (n_total == last_n) return last_bytes;
  size_t bytes = 0;
  hipcub::DoubleBuffer<uint64_t> k(nullptr, nullptr);
  hipcub::DoubleBuffer<uint32_t> v(nullptr, nullptr);
  const int n = static_cast<int>(n_total > 0 ? n_total : 1);
  if (hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, k, v, n, 0, key_bits(n_total)) !=
      hipSuccess)
    return 0;
  last_n = n_total;
  last_bytes = bytes;
  return bytes;
}

hipError_t launch_compact_variant(int mode, double *const z[6], uint32_t *id, int64_t *lost_at,
                                  int64_t *n_alive, int64_t n_total, const Workspace &w,
                                  hipStream_t st) {
  const int64_t nb = compact_tiles(n_total);
  if (nb < 1) return hipSuccess;
  const int grid = static_cast<int>(nb);
  const int sgrid = static_cast<int>(nblocks(n_total) < kMaxGridStride ? nblocks(n_total)
                                                                        : kMaxGridStride);
  BeamPtrs beam, stage;
  for (int k = 0; k < 6; ++k) {
    beam.z[k] = z[k];
    stage.z[k] = w.tz[k];
  }
  beam.id = id;
  beam.lost_at = lost_at;
  stage.id = w.tid;
  stage.lost_at = w.tlost;
  hipLaunchKernelGGL(k_cmp_count, dim3(grid), dim3(kBlock), 0, st, lost_at, n_alive, n_total,
                     w.cmp_blk);
  hipLaunchKernelGGL(k_cmp_scan, dim3(1), dim3(kScanThreads), 0, st, w.cmp_blk, nb, w.cmp_hdr,
                     n_alive, n_total);
  if (mode == TRK_COMPACT_SWAP) {
    hipLaunchKernelGGL(k_swap_list, dim3(grid), dim3(kBlock), 0, st, lost_at, w.cmp_blk, w.cmp_hdr,
                       w.pos_a, w.pos_b);
    hipLaunchKernelGGL(k_swap_move, dim3(sgrid), dim3(kBlock), 0, st, beam, w.cmp_hdr, w.pos_a,
                       w.pos_b);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_sortkey_fill, dim3(sgrid), dim3(kBlock), 0, st, lost_at, w.cmp_hdr, n_total,
                     w.key_a, w.pos_a);
  hipcub::DoubleBuffer<uint64_t> keys(w.key_a, w.key_b);
  hipcub::DoubleBuffer<uint32_t> vals(w.pos_a, w.pos_b);
  size_t bytes = w.sort_tmp_bytes;
  hipError_t e = hipcub::DeviceRadixSort::SortPairs(w.sort_tmp, bytes, keys, vals,
                                                    static_cast<int>(n_total), 0,
                                                    key_bits(n_total), st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sortkey_gather, dim3(sgrid), dim3(kBlock), 0, st, beam, stage, w.cmp_hdr,
                     vals.Current());
  hipLaunchKernelGGL(k_sortkey_copy, dim3(sgrid), dim3(kBlock), 0, st, beam, stage, w.cmp_hdr);
  return hipGetLastError();
}

}  // namespace trk
