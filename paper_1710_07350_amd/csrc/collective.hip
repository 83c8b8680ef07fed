// collective.hip -- the cross-particle steps: range of s, histogram, wake
// convolution (binary64 sequential and FP32 matrix-core), wake kick and beam
// moments.
#include <type_traits>

#include "elements.h"
#include "reduce.h"

namespace trk {

constexpr double kCLight = 299792458.0;

// ------------------------------------------------------------------ range
__global__ __launch_bounds__(kBlock) void k_minmax(const double *__restrict__ s,
                                                   const int64_t *__restrict__ n_alive,
                                                   int64_t n_total, double *__restrict__ part,
                                                   uint32_t *zero_buf, int zero_n) {
  const int64_t n = min(*n_alive, n_total);
  if (zero_buf != nullptr && blockIdx.x == 0)
    for (int i = threadIdx.x; i < zero_n; i += kBlock) zero_buf[i] = 0u;
  double mn = __builtin_huge_val(), mx = -__builtin_huge_val();
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    const double v = s[i];
    mn = fmin(mn, v);
    mx = fmax(mx, v);
  }
  block_minmax(mn, mx);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = mn;
    part[2 * blockIdx.x + 1] = mx;
  }
}

hipError_t launch_minmax(const double *s, const int64_t *n_alive, int64_t n_total, double *mm_part,
                         int grid, uint32_t *zero_buf, int zero_n, hipStream_t st) {
  hipLaunchKernelGGL(k_minmax, dim3(grid), dim3(kBlock), 0, st, s, n_alive, n_total, mm_part,
                     zero_buf, zero_n);
  return hipGetLastError();
}

// ------------------------------------------------------------------ histogram
// Sub-histograms in LDS cut the contention of lanes hitting the same bin (the
// paper's sub-histogram scheme, Sec. 2.2): one per group of waves, as many as
// fit in 32 KB.  Blocks then add their non-zero bins to the global counts
// with integer atomics (exact, so the result is order-free).  Every block
// reduces the (min, max) partials of the preceding kernel itself, in the same
// order, so no extra launch is needed.
#ifndef TRK_HIST_THREADS
#define TRK_HIST_THREADS 1024
#endif
constexpr int kHistThreads = TRK_HIST_THREADS;
#ifndef TRK_HIST_ITEMS
#define TRK_HIST_ITEMS 32
#endif
constexpr int kHistItems = TRK_HIST_ITEMS;  // particles per thread (sets the grid)
constexpr int kHistMaxGrid = 512;
#ifndef TRK_HIST_UNROLL
#define TRK_HIST_UNROLL 8
#endif
constexpr int kHistUnroll = TRK_HIST_UNROLL;

// A transverse coordinate as an integer multiple of 2^-40 m (clamped to
// [-1, 1] m, ties to even, NaN counts 0), as a two's-complement word: sums of
// these words modulo 2^64 are exact and independent of their order.
__device__ __forceinline__ unsigned long long dip_quantum(double x) {
  if (x != x) return 0ull;
  x = x > 1.0 ? 1.0 : (x < -1.0 ? -1.0 : x);
  return static_cast<unsigned long long>(static_cast<long long>(__builtin_rint(x * 0x1p40)));
}

// kDip: the same histogram, plus per bin the sums of the quantised x and y
// (LDS sub-histograms of 64-bit words after the counts).
template <bool kDip>
__global__ __launch_bounds__(kHistThreads) void k_histogram(
    const double *__restrict__ s, const double *__restrict__ xs, const double *__restrict__ ys,
    const int64_t *__restrict__ n_alive, int64_t n_total, const double *__restrict__ mm_part,
    int mm_n, int nbins, int nsub, uint32_t *__restrict__ counts, unsigned long long *__restrict__ dip,
    double *__restrict__ range) {
  extern __shared__ uint32_t sub[];  // [nsub][nbins] counts; kDip: then [nsub][2][nbins] words
  __shared__ double pm[kHistThreads / 64][2];
  unsigned long long *subd =
      reinterpret_cast<unsigned long long *>(sub + ((nsub * nbins + 1) & ~1));
  const int64_t n = min(*n_alive, n_total);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double mn = __builtin_huge_val(), mx = -__builtin_huge_val();
  for (int j = threadIdx.x; j < mm_n; j += kHistThreads) {
    mn = fmin(mn, mm_part[2 * j]);
    mx = fmax(mx, mm_part[2 * j + 1]);
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    mn = fmin(mn, __shfl_xor(mn, m, 64));
    mx = fmax(mx, __shfl_xor(mx, m, 64));
  }
  if (lane == 0) {
    pm[wave][0] = mn;
    pm[wave][1] = mx;
  }
  for (int j = threadIdx.x; j < nsub * nbins; j += kHistThreads) sub[j] = 0u;
  if constexpr (kDip)
    for (int j = threadIdx.x; j < 2 * nsub * nbins; j += kHistThreads) subd[j] = 0ull;
  __syncthreads();
  mn = pm[0][0];
  mx = pm[0][1];
  for (int w = 1; w < kHistThreads / 64; ++w) {
    mn = fmin(mn, pm[w][0]);
    mx = fmax(mx, pm[w][1]);
  }
  if (!(mn <= mx)) {  // nobody alive
    mn = 0.0;
    mx = 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    range[0] = mn;
    range[1] = mx;
  }
  const double width = mx - mn;
  const double inv = width > 0.0 ? static_cast<double>(nbins) / width : 0.0;
  uint32_t *mine = sub + (wave % nsub) * nbins;
  unsigned long long *mined = subd + 2 * (wave % nsub) * nbins;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kHistThreads;
  // loads in flight per thread
  constexpr int kU = kHistUnroll;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kHistThreads + threadIdx.x; i < n;
       i += kU * stride) {
    double v[kU], vx[kU], vy[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const bool in = i + u * stride < n;
      v[u] = in ? s[i + u * stride] : -1.0;
      if constexpr (kDip) {
        vx[u] = in ? xs[i + u * stride] : 0.0;
        vy[u] = in ? ys[i + u * stride] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const double f = (v[u] - mn) * inv;
      if (i + u * stride < n && f >= 0.0) {
        const int b = min(static_cast<int>(f), nbins - 1);
        atomicAdd(mine + b, 1u);
        if constexpr (kDip) {
          atomicAdd(mined + b, dip_quantum(vx[u]));
          atomicAdd(mined + nbins + b, dip_quantum(vy[u]));
        }
      }
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nbins; b += kHistThreads) {
    uint32_t c = 0;
    for (int w = 0; w < nsub; ++w) c += sub[w * nbins + b];
    if (c != 0u) atomicAdd(counts + b, c);
    if constexpr (kDip) {
      unsigned long long sx = 0ull, sy = 0ull;
      for (int w = 0; w < nsub; ++w) {
        sx += subd[2 * w * nbins + b];
        sy += subd[(2 * w + 1) * nbins + b];
      }
      if (sx != 0ull) atomicAdd(dip + b, sx);
      if (sy != 0ull) atomicAdd(dip + nbins + b, sy);
    }
  }
}

hipError_t launch_histogram(const double *s, const int64_t *n_alive, int64_t n_total,
                            const double *mm_part, int mm_n, int nbins, uint32_t *counts,
                            double *range, hipStream_t st, const double *x, const double *y,
                            int64_t *dip) {
  const int64_t chunk = static_cast<int64_t>(kHistThreads) * kHistItems;
  const int64_t want = (n_total + chunk - 1) / chunk;
  const int grid = static_cast<int>(want < 1 ? 1 : (want > kHistMaxGrid ? kHistMaxGrid : want));
  const bool d = dip != nullptr;
  // bytes of one sub-histogram; sub-histograms share at most 32 KB (48 KB
  // with the dipole words)
  const size_t per = static_cast<size_t>(nbins) * (d ? 20 : 4);
  const size_t budget = d ? 49152 : 32768;
  int nsub = kHistThreads / 64;
  while (nsub > 1 && static_cast<size_t>(nsub) * per > budget) nsub >>= 1;
  if (static_cast<size_t>(nsub) * per > budget) return hipErrorInvalidValue;
  const size_t lds = static_cast<size_t>(nsub) * per + (d ? 8 : 0);
  auto *du = reinterpret_cast<unsigned long long *>(dip);
  if (d)
    TRK_LAUNCH((k_histogram<true>), dim3(grid), dim3(kHistThreads), lds, st, s, x, y,
                       n_alive, n_total, mm_part, mm_n, nbins, nsub, counts, du, range);
  else
    TRK_LAUNCH((k_histogram<false>), dim3(grid), dim3(kHistThreads), lds, st, s, x, y,
                       n_alive, n_total, mm_part, mm_n, nbins, nsub, counts, du, range);
  return hipGetLastError();
}

// ------------------------------------------------------------------ convolution
// Normalised resonator wakes on the bin lags t = m * delta / c:
//   longitudinal W~[0] = 1/2 (a particle sees half of its own wake),
//                W~[m] = exp(-t/tau0) cos(omega t);
//   transverse   Wt[0] = 0,  Wt[m] = exp(-t/tau0) sin(omega t).
template <bool kTr>
__device__ __forceinline__ double wake_table_entry(int m, double dt, double tau0, double omega) {
  if (m == 0) return kTr ? 0.0 : 0.5;
  const double t = static_cast<double>(m) * dt;
  return dm::own_exp(-(t / tau0)) * (kTr ? dm::own_sin(omega * t) : dm::own_cos(omega * t));
}

// Convolution weights: the counts, or (transverse, plane blockIdx.y) the
// dipole sums in metres, 2^-40 times the integer (one rounding).
// counts of bin m summed over the ncopy (<= kHistCopies) copies [ncopy][nbins]
// (an exact integer sum).  Every load is unconditional, from copy k or, past
// ncopy, from copy 0 again (always in bounds) with the value dropped, so
// all of them are in flight together.
__device__ __forceinline__ uint32_t bin_count(const uint32_t *counts, int nbins, int ncopy, int m) {
  uint32_t c = counts[m];
#pragma unroll
  for (int k = 1; k < kHistCopies; ++k) {
    const bool use = k < ncopy;
    const uint32_t x = counts[(use ? k : 0) * nbins + m];
    c += use ? x : 0u;
  }
  return c;
}

template <bool kTr>
__device__ __forceinline__ double conv_weight(const void *src, int nbins, int ncopy, int m) {
  if constexpr (kTr)
    return static_cast<double>(static_cast<const long long *>(src)[blockIdx.y * nbins + m]) * 0x1p-40;
  else
    return static_cast<double>(bin_count(static_cast<const uint32_t *>(src), nbins, ncopy, m));
}

// the first workgroup clears the buffer the following run bins into
__device__ __forceinline__ void clear_next(uint32_t *zbuf, int zn) {
  if (zbuf != nullptr && blockIdx.x == 0 && blockIdx.y == 0)
    for (int i = threadIdx.x; i < zn; i += blockDim.x) zbuf[i] = 0u;
}

constexpr int kTile = 256;  // outputs per convolution workgroup

__device__ __forceinline__ void write_wake_par(double smin, double width, int nbins,
                                               double *wake_par) {
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0 && wake_par != nullptr) {
    wake_par[0] = smin;
    wake_par[1] = width > 0.0 ? static_cast<double>(nbins) / width : 0.0;
  }
}

// Binary64: V[i] = sum_{j<=i} c_j W[i-j], j ascending, one fma chain per
// output -- the plain causal convolution, bit-exact with a sequential CPU
// loop.  Workgroup g owns outputs [256 g, 256 g + 256) (of plane blockIdx.y).
template <bool kTr>
__global__ __launch_bounds__(kTile) void k_conv_fp64(const void *__restrict__ src, int nbins,
                                                     int ncopy, const double *__restrict__ range,
                                                     double tau0, double omega,
                                                     double *__restrict__ v,
                                                     double *__restrict__ wake_par, uint32_t *zbuf,
                                                     int zn) {
  constexpr int kN = kTr ? TRK_MAX_TRBINS : TRK_MAX_BINS;
  __shared__ double W[kN];
  __shared__ std::conditional_t<kTr, double, uint32_t> C[kN];
  const double smin = range[0], smax = range[1];
  const double width = smax - smin;
  const double delta = width > 0.0 ? width / static_cast<double>(nbins) : 0.0;
  const double dt = delta / kCLight;
  const int hi = min(nbins, kTile * static_cast<int>(blockIdx.x + 1));
  for (int m = threadIdx.x; m < hi; m += kTile) {
    W[m] = wake_table_entry<kTr>(m, dt, tau0, omega);
    if constexpr (kTr)
      C[m] = conv_weight<kTr>(src, nbins, 1, m);
    else
      C[m] = bin_count(static_cast<const uint32_t *>(src), nbins, ncopy, m);
  }
  clear_next(zbuf, zn);
  __syncthreads();
  const int i = kTile * blockIdx.x + threadIdx.x;
  if (i < nbins) {
    double acc = 0.0;
    for (int j = 0; j <= i; ++j) acc = fma(static_cast<double>(C[j]), W[i - j], acc);
    v[blockIdx.y * nbins + i] = acc;
  }
  write_wake_par(smin, width, nbins, wake_par);
}

// FP32 on the matrix cores.  With V, c laid out as 16-row matrices
// Vm[b][a] = V[16a+b], the causal convolution is a sum of products of
// lower-Toeplitz 16x16 tiles T_d[b][b'] = W[16d+b-b'] with column-shifted
// weight tiles S_d[b'][a] = c[16(a-d)+b']:  Vm = sum_d T_d S_d, a dense
// contraction that v_mfma_f32_16x16x4_f32 executes.  Workgroup g owns the
// 16 columns (256 outputs) of tile g and needs d < 16g + 16; its 16 waves
// split d and their partial tiles are added in wave order (deterministic).
// W and c are rounded once to binary32 (counts are exact below 2^24).
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kConvWaves = 16;

template <bool kTr>
__global__ __launch_bounds__(64 * kConvWaves) void k_conv_mfma(
    const void *__restrict__ src, int nbins, int ncopy, const double *__restrict__ range,
    double tau0, double omega, double *__restrict__ v, double *__restrict__ wake_par,
    uint32_t *zbuf, int zn) {
  __shared__ float Wf[TRK_MAX_BINS];
  __shared__ float Cf[TRK_MAX_BINS];
  __shared__ float part[kConvWaves][kTile];
  const double smin = range[0], smax = range[1];
  const double width = smax - smin;
  const double delta = width > 0.0 ? width / static_cast<double>(nbins) : 0.0;
  const double dt = delta / kCLight;
  const int g = blockIdx.x;
  const int hi = kTile * (g + 1);  // entries this tile can touch
  for (int m = threadIdx.x; m < hi; m += blockDim.x) {
    Wf[m] = m < nbins ? static_cast<float>(wake_table_entry<kTr>(m, dt, tau0, omega)) : 0.0f;
    Cf[m] = m < nbins ? static_cast<float>(conv_weight<kTr>(src, nbins, ncopy, m)) : 0.0f;
  }
  clear_next(zbuf, zn);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = lane & 15, kq = lane >> 4;
  const int col = 16 * g + r;  // Vm column of this lane's B operand
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int d = wave; d < 16 * g + 16; d += kConvWaves) {
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      const int k = 4 * kb + kq;
      const int m = 16 * d + r - k;
      const float av = m >= 0 ? Wf[m] : 0.0f;
      const float bv = col >= d ? Cf[16 * (col - d) + k] : 0.0f;
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
    }
  }
  // lane holds Vm[4 kq + q][16 g + r] = V[256 g + 16 r + 4 kq + q]
#pragma unroll
  for (int q = 0; q < 4; ++q) part[wave][16 * r + 4 * kq + q] = acc[q];
  __syncthreads();
  if (threadIdx.x < kTile) {
    float sum = part[0][threadIdx.x];
#pragma unroll
    for (int w = 1; w < kConvWaves; ++w) sum += part[w][threadIdx.x];
    const int i = kTile * g + threadIdx.x;
    if (i < nbins) v[blockIdx.y * nbins + i] = static_cast<double>(sum);
  }
  write_wake_par(smin, width, nbins, wake_par);
}

template <bool kTr>
hipError_t launch_conv(const void *src, int nbins, int ncopy, const double *range, double tau0,
                       double omega, int mode, double *v, double *wake_par, uint32_t *zbuf, int zn,
                       hipStream_t st) {
  const dim3 grid((nbins + kTile - 1) / kTile, kTr ? 2 : 1);
  if (mode == TRK_WAKE_FP32_MFMA)
    TRK_LAUNCH((k_conv_mfma<kTr>), grid, dim3(64 * kConvWaves), 0, st, src, nbins, ncopy,
                       range, tau0, omega, v, wake_par, zbuf, zn);
  else
    TRK_LAUNCH((k_conv_fp64<kTr>), grid, dim3(kTile), 0, st, src, nbins, ncopy, range, tau0,
                       omega, v, wake_par, zbuf, zn);
  return hipGetLastError();
}

hipError_t launch_convolve(const uint32_t *counts, int nbins, const double *range, double tau0,
                           double omega, int mode, double *v, double *wake_par, hipStream_t st,
                           int ncopy, uint32_t *zbuf, int zn) {
  if (ncopy < 1 || ncopy > kHistCopies) return hipErrorInvalidValue;
  return launch_conv<false>(counts, nbins, ncopy, range, tau0, omega, mode, v, wake_par, zbuf, zn,
                            st);
}

hipError_t launch_convolve_tr(const int64_t *dip, int nbins, const double *range, double tau0,
                              double omega, int mode, double *v, double *wake_par,
                              hipStream_t st, uint32_t *zbuf, int zn) {
  return launch_conv<true>(dip, nbins, 1, range, tau0, omega, mode, v, wake_par, zbuf, zn, st);
}

// ------------------------------------------------------------------ wake kick
__global__ __launch_bounds__(kBlock) void k_wake_kick(const double *__restrict__ s,
                                                      double *__restrict__ dp,
                                                      const int64_t *__restrict__ n_alive,
                                                      int64_t n_total, const double *__restrict__ v,
                                                      const double *__restrict__ wake_par,
                                                      int nbins, double kfac) {
  const int64_t n = min(*n_alive, n_total);
  const double smin = wake_par[0], inv = wake_par[1];
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    const double vs = el::wake_interp(s[i], smin, inv, v, nbins);
    dp[i] = fma(-kfac, vs, dp[i]);
  }
}

hipError_t launch_wake_kick(double *s, double *dp, const int64_t *n_alive, int64_t n_total,
                            const double *v, const double *wake_par, int nbins, double kfac,
                            hipStream_t st) {
  const int64_t want = nblocks(n_total);
  const int grid = static_cast<int>(want < 1 ? 1 : (want > kMaxRunGrid ? kMaxRunGrid : want));
  hipLaunchKernelGGL(k_wake_kick, dim3(grid), dim3(kBlock), 0, st, s, dp, n_alive, n_total, v,
                     wake_par, nbins, kfac);
  return hipGetLastError();
}

// ------------------------------------------------------------------ transverse wake kick
__global__ __launch_bounds__(kBlock) void k_trwake_kick(double *__restrict__ xp,
                                                        double *__restrict__ yp,
                                                        const double *__restrict__ s,
                                                        const double *__restrict__ dp,
                                                        const int64_t *__restrict__ n_alive,
                                                        int64_t n_total,
                                                        const double *__restrict__ v,
                                                        const double *__restrict__ wake_par,
                                                        int nbins, double kfac) {
  const int64_t n = min(*n_alive, n_total);
  const double smin = wake_par[0], inv = wake_par[1];
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    double z[6] = {0.0, xp[i], 0.0, yp[i], s[i], dp[i]};
    el::trwake(z, kfac, el::wake_interp(z[4], smin, inv, v, nbins),
               el::wake_interp(z[4], smin, inv, v + nbins, nbins));
    xp[i] = z[1];
    yp[i] = z[3];
  }
}

hipError_t launch_trwake_kick(double *const z[6], const int64_t *n_alive, int64_t n_total,
                              const double *v, const double *wake_par, int nbins, double kfac,
                              hipStream_t st) {
  const int64_t want = nblocks(n_total);
  const int grid = static_cast<int>(want < 1 ? 1 : (want > kMaxRunGrid ? kMaxRunGrid : want));
  hipLaunchKernelGGL(k_trwake_kick, dim3(grid), dim3(kBlock), 0, st, z[1], z[3], z[4], z[5],
                     n_alive, n_total, v, wake_par, nbins, kfac);
  return hipGetLastError();
}

// ------------------------------------------------------------------ moments
// Shifted sums over survivors: row = (n, sum d_k, sum d_k d_l (k<=l)),
// d = z - shift.  Each thread accumulates its particles in index order, then
// the block sums in fixed order: deterministic for a given grid.
struct Z6 {
  const double *p[6];
};

__global__ __launch_bounds__(kBlock) void k_mom_partial(Z6 z, const int64_t *__restrict__ n_alive,
                                                        int64_t n_total,
                                                        const double *__restrict__ shift,
                                                        double *__restrict__ part) {
  const int64_t n = min(*n_alive, n_total);
  double c[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) c[k] = shift ? shift[k] : 0.0;
  double acc[28];
#pragma unroll
  for (int k = 0; k < 28; ++k) acc[k] = 0.0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    double d[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) d[k] = z.p[k][i] - c[k];
    acc[0] += 1.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[1 + k] += d[k];
    int o = 7;
#pragma unroll
    for (int k = 0; k < 6; ++k)
#pragma unroll
      for (int l = k; l < 6; ++l) acc[o++] += d[k] * d[l];
  }
  const double *tot = block_sum<28>(acc);
  if (threadIdx.x < 28) part[static_cast<int64_t>(blockIdx.x) * 28 + threadIdx.x] = tot[threadIdx.x];
}

hipError_t launch_mom_partial(double *const z[6], const int64_t *n_alive, int64_t n_total,
                              const double *shift, double *part, int grid, hipStream_t st) {
  Z6 zz;
  for (int k = 0; k < 6; ++k) zz.p[k] = z[k];
  hipLaunchKernelGGL(k_mom_partial, dim3(grid), dim3(kBlock), 0, st, zz, n_alive, n_total, shift,
                     part);
  return hipGetLastError();
}

// One block per pass: sum the rows in fixed order, then
// mean_k = shift_k + S_k/n, cov_kl = S_kl/n - (S_k/n)(S_l/n); with nobody
// alive every output (and the mean handed on as the next shift) is 0.
__global__ __launch_bounds__(kBlock) void k_mom_finalize(const double *__restrict__ part, int nrows,
                                                         const double *__restrict__ shift,
                                                         double *__restrict__ out, int out_stride,
                                                         double *__restrict__ mean_out) {
  const double *pp = part + static_cast<int64_t>(blockIdx.x) * nrows * 28;
  double acc[28];
#pragma unroll
  for (int k = 0; k < 28; ++k) acc[k] = 0.0;
  for (int r = threadIdx.x; r < nrows; r += kBlock) {
#pragma unroll
    for (int k = 0; k < 28; ++k) acc[k] += pp[static_cast<int64_t>(r) * 28 + k];
  }
  const double *tot = block_sum<28>(acc);
  if (threadIdx.x == 0) {
    double *o = out + static_cast<int64_t>(blockIdx.x) * out_stride;
    const double n = tot[0];
    if (n == 0.0) {
      for (int k = 0; k < 28; ++k) o[k] = 0.0;
      if (mean_out)
        for (int k = 0; k < 6; ++k) mean_out[k] = 0.0;
      return;
    }
    double m[6];
    for (int k = 0; k < 6; ++k) m[k] = tot[1 + k] / n;
    o[0] = n;
    for (int k = 0; k < 6; ++k) {
      const double c = shift ? shift[k] : 0.0;
      o[1 + k] = c + m[k];
      if (mean_out) mean_out[k] = c + m[k];
    }
    int idx = 7;
    for (int k = 0; k < 6; ++k)
      for (int l = k; l < 6; ++l, ++idx) o[idx] = tot[idx] / n - m[k] * m[l];
  }
}

hipError_t launch_mom_finalize(const double *part, int nrows, int npass, const double *shift,
                               double *out, int out_stride, double *mean_out, hipStream_t st) {
  hipLaunchKernelGGL(k_mom_finalize, dim3(npass), dim3(kBlock), 0, st, part, nrows, shift, out,
                     out_stride, mean_out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ compensated moments
// The optional compensated reductions of Sec. 2.4: every sum is carried as
// an unevaluated pair (s, c).  A thread adds its particles with Neumaier's
// variant of Kahan summation; pairs are combined with TwoSum (the exact
// rounding error of s1 + s2 goes into c) in the fixed order of the plain
// reductions; the value of a sum is s + c.
__device__ __forceinline__ void neu_add(double &s, double &c, double x) {
  const double t = s + x;
  c += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
  s = t;
}
__device__ __forceinline__ void pair_add(double &s, double &c, double s2, double c2) {
  const double t = s + s2;
  const double bp = t - s;
  const double e = (s - (t - bp)) + (s2 - bp);
  s = t;
  c = (c + c2) + e;
}

// pairs of one block summed: wave butterfly, then the waves in order;
// row[0..28) = s, row[28..56) = c
__device__ __forceinline__ void block_pair_row(double (&s)[28], double (&c)[28], double *row) {
  __shared__ double ps[kWaves][28], pc[kWaves][28];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 28; ++k) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
      const double s2 = __shfl_xor(s[k], m, 64), c2 = __shfl_xor(c[k], m, 64);
      pair_add(s[k], c[k], s2, c2);
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 28; ++k) {
      ps[wave][k] = s[k];
      pc[wave][k] = c[k];
    }
  }
  __syncthreads();
  if (threadIdx.x < 28) {
    double a = ps[0][threadIdx.x], b = pc[0][threadIdx.x];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) pair_add(a, b, ps[w][threadIdx.x], pc[w][threadIdx.x]);
    row[threadIdx.x] = a;
    row[28 + threadIdx.x] = b;
  }
}

__global__ __launch_bounds__(kBlock) void k_mom_partial_c(Z6 z, const int64_t *__restrict__ n_alive,
                                                          int64_t n_total,
                                                          const double *__restrict__ shift,
                                                          double *__restrict__ part) {
  const int64_t n = min(*n_alive, n_total);
  double cs[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) cs[k] = shift ? shift[k] : 0.0;
  double s[28], c[28];
#pragma unroll
  for (int k = 0; k < 28; ++k) s[k] = c[k] = 0.0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    double d[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) d[k] = z.p[k][i] - cs[k];
    s[0] += 1.0;  // counts stay exact integers
#pragma unroll
    for (int k = 0; k < 6; ++k) neu_add(s[1 + k], c[1 + k], d[k]);
    int o = 7;
#pragma unroll
    for (int k = 0; k < 6; ++k)
#pragma unroll
      for (int l = k; l < 6; ++l, ++o) neu_add(s[o], c[o], d[k] * d[l]);
  }
  block_pair_row(s, c, part + static_cast<int64_t>(blockIdx.x) * 56);
}

// sum of the nrows rows of pairs in a fixed order; then as k_mom_finalize
__global__ __launch_bounds__(kBlock) void k_mom_finalize_c(const double *__restrict__ part, int nrows,
                                                           const double *__restrict__ shift,
                                                           double *__restrict__ out,
                                                           double *__restrict__ mean_out) {
  double s[28], c[28];
#pragma unroll
  for (int k = 0; k < 28; ++k) s[k] = c[k] = 0.0;
  for (int r = threadIdx.x; r < nrows; r += kBlock) {
#pragma unroll
    for (int k = 0; k < 28; ++k)
      pair_add(s[k], c[k], part[static_cast<int64_t>(r) * 56 + k],
               part[static_cast<int64_t>(r) * 56 + 28 + k]);
  }
  __shared__ double tot[56];
  block_pair_row(s, c, tot);
  __syncthreads();
  if (threadIdx.x == 0) {
    double v[28];
    for (int k = 0; k < 28; ++k) v[k] = tot[k] + tot[28 + k];
    const double n = v[0];
    if (n == 0.0) {
      for (int k = 0; k < 28; ++k) out[k] = 0.0;
      if (mean_out)
        for (int k = 0; k < 6; ++k) mean_out[k] = 0.0;
      return;
    }
    double m[6];
    for (int k = 0; k < 6; ++k) m[k] = v[1 + k] / n;
    out[0] = n;
    // the compensated first pass already gives the means to about an ulp;
    // the second pass (sums of z - mean) only centres the second moments
    for (int k = 0; k < 6; ++k) {
      out[1 + k] = shift ? shift[k] : m[k];
      if (mean_out) mean_out[k] = m[k];
    }
    int idx = 7;
    for (int k = 0; k < 6; ++k)
      for (int l = k; l < 6; ++l, ++idx) out[idx] = v[idx] / n - m[k] * m[l];
  }
}

hipError_t launch_mom_partial_c(double *const z[6], const int64_t *n_alive, int64_t n_total,
                                const double *shift, double *part, int grid, hipStream_t st) {
  Z6 zz;
  for (int k = 0; k < 6; ++k) zz.p[k] = z[k];
  hipLaunchKernelGGL(k_mom_partial_c, dim3(grid), dim3(kBlock), 0, st, zz, n_alive, n_total, shift,
                     part);
  return hipGetLastError();
}

hipError_t launch_mom_finalize_c(const double *part, int nrows, const double *shift, double *out,
                                 double *mean_out, hipStream_t st) {
  hipLaunchKernelGGL(k_mom_finalize_c, dim3(1), dim3(kBlock), 0, st, part, nrows, shift, out,
                     mean_out);
  return hipGetLastError();
}

__global__ void k_zero_u32(uint32_t *p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}
hipError_t launch_zero_u32(uint32_t *p, int n, hipStream_t st) {
  const int g = n <= kBlock ? 1 : (n / kBlock > 1024 ? 1024 : (n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_zero_u32, dim3(g), dim3(kBlock), 0, st, p, n);
  return hipGetLastError();
}

}  // namespace trk
